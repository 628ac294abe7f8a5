"""GPU parity of the setup path: FP64 grid build (a9), exact fit (a10) and the physical
model against the direct sums.

build: the GPU's Fourier-form Coulomb lattice sum and image-summed Morse channels at
sampled nodes against the oracle's 2D Ewald and direct image sums, relative 1e-11.
fit: GPU coefficients against the oracle's on the same V (relative 1e-12), and the
defining node equations on the GPU's own output (residual <= 1e-12 max|V|).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2508_15522_amd import configs, device as D, gridff as G, synth as S
from tests.gpu_common import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    D.require_gpu()


def _build(sub, spec):
    n = spec.nx * spec.ny * spec.nz
    V = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    work = torch.empty(G.build_grid_workspace_bytes(spec, sub), dtype=torch.uint8, device="cuda")
    G.build_grid(sub, spec, V, work)
    torch.cuda.synchronize()
    return V.cpu().numpy().reshape(3, spec.nx, spec.ny, spec.nz)


def _sample_nodes(spec, m, seed):
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.integers(0, spec.nx, m), rng.integers(0, spec.ny, m), rng.integers(0, spec.nz, m)], 1)
    idx[:8, 2] = [0, 0, 1, 2, spec.nz - 1, spec.nz - 1, spec.nz // 2, 3]       # first/last planes
    idx[:4, 0] = [0, spec.nx - 1, 0, spec.nx - 1]
    return idx


def _geo(spec, sub):
    return dict(nx=spec.nx, ny=spec.ny, nz=spec.nz, x0=spec.x0, y0=spec.y0, z0=spec.z0,
                dx=sub.Lx / spec.nx, dy=sub.Ly / spec.ny, dz=spec.dz)


@pytest.mark.parametrize("rcut", [17.0, 30.0])
def test_build_grid_small_substrate_sampled_nodes(rcut):
    cfg = configs.GRID_SMALL
    announce(f"build small grid rcut={rcut}")
    sub = cfg.substrate()
    spec = G.grid_spec(cfg.nx, cfg.ny, cfg.nz, 0.0, 0.0, cfg.z0, cfg.dz, cfg.alpha, rcut)
    V = _build(sub, spec)
    idx = _sample_nodes(spec, 600, 1)
    Vo = O.grid_values(sub, _geo(spec, sub), idx, rcut=rcut)
    Vg = V[:, idx[:, 0], idx[:, 1], idx[:, 2]]
    for c in range(3):
        err = np.abs(Vg[c] - Vo[c]).max() / np.abs(Vo[c]).max()
        announce(f"  channel {c}: max rel err {err:.2e}")
        assert err < 1e-11
    assert np.isfinite(V).all()


def test_build_grid_large_substrate_sampled_nodes():
    """8x8 cells, 12 planes (3072 atoms), 452 x 452 x 200 nodes: the large configuration."""
    cfg = configs.GRID_LARGE
    announce("build large grid")
    sub = cfg.substrate()
    spec = D.spec_for(cfg)
    V = _build(sub, spec)
    idx = _sample_nodes(spec, 40, 2)
    # eta only sets the oracle's cost (its result is eta independent); 0.2 keeps it short
    VP, VL, _, _ = O.morse_direct(sub, O.node_coords(_geo(spec, sub), idx), rcut=cfg.rcut)
    VC, _ = O.coulomb_ewald2d(sub, O.node_coords(_geo(spec, sub), idx), eta=0.2)
    Vg = V[:, idx[:, 0], idx[:, 1], idx[:, 2]]
    for c, Vo in enumerate((VP, VL, VC)):
        err = np.abs(Vg[c] - Vo).max() / np.abs(Vo).max()
        announce(f"  channel {c}: max rel err {err:.2e}")
        assert err < 1e-11


def _node_operator(B):
    out = (np.roll(B, 1, -3) + 4 * B + np.roll(B, -1, -3)) / 6
    out = (np.roll(out, 1, -2) + 4 * out + np.roll(out, -1, -2)) / 6
    lo = np.concatenate([out[..., 1:2], out[..., :-1]], -1)
    hi = np.concatenate([out[..., 1:], out[..., -2:-1]], -1)
    return (lo + 4 * out + hi) / 6


@pytest.mark.parametrize("shape", [(112, 112, 150), (13, 7, 5)])
def test_fit_bspline_matches_oracle(shape):
    nx, ny, nz = shape
    announce(f"fit {shape}")
    rng = np.random.default_rng(4)
    V = rng.normal(size=(3, nx, ny, nz)) * np.array([3.0, 0.5, 0.1])[:, None, None, None]
    spec = G.grid_spec(nx, ny, nz, 0.0, 0.0, 1.0, 0.1)
    dV = torch.from_numpy(V).cuda()
    dB = torch.empty_like(dV)
    work = torch.empty(G.fit_workspace_bytes(spec), dtype=torch.uint8, device="cuda")
    G.fit_bspline(spec, dV, dB, work)
    torch.cuda.synchronize()
    Bg = dB.cpu().numpy()
    Bo = O.fit_bspline(V)
    assert np.abs(Bg - Bo).max() <= 1e-12 * np.abs(Bo).max()
    assert np.abs(_node_operator(Bg) - V).max() <= 1e-12 * np.abs(V).max()


def test_physical_model_vs_direct_and_f16_accuracy():
    """GPU build -> fit -> pack -> interpolate on the small substrate's 0.1 A grid, at sampled
    atom positions 2.5-6 A above the top plane (C/O/H mixing coefficients).
    (i) The model against the exact channels: the cubic B-spline interpolation error, bounded
        per axis by (1/24) h^3 |d^4 V| for the force and (5/384) h^4 |d^4 V| for the energy;
        with |d^4 V_P| <= (2 alpha)^4 V_P dominating near the surface this is ~4e-3 eV/A and
        ~1e-4 eV at 2.5 A.  Reported, and checked against those bounds.
    (ii) FP16 storage against FP32 storage on the same grid and points: <= 1e-3 eV/A at
        every point."""
    cfg = configs.GRID_SMALL
    announce("physical model vs direct")
    sub = cfg.substrate()
    spec = D.spec_for(cfg)
    pts = S.random_points(3000, sub.Lx, sub.Ly, 2.5, 6.0, 21, lateral_span=2.0)
    rng = np.random.default_rng(3)
    el = rng.choice(["C", "O", "H"], len(pts))
    plq = S.f32(O.mixing(np.array([S.MORSE_EPS[e] for e in el]), np.array([S.MORSE_R[e] for e in el]),
                         rng.normal(0, 0.3, len(pts))))
    V, g = O.channels_direct(sub, pts, rcut=cfg.rcut)
    E_ref = (plq * V.T).sum(1)
    F_ref = -np.einsum("pc,cpk->pk", plq, g)
    dpos = torch.from_numpy(np.ascontiguousarray(pts.T, np.float32)).cuda()
    dplq = torch.from_numpy(np.ascontiguousarray(plq.T, np.float32)).cuda()
    out = {}
    for storage in (G.STORE_F32, G.STORE_F16):
        grid = D.build_physical_grid(sub, spec, storage)
        F = torch.empty_like(dpos)
        E = torch.empty(len(pts), device="cuda")
        G.interp_points(grid.desc, dpos, dplq, F, E)
        torch.cuda.synchronize()
        out[storage] = (E.cpu().numpy().astype(np.float64), F.cpu().numpy().T.astype(np.float64))
    E32, F32 = out[G.STORE_F32]
    E16, F16 = out[G.STORE_F16]
    dF = np.linalg.norm(F32 - F_ref, axis=1)
    dE = np.abs(E32 - E_ref)
    h = cfg.dz
    d4 = (2 * cfg.alpha) ** 4 * np.abs(plq[:, 0] * V[0]) + cfg.alpha ** 4 * np.abs(plq[:, 1] * V[1])
    announce(f"  model vs direct (FP32): max |dF| {dF.max():.2e} eV/A, max |dE| {dE.max():.2e} eV; "
             f"max |F| {np.abs(F_ref).max():.2f}")
    assert (dF <= np.sqrt(3) * h ** 3 / 24 * d4 * 2 + 1e-4).all()
    assert (dE <= 3 * 5 / 384 * h ** 4 * d4 * 2 + 2e-5).all()
    d16 = np.linalg.norm(F16 - F32, axis=1)
    announce(f"  FP16 vs FP32 storage: max |dF| {d16.max():.2e} eV/A (z < 2.8 A: {d16[pts[:, 2] < 2.8].max():.2e}), "
             f"max |dE| {np.abs(E16 - E32).max():.2e} eV")
    # with one half per channel the FP16 relative step 2^-11 times the steep Pauli term gave
    # 1.4e-3 eV/A at 2.5-2.8 A; the Pauli residual half brings it under the bound everywhere
    assert d16.max() < 1e-3


def test_build_grid_defect_supercell_sampled_nodes():
    """The large-memory regime: a 20x20x3 supercell (112.8 A square) with a neutral
    cation-anion vacancy pair at its centre, 1128 x 1128 x 80 nodes (1.0e8 nodes, 2.4 GB per
    FP64 array).  Nodes sampled around the defect and far from it against the oracle's
    direct Morse image sums and 2D Ewald sum; the defect is visible in every channel."""
    cfg = configs.GRID_DEFECT
    announce("build defect supercell grid")
    sub = cfg.substrate()
    spec = D.spec_for(cfg)
    n = spec.nx * spec.ny * spec.nz
    V = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    work = torch.empty(G.build_grid_workspace_bytes(spec, sub), dtype=torch.uint8, device="cuda")
    G.build_grid(sub, spec, V, work)
    torch.cuda.synchronize()
    del work
    geo = _geo(spec, sub)
    rng = np.random.default_rng(5)
    c = sub.Lx / 2                                        # the vacancy pair sits at (c, c) and (c + a/2, c)
    near = np.stack([rng.integers(int((c - 4) / geo["dx"]), int((c + 7) / geo["dx"]), 16),
                     rng.integers(int((c - 4) / geo["dy"]), int((c + 4) / geo["dy"]), 16),
                     rng.integers(0, 30, 16)], 1)
    a2 = S.SLAB_A / 2
    near[0] = [int(round(c / geo["dx"])), int(round(c / geo["dy"])), 0]            # 1 A above the vacancies
    near[1] = [int(round((c + a2) / geo["dx"])), int(round(c / geo["dy"])), 0]
    far = _sample_nodes(spec, 8, 6)
    idx = np.concatenate([near, far])
    flat = torch.from_numpy((idx[:, 0] * spec.ny + idx[:, 1]) * spec.nz + idx[:, 2]).cuda()
    Vg = torch.stack([V[k * n + flat] for k in range(3)]).cpu().numpy()
    pts = O.node_coords(geo, idx)
    VP, VL, _, _ = O.morse_direct(sub, pts, rcut=cfg.rcut)
    # eta only sets the oracle's cost (its result is eta independent); on this wide cell a
    # small eta keeps the reciprocal sum short
    VC, _ = O.coulomb_ewald2d(sub, pts, eta=0.06)
    for ch, Vo in enumerate((VP, VL, VC)):
        err = np.abs(Vg[ch] - Vo).max() / np.abs(Vo).max()
        announce(f"  channel {ch}: max rel err {err:.2e}")
        assert err < 1e-11
    # directly above a vacancy the missing atom's Pauli term is gone: against the pristine slab
    # the channel drops by most of its value there
    VPp, _, _, _ = O.morse_direct(configs.GRID_DEFECT_PRISTINE.substrate(), pts[:2], rcut=cfg.rcut)
    announce(f"  Pauli channel above the vacancies: {VP[:2]} (pristine {VPp})")
    assert (VP[:2] < 0.5 * VPp).all()
