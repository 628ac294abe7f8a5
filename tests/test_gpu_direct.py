"""The all-atom comparison mode (direct molecule-substrate sums over the cell and its 8
lateral neighbours, Section "Configuration sampling on GPU") against the FP64 oracle.

Tolerances.  The kernel sums 9 x 48 substrate terms per atom in FP32; the bare Coulomb terms
are individually up to ~1 eV with alternating signs, so the FP32 sum carries ~1e-5 eV of
rounding per atom and forces ~1e-5 eV/A: energies are compared at 1e-4 eV per atom and forces
at 1e-4 eV/A (relative to the force scale above 1 eV/A).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2508_15522_amd import configs, device as D, gridff as G, synth as S
from tests.gpu_common import announce, mixing_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def world():
    D.require_gpu()
    sub = configs.GRID_SMALL.substrate()
    mols = [S.mol_chain24(), S.mol_pah38(), S.mol_size(52, 6)]
    return sub, mols, G.Topology(mols), G.Direct(sub, S.ALPHA, 1)


def _batch(sub, mols, rep_type, seed):
    pos = []
    for k, t in enumerate(rep_type):
        pos.append(S.f32(S.place_replicas(mols[t], 1, sub, seed + k, h_range=(2.5, 4.5))[0]))
    return pos


def test_direct_eval_matches_oracle(world):
    sub, mols, topo, direct = world
    announce("all-atom eval")
    rng = np.random.default_rng(4)
    rep_type = rng.integers(0, len(mols), 37)
    plan = G.Plan(topo, rep_type, block_threads=192)
    pos = _batch(sub, mols, rep_type, 300)
    dpos = D.soa(plan, pos)
    F = torch.empty_like(dpos)
    Ea = torch.empty(plan.n_atoms, device="cuda")
    Er = torch.empty(plan.n_rep, dtype=torch.float64, device="cuda")
    st = torch.empty(plan.n_rep, dtype=torch.int32, device="cuda")
    # substrate part alone
    G.eval_forces_direct(direct, topo, plan, False, dpos, F, Ea, Er, st)
    torch.cuda.synchronize()
    P = np.concatenate(pos)
    plq = mixing_for(mols, rep_type)
    Eo, Fo = O.direct_images(sub, P, plq, nimg=1)
    Fg = F.cpu().numpy().T.astype(np.float64)
    dF = np.linalg.norm(Fg - Fo, axis=1)
    dE = np.abs(Ea.cpu().numpy() - Eo)
    announce(f"  substrate part: max |dF| = {dF.max():.3e} (max |F| {np.abs(Fo).max():.2f}), max |dE| = {dE.max():.3e}")
    assert dF.max() < 1e-4 * max(1.0, np.abs(Fo).max())
    assert dE.max() < 1e-4
    assert (st.cpu().numpy() == 0).all()
    # with the intramolecular field: the oracle's field on a zero grid supplies that part
    G.eval_forces_direct(direct, topo, plan, True, dpos, F, Ea, Er, st)
    torch.cuda.synchronize()
    B0 = np.zeros((3, 8, 8, 8))
    geo = dict(nx=8, ny=8, nz=8, x0=0.0, y0=0.0, z0=-50.0, dx=1.0, dy=1.0, dz=1.0)
    Fi, Eri, _, _ = O.eval_batch(B0, geo, mols, rep_type, P)
    Fg = F.cpu().numpy().T.astype(np.float64)
    dF = np.linalg.norm(Fg - (Fo + Fi), axis=1)
    off = plan.atom_off
    Ero = np.add.reduceat(Eo, off[:-1]) + Eri
    announce(f"  with intramolecular: max |dF| = {dF.max():.3e}, max |dE_rep| = "
             f"{np.abs(Er.cpu().numpy() - Ero).max():.3e}")
    assert dF.max() < 1e-4 * max(1.0, np.abs(Fo + Fi).max())
    nat = np.array([mols[t].n for t in rep_type])
    assert (np.abs(Er.cpu().numpy() - Ero) < 1e-4 * nat).all()


def test_direct_nve_conserves_energy_and_matches_eval(world):
    sub, mols, topo, direct = world
    announce("all-atom NVE")
    rep_type = np.full(64, 1)
    plan = G.Plan(topo, rep_type, block_threads=192)
    pos = _batch(sub, mols, rep_type, 900)
    vel = list(S.mb_velocities(mols[1].mass, len(rep_type), 300.0, S.SEED_NVE))
    st = D.fire_state(plan, pos, vel_per_rep=vel)
    out = D.outputs(plan)
    G.relax_batch_direct(direct, topo, plan, G.relax_params(G.MODE_NVE, 400, True, dt=0.5, drift_every=1), st,
                         out["E"], out["fnorm"], out["steps"], out["drift"])
    torch.cuda.synchronize()
    dr = out["drift"].cpu().numpy()
    announce(f"  max |E(t) - E(0)| over 400 steps: {dr[:, 2].max():.3e} eV")
    assert (out["steps"].cpu().numpy() == 400).all()
    assert (dr[:, 5] == 401).all()
    # velocity Verlet at 0.5 fs: the total energy fluctuates by O(dt^2) without drifting; the
    # bound is under 1% of the 300 K kinetic energy (38 x 3/2 kT = 1.5 eV)
    assert dr[:, 2].max() < 1e-2
    # the energy the integrator reports is the evaluation's energy at the final positions
    Er = torch.empty(plan.n_rep, dtype=torch.float64, device="cuda")
    F = torch.empty_like(st["pos"])
    G.eval_forces_direct(direct, topo, plan, True, st["pos"], F, None, Er, None)
    torch.cuda.synchronize()
    vel_g = D.unsoa(plan, st["vel"])
    ke = np.array([0.5 * np.sum(mols[1].mass[:, None] * 103.6426965 * v.astype(np.float64) ** 2) for v in vel_g])
    assert np.abs(Er.cpu().numpy() + ke - dr[:, 1]).max() < 1e-3


def test_direct_rejects_mismatched_alpha(world):
    sub, mols, topo, _ = world
    d2 = G.Direct(sub, 1.5, 1)
    plan = G.Plan(topo, np.array([0]))
    pos = torch.zeros(3, plan.n_atoms, device="cuda")
    F = torch.empty_like(pos)
    with pytest.raises(G.GffError):
        G.eval_forces_direct(d2, topo, plan, False, pos, F)


def test_direct_langevin_without_friction_is_velocity_verlet(world):
    """The all-atom mode's Langevin integrator at zero friction reduces to its velocity
    Verlet (the O step is the identity), up to the rounding of two half drifts."""
    sub, mols, topo, direct = world
    announce("all-atom Langevin at zero friction")
    rep_type = np.full(24, 1)
    plan = G.Plan(topo, rep_type, block_threads=192)
    pos = _batch(sub, mols, rep_type, 1300)
    vel = list(S.mb_velocities(mols[1].mass, len(rep_type), 300.0, S.SEED_NVE + 3))
    res = []
    for mode, kw in ((G.MODE_NVE, {}), (G.MODE_LANGEVIN, dict(gamma=0.0, seed=5))):
        st = D.fire_state(plan, pos, vel_per_rep=vel)
        out = D.outputs(plan)
        G.relax_batch_direct(direct, topo, plan, G.relax_params(mode, 60, True, dt=0.5, **kw), st, out["E"],
                             out["fnorm"], out["steps"])
        torch.cuda.synchronize()
        res.append((st["pos"].cpu().numpy(), out["E"].cpu().numpy()))
    dx = np.abs(res[0][0] - res[1][0]).max()
    announce(f"  max |dx| NVE vs Langevin(gamma=0) = {dx:.2e} A")
    assert dx < 1e-4
    assert np.abs(res[0][1] - res[1][1]).max() < 1e-3
