"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties an oracle function to something other than itself: a closed form,
an invariant, a published known-answer vector, an independent formula or a
finite-difference derivative.  No GPU.
"""
import numpy as np
import pytest

import oracle as O
from paper_2508_15522_amd import synth as S

RNG = np.random.default_rng(12345)


# ------------------------------------------------------------------ P1: basis (Eq. Bspline)
def test_p1_basis_node_values_and_partition_of_unity():
    # at a node (t = 0) the four weights are 1/6, 2/3, 1/6, 0 -> f = (b_{k-1} + 4 b_k + b_{k+1})/6
    assert O.bspline_B(1.0) == pytest.approx(1 / 6, abs=1e-15)
    assert O.bspline_B(0.0) == pytest.approx(2 / 3, abs=1e-15)
    assert O.bspline_B(-1.0) == pytest.approx(1 / 6, abs=1e-15)
    assert O.bspline_B(2.0) == 0.0 and O.bspline_B(-2.0) == 0.0
    for t in RNG.random(200):
        s = sum(O.bspline_B(t - j) for j in range(-1, 3))
        ds = sum(O.bspline_dB(t - j) for j in range(-1, 3))
        assert abs(s - 1) < 1e-15 and abs(ds) < 1e-15
    # derivative is the FD slope of B
    for t in np.linspace(-2.2, 2.2, 41):
        h = 1e-6
        fd = (O.bspline_B(t + h) - O.bspline_B(t - h)) / (2 * h)
        assert abs(fd - O.bspline_dB(t)) < 1e-8


# ------------------------------------------------------------------ P2: cubic exactness
def _poly_grid(nx, ny, nz, d):
    """Coefficients b = prod_axes (1 - d^2/6 d^2/dx^2) p for p = px(x) py(y) pz(z) + q(x,y,z)."""
    cx = RNG.normal(size=4); cy = RNG.normal(size=4); cz = RNG.normal(size=4)
    x = np.arange(nx) * d[0]; y = np.arange(ny) * d[1]; z = np.arange(nz) * d[2]

    def p_and_op(c, t, h):
        p = c[0] + c[1] * t + c[2] * t ** 2 + c[3] * t ** 3
        p2 = 2 * c[2] + 6 * c[3] * t
        return p, p - h * h / 6 * p2
    px, bx = p_and_op(cx, x, d[0]); py, by = p_and_op(cy, y, d[1]); pz, bz = p_and_op(cz, z, d[2])
    B = np.einsum("i,j,k->ijk", bx, by, bz)

    def P(r):
        vx = np.polyval(cx[::-1], r[:, 0]); vy = np.polyval(cy[::-1], r[:, 1]); vz = np.polyval(cz[::-1], r[:, 2])
        gx = np.polyval(np.polyder(cx[::-1]), r[:, 0]); gy = np.polyval(np.polyder(cy[::-1]), r[:, 1])
        gz = np.polyval(np.polyder(cz[::-1]), r[:, 2])
        return vx * vy * vz, np.stack([gx * vy * vz, vx * gy * vz, vx * vy * gz], 1)
    return B, P


def test_p2_cubic_polynomial_exactness():
    nx, ny, nz = 12, 10, 9
    d = (0.3, 0.25, 0.2)
    Bp, P = _poly_grid(nx, ny, nz, d)
    B = np.zeros((3, nx, ny, nz)); B[0] = Bp
    spec = dict(nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=0.0, dx=d[0], dy=d[1], dz=d[2])
    n = 400
    # interior cells: stencil i-1..i+2 inside [0, n-1] on every axis (no wrap, no mirror)
    r = np.stack([RNG.uniform(1, nx - 3, n) * d[0], RNG.uniform(1, ny - 3, n) * d[1],
                  RNG.uniform(1, nz - 3, n) * d[2]], 1)
    plq = np.tile([1.0, 0.0, 0.0], (n, 1))
    E, F, fl = O.bspline_eval(B, spec, r, plq)
    pv, pg = P(r)
    assert np.abs(E - pv).max() < 1e-12 * max(1, np.abs(pv).max())
    assert np.abs(-F - pg).max() < 1e-11 * max(1, np.abs(pg).max())
    assert (fl == 0).all()
    # channel routing: the same grid in channel 2 with Q = 1
    B2 = np.zeros_like(B); B2[2] = Bp
    E2, F2, _ = O.bspline_eval(B2, spec, r, np.tile([0.0, 0.0, 1.0], (n, 1)))
    assert np.array_equal(E2, E) and np.array_equal(F2, F)


# ------------------------------------------------------------------ P3 / P4: fit
def test_p3_periodic_cosine_fit_closed_form():
    nx, ny, nz = 16, 5, 6
    for m in (1, 3, 7):
        V = np.cos(2 * np.pi * m * np.arange(nx) / nx)[:, None, None] * np.ones((nx, ny, nz))
        Bc = O.fit_bspline(V)
        expect = V * 3 / (2 + np.cos(2 * np.pi * m / nx))
        assert np.abs(Bc - expect).max() < 1e-14
    # same along y
    V = np.cos(2 * np.pi * 2 * np.arange(ny) / ny)[None, :, None] * np.ones((nx, ny, nz))
    assert np.abs(O.fit_bspline(V) - V * 3 / (2 + np.cos(2 * np.pi * 2 / ny))).max() < 1e-14


def _apply_node_operator(B):
    """(b_{i-1} + 4 b_i + b_{i+1})/6 along x, y periodic and z even-mirror."""
    out = (np.roll(B, 1, -3) + 4 * B + np.roll(B, -1, -3)) / 6
    out = (np.roll(out, 1, -2) + 4 * out + np.roll(out, -1, -2)) / 6
    lo = np.concatenate([out[..., 1:2], out[..., :-1]], -1)
    hi = np.concatenate([out[..., 1:], out[..., -2:-1]], -1)
    return (lo + 4 * out + hi) / 6


def test_p4_fit_node_residual_random_and_model_reproduces_nodes():
    V = RNG.normal(size=(3, 9, 11, 13))
    B = O.fit_bspline(V)
    assert np.abs(_apply_node_operator(B) - V).max() <= 1e-12 * np.abs(V).max()
    # the model evaluated at nodes equals V (the last z plane is left out: a rounding
    # error in its coordinate can put it just above the grid, where the model is zero)
    spec = dict(nx=9, ny=11, nz=13, x0=0.3, y0=-0.2, z0=1.0, dx=0.1, dy=0.12, dz=0.1)
    I, J, K = np.meshgrid(np.arange(9), np.arange(11), np.arange(12), indexing="ij")
    idx = np.stack([I.ravel(), J.ravel(), K.ravel()], 1)
    r = O.node_coords(spec, idx)
    for c in range(3):
        plq = np.zeros((len(r), 3)); plq[:, c] = 1
        E, _, fl = O.bspline_eval(B, spec, r, plq)
        assert np.abs(E - V[c, :, :, :12].ravel()).max() < 1e-12
        assert (fl == 0).all()


def test_eval_domain_rules():
    V = RNG.normal(size=(3, 8, 8, 10))
    B = O.fit_bspline(V)
    spec = dict(nx=8, ny=8, nz=10, x0=0.0, y0=0.0, z0=1.0, dx=0.2, dy=0.2, dz=0.1)
    plq = np.array([[0.3, -0.7, 0.2]] * 4)
    r = np.array([[0.33, 0.41, 0.5], [0.33, 0.41, 1.0], [0.33, 0.41, 1.9 + 1e-9], [0.33, 0.41, np.nan]])
    E, F, fl = O.bspline_eval(B, spec, r, plq)
    assert fl[0] == 2 and fl[1] == 0 and fl[2] == 0 and fl[3] == 4
    assert E[0] == E[1] and np.array_equal(F[0], F[1])        # below z0: evaluated at z0
    assert E[2] == 0 and (F[2] == 0).all()                      # above the last node: zero
    assert np.isnan(E[3])
    # periodic wrap in x and y: shifting by a whole period gives the same value
    r = np.array([[0.33, 0.41, 1.37]])
    e0 = O.bspline_eval(B, spec, r, plq[:1])[0]
    e1 = O.bspline_eval(B, spec, r + [8 * 0.2, -2 * 8 * 0.2, 0], plq[:1])[0]
    assert abs(e0 - e1) < 1e-13


# ------------------------------------------------------------------ P5: forces = -grad E
def test_p5_model_force_is_gradient_fd():
    V = RNG.normal(size=(3, 10, 9, 12))
    B = O.fit_bspline(V)
    spec = dict(nx=10, ny=9, nz=12, x0=0.0, y0=0.0, z0=1.0, dx=0.15, dy=0.17, dz=0.1)
    n = 50
    r = np.stack([RNG.uniform(-2, 3, n), RNG.uniform(-2, 3, n), RNG.uniform(1.1, 1.9, n)], 1)
    plq = RNG.normal(size=(n, 3))
    E, F, _ = O.bspline_eval(B, spec, r, plq)
    h = 2e-6
    for c in range(3):
        dr = np.zeros(3); dr[c] = h
        ep = O.bspline_eval(B, spec, r + dr, plq)[0]
        em = O.bspline_eval(B, spec, r - dr, plq)[0]
        assert np.abs((ep - em) / (2 * h) + F[:, c]).max() < 1e-8 * np.abs(F).max()


# ------------------------------------------------------------------ substrate channels
def test_morse_single_atom_closed_form_and_gradient():
    sub = S.rocksalt_slab(1, 1)
    sub.pos = np.array([[1.0, 2.0, 0.0]]); sub.q = np.array([0.0]); sub.eps = np.array([0.15])
    sub.R = np.array([2.0]); sub.Lx = sub.Ly = 100.0
    pts = np.array([[1.3, 2.4, 2.5], [4.0, 0.0, 3.0], [1.0, 2.0, 1.2]])
    VP, VL, gP, gL = O.morse_direct(sub, pts, alpha=1.6, rcut=30.0)
    r = np.linalg.norm(pts - sub.pos[0], axis=1)
    assert np.allclose(VP, 0.15 * np.exp(-3.2 * (r - 2.0)), rtol=1e-14)
    assert np.allclose(VL, 0.15 * np.exp(-1.6 * (r - 2.0)), rtol=1e-14)
    h = 1e-6
    for c in range(3):
        d = np.zeros(3); d[c] = h
        fd = (O.morse_direct(sub, pts + d)[0] - O.morse_direct(sub, pts - d)[0]) / (2 * h)
        assert np.allclose(fd, gP[:, c], rtol=1e-7, atol=1e-12)


def test_p6_substrate_symmetries():
    sub = S.rocksalt_slab(2, 3)
    a = sub.a
    p = S.random_points(30, sub.Lx, sub.Ly, 1.5, 5.0, 7)
    V, g = O.channels_direct(sub, p)
    for shift in ([sub.Lx, 0, 0], [0, sub.Ly, 0], [a / 2, a / 2, 0], [-a / 2, a / 2, 0]):
        V2, _ = O.channels_direct(sub, p + shift)
        assert np.abs(V2 - V).max() < 1e-11 * np.abs(V).max()
    # mirror x -> -x and 90 degree rotation about the ion column at the origin
    V3, _ = O.channels_direct(sub, p * [-1, 1, 1])
    assert np.abs(V3 - V).max() < 1e-11 * np.abs(V).max()
    V4, _ = O.channels_direct(sub, np.stack([-p[:, 1], p[:, 0], p[:, 2]], 1))
    assert np.abs(V4 - V).max() < 1e-11 * np.abs(V).max()
    # swapping cation and anion charges negates V^C and leaves the Morse channels unchanged
    sub2 = S.rocksalt_slab(2, 3); sub2.q = -sub2.q
    V5, _ = O.channels_direct(sub2, p)
    assert np.abs(V5[2] + V[2]).max() < 1e-12 and np.abs(V5[:2] - V[:2]).max() == 0


def test_p7_coulomb_ewald_eta_independence_fourier_and_decay():
    sub = S.rocksalt_slab(2, 3)
    p = S.random_points(25, sub.Lx, sub.Ly, 1.0, 8.0, 3)
    Vs = [O.coulomb_ewald2d(sub, p, eta) for eta in (0.2, 0.35, 0.5)]
    scale = np.abs(Vs[1][0]).max()
    for V, g in Vs[::2]:
        assert np.abs(V - Vs[1][0]).max() < 1e-12 * scale
        assert np.abs(g - Vs[1][1]).max() < 1e-11 * np.abs(Vs[1][1]).max()
    Vf, gf = O.coulomb_fourier_above(sub, p)
    assert np.abs(Vf - Vs[1][0]).max() < 1e-12 * scale
    assert np.abs(gf - Vs[1][1]).max() < 1e-11 * np.abs(Vs[1][1]).max()
    # FD gradient of the Ewald form
    h = 1e-5
    for c in range(3):
        d = np.zeros(3); d[c] = h
        fd = (O.coulomb_ewald2d(sub, p + d)[0] - O.coulomb_ewald2d(sub, p - d)[0]) / (2 * h)
        assert np.abs(fd - Vs[1][1][:, c]).max() < 1e-8
    # corrugation decays with the shortest surface reciprocal vector |G| = 2 pi sqrt(2)/a
    z = np.arange(6.0, 12.0, 1.0)
    pts = np.stack([np.zeros_like(z), np.zeros_like(z), z], 1)
    V, _ = O.coulomb_ewald2d(sub, pts)
    slope = np.diff(np.log(np.abs(V)))
    assert np.allclose(slope, -2 * np.pi * np.sqrt(2) / sub.a, atol=1e-6)


def test_p7_constant_gauge_irrelevant_for_neutral_molecule():
    V = RNG.normal(size=(3, 8, 8, 10))
    spec = dict(nx=8, ny=8, nz=10, x0=0.0, y0=0.0, z0=1.0, dx=0.2, dy=0.2, dz=0.1)
    mol = S.mol_chain24()
    x = mol.pos * 0.3 + [0.5, 0.5, 1.5]
    plq = O.mixing(mol.eps, mol.R, mol.q)
    E0 = O.bspline_eval(O.fit_bspline(V), spec, x, plq)[0].sum()
    V2 = V.copy(); V2[2] += 0.37
    E1 = O.bspline_eval(O.fit_bspline(V2), spec, x, plq)[0].sum()
    # a constant c added to V^C shifts E by exactly c * sum Q (zero for a neutral molecule;
    # the FP32-rounded charges sum to ~1e-8)
    assert abs(E1 - E0 - 0.37 * mol.q.sum()) < 1e-12 * (1 + abs(E0))
    assert abs(mol.q.sum()) < 1e-6


# ------------------------------------------------------------------ P8: model vs direct
def test_p8_model_vs_direct_converges_fourth_order():
    """Interpolation error of the fitted model against the direct Morse sums falls by
    ~16x when the spacing halves (cubic B-spline interpolation: O(h^4) energy error)
    and stays within the tensor-product bound 3 * (5/384) h^4 max|d^4 V|."""
    sub = S.rocksalt_slab(1, 2)
    pts = S.random_points(200, sub.Lx, sub.Ly, 3.0, 3.6, 11)
    VP, VL, _, _ = O.morse_direct(sub, pts, rcut=20.0)
    errs = []
    for n in (56, 112):
        h = sub.Lx / n
        spec = dict(nx=n, ny=n, nz=int(round(3.5 / h)) + 1, x0=0.0, y0=0.0, z0=1.5, dx=h, dy=h, dz=h)
        I, J, K = np.meshgrid(np.arange(n), np.arange(n), np.arange(spec["nz"]), indexing="ij")
        idx = np.stack([I.ravel(), J.ravel(), K.ravel()], 1)
        vp, vl, _, _ = O.morse_direct(sub, O.node_coords(spec, idx), rcut=20.0)
        B = np.zeros((3, n, n, spec["nz"]))
        B[0] = O.fit_bspline(vp.reshape(n, n, -1))
        B[1] = O.fit_bspline(vl.reshape(n, n, -1))
        E0 = O.bspline_eval(B, spec, pts, np.tile([1.0, 0, 0], (len(pts), 1)))[0]
        E1 = O.bspline_eval(B, spec, pts, np.tile([0.0, 1.0, 0], (len(pts), 1)))[0]
        errs.append((np.abs(E0 - VP).max(), np.abs(E1 - VL).max()))
        # |d^4/dx^4| of a sum of exp(-k r) terms is at most k^4 times the channel value
        # near the point; the value is bounded by its maximum over the stencil (~2x at 0.1 A)
        assert errs[-1][0] < 3 * (5 / 384) * h ** 4 * 3.2 ** 4 * 2 * VP.max()
        assert errs[-1][1] < 3 * (5 / 384) * h ** 4 * 1.6 ** 4 * 2 * VL.max()
    for c in range(2):
        assert 12 < errs[0][c] / errs[1][c] < 22


# ------------------------------------------------------------------ P11: intramolecular
@pytest.mark.parametrize("mk", [S.mol_chain24, S.mol_pah38, lambda: S.mol_size(52, 6)])
def test_p11_intra_fd_and_invariants(mk):
    mol = mk()
    rng = np.random.default_rng(5)
    x = mol.pos + rng.normal(scale=0.08, size=mol.pos.shape)
    E, F = O.intra(mol, x)
    h = 1e-6
    Ffd = np.zeros_like(F)
    for i in range(mol.n):
        for c in range(3):
            xp = x.copy(); xp[i, c] += h
            xm = x.copy(); xm[i, c] -= h
            Ffd[i, c] = -(O.intra(mol, xp)[0] - O.intra(mol, xm)[0]) / (2 * h)
    assert np.abs(Ffd - F).max() < 1e-6 * max(1, np.abs(F).max())
    assert np.abs(F.sum(0)).max() < 1e-10 * max(1, np.abs(F).max())
    assert np.abs(np.cross(x - x.mean(0), F).sum(0)).max() < 1e-9 * max(1, np.abs(F).max())
    R = S.random_rotations(1, rng)[0]
    E2, F2 = O.intra(mol, x @ R.T + [3.0, -2.0, 7.0])
    assert abs(E2 - E) < 1e-10 * max(1, abs(E))
    assert np.abs(F2 - F @ R.T).max() < 1e-9 * max(1, np.abs(F).max())


def test_intra_reference_geometry_bonded_terms_at_rest():
    """Bond, angle and torsion parameters are taken at the reference geometry, so the
    bonded part of the field is at a minimum there (only non-bonded forces remain)."""
    mol = S.mol_pah38()
    Ez, Fz = O.intra(S.Molecule(**{**mol.__dict__, "q": np.zeros(mol.n), "eps": np.zeros(mol.n)}), mol.pos)
    assert abs(Ez) < 1e-9 and np.abs(Fz).max() < 1e-5


# ------------------------------------------------------------------ trilinear E/F scheme
def test_trilinear_reproduces_nodes_and_multilinear_fields():
    """Trilinear interpolation returns the stored values at nodes and reproduces any field
    that is linear in each coordinate separately (a + bx + cy + dz + exy + fyz + gxz + hxyz)
    inside the lattice, for the energy and each force component independently."""
    nx, ny, nz = 9, 8, 7
    spec = dict(nx=nx, ny=ny, nz=nz, x0=0.5, y0=-0.3, z0=1.0, dx=0.3, dy=0.25, dz=0.2)
    co = RNG.normal(size=(3, 4, 8))
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    X = spec["x0"] + ii * spec["dx"]; Y = spec["y0"] + jj * spec["dy"]; Z = spec["z0"] + kk * spec["dz"]

    def f(c, q, x, y, z):
        a = co[c, q]
        return a[0] + a[1] * x + a[2] * y + a[3] * z + a[4] * x * y + a[5] * y * z + a[6] * x * z + a[7] * x * y * z
    N = np.zeros((3, nx, ny, nz, 4))
    for c in range(3):
        for q in range(4):
            N[c, ..., q] = f(c, q, X, Y, Z)
    plq = RNG.normal(size=(200, 3))
    # interior points (away from the periodic wrap cell, where a non-periodic field jumps)
    pts = np.stack([spec["x0"] + RNG.uniform(0, (nx - 1) * spec["dx"], 200),
                    spec["y0"] + RNG.uniform(0, (ny - 1) * spec["dy"], 200),
                    spec["z0"] + RNG.uniform(0, (nz - 1) * spec["dz"], 200)], 1)
    E, F, fl = O.trilinear_eval(N, spec, pts, plq)
    want = [sum(plq[:, c] * f(c, q, pts[:, 0], pts[:, 1], pts[:, 2]) for c in range(3)) for q in range(4)]
    assert (fl == 0).all()
    assert np.abs(E - want[0]).max() < 1e-12 and np.abs(F - np.stack(want[1:], 1)).max() < 1e-12
    # at nodes: the stored values
    idx = [(0, 0, 0), (3, 5, 5), (8, 7, 2)]
    pn = np.array([[X[i], Y[i], Z[i]] for i in idx])
    E, F, _ = O.trilinear_eval(N, spec, pn, np.tile([1.0, 0.0, 0.0], (3, 1)))
    for r, i in enumerate(idx):
        assert abs(E[r] - N[0][i][0]) < 1e-12 and np.abs(F[r] - N[0][i][1:]).max() < 1e-12
    # domain: below z0 evaluated on the first plane and flagged; above the last plane zero
    E1, _, f1 = O.trilinear_eval(N, spec, np.array([[0.7, 0.1, 0.5], [0.7, 0.1, 1.0]]), np.tile([1.0, 0, 0], (2, 1)))
    assert f1[0] == 2 and f1[1] == 0 and E1[0] == E1[1]
    E2, F2, f2 = O.trilinear_eval(N, spec, np.array([[0.7, 0.1, 2.21]]), np.array([[1.0, 1.0, 1.0]]))
    assert E2[0] == 0 and (F2 == 0).all() and f2[0] == 0


def test_trilinear_nodes_are_the_model_at_the_nodes():
    """The stored table is the B-spline model's energy and force at each node, channel by
    channel: between nodes the trilinear force then differs from minus the gradient of the
    trilinear energy (the inconsistency the paper describes), while at nodes both agree with
    the model."""
    nx, ny, nz = 10, 10, 12
    spec = dict(nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=1.0, dx=0.3, dy=0.3, dz=0.25)
    B = O.fit_bspline(RNG.normal(size=(3, nx, ny, nz)))
    N = O.trilinear_nodes(B, spec)
    p = np.array([[0.9, 1.2, 1.0 + 5 * 0.25]])
    for c in range(3):
        m = np.zeros((1, 3)); m[0, c] = 1
        E, F, _ = O.bspline_eval(B, spec, p, m)
        assert abs(N[c, 3, 4, 5, 0] - E[0]) < 1e-12 and np.abs(N[c, 3, 4, 5, 1:] - F[0]).max() < 1e-12
    q = np.array([[1.0, 1.3, 2.33]]); m = np.array([[0.3, -0.7, 1.1]]); h = 1e-6
    _, Fq, _ = O.trilinear_eval(N, spec, q, m)
    g = [(O.trilinear_eval(N, spec, q + h * e, m)[0][0] - O.trilinear_eval(N, spec, q - h * e, m)[0][0]) / (2 * h)
         for e in np.eye(3)]
    assert np.abs(Fq[0] + np.array(g)).max() > 1e-3
    # the replica functions take the table in place of the coefficients
    mol = S.mol_chain24()
    x = mol.pos * 0.2 + [1.5, 1.5, 2.5]
    plq = O.mixing(mol.eps, mol.R, mol.q)
    Fb, Er, Ea, st = O.eval_batch(N, spec, [mol], [0], x, intra_on=False)
    Et, Ft, _ = O.trilinear_eval(N, spec, x, plq)
    assert np.abs(Ea - Et).max() < 1e-14 and np.abs(Fb - Ft).max() < 1e-14


# ------------------------------------------------------------------ P10: FIRE
def _one_atom():
    return S.Molecule(name="atom", elem=["C"], pos=np.zeros((1, 3)), q=np.zeros(1), eps=np.array([0.0]),
                      R=np.array([0.0]), mass=np.array([12.011]), bonds=np.zeros((0, 2), np.int32),
                      bond_k=np.zeros(0), bond_r0=np.zeros(0), angles=np.zeros((0, 3), np.int32),
                      angle_k=np.zeros(0), angle_cos0=np.zeros(0), tors=np.zeros((0, 4), np.int32),
                      tors_V=np.zeros(0), tors_n=np.zeros(0, np.int32), tors_phi0=np.zeros(0))


def test_p10_fire_converges_on_quadratic_bowl():
    """A one-atom 'molecule' with Q = 1 in a Coulomb channel whose B-spline model is the
    exact quadratic k|r - r*|^2 (coefficients from the P2 construction): FIRE reaches
    r* to the force tolerance."""
    d = 0.25
    nx = ny = nz = 24
    x = np.arange(nx) * d
    k, rs = 0.8, np.array([2.61, 3.07, 2.83])
    # p = k[(x-x*)^2 + (y-y*)^2 + (z-z*)^2]; per-axis operator (1 - d^2/6 D^2) of (x-x*)^2 is (x-x*)^2 - d^2/3
    gx = (x - rs[0]) ** 2; gy = (x - rs[1]) ** 2; gz = (x - rs[2]) ** 2
    B = np.zeros((3, nx, ny, nz))
    B[2] = k * ((gx - d * d / 3)[:, None, None] + (gy - d * d / 3)[None, :, None] + (gz - d * d / 3)[None, None, :])
    spec = dict(nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=0.0, dx=d, dy=d, dz=d)
    mol = _one_atom(); mol.q = np.array([1.0])
    starts = np.array([[1.5, 4.0, 3.5], [3.9, 2.2, 2.0], [2.0, 2.0, 4.2]])
    out = O.fire_batch(B, spec, [mol], [0, 0, 0], starts, 2000, intra_on=False, f_conv=1e-6)
    assert (out["status"] & 1).all()
    assert np.abs(out["pos"] - rs).max() < 1e-6 / (2 * k) * 1.01
    assert (out["fnorm"] < 1e-6).all()
    # a second call starting converged does not move and keeps the flag
    out2 = O.fire_batch(B, spec, [mol], [0, 0, 0], out["pos"], 50, vel=out["vel"],
                        state=dict(dt=out["dt"], alpha=out["alpha"], npos=out["npos"], status=out["status"]),
                        intra_on=False, f_conv=1e-6)
    assert np.array_equal(out2["pos"], out["pos"]) and (out2["steps"] == 0).all()


def _dimer():
    m = _one_atom()
    m.elem = ["C", "C"]; m.pos = np.zeros((2, 3)); m.q = np.zeros(2); m.eps = np.zeros(2); m.R = np.zeros(2)
    m.mass = np.array([12.011, 12.011]); m.bonds = np.array([[0, 1]], np.int32)
    m.bond_k = np.array([20.0]); m.bond_r0 = np.array([1.4])
    return m


def test_fire_restraint_holds_atom_and_relaxes_the_rest():
    """A restrained atom never moves; its bonded partner relaxes along the bond to the rest
    length (the bond force is radial and FIRE starts from rest, so the direction is kept);
    replicas without a restraint are unaffected."""
    spec = dict(nx=4, ny=4, nz=4, x0=0.0, y0=0.0, z0=-50.0, dx=1.0, dy=1.0, dz=1.0)
    B = np.zeros((3, 4, 4, 4))
    m = _dimer()
    x0 = np.array([[0.3, 0.2, 0.1], [2.2, 0.6, -0.3], [0.0, 0.0, 0.0], [1.0, 0.9, 0.0]])
    target = np.array([[0.0, 0.0, 0.0], [9.0, 9.0, 9.0]])
    out = O.fire_batch(B, spec, [m], [0, 0], x0, 3000, f_conv=1e-8, intra_on=True,
                       fixed_atom=np.array([0, -1]), fixed_pos=target)
    assert (out["status"] & 1).all()
    assert np.array_equal(out["pos"][0], target[0])
    d = out["pos"][1] - out["pos"][0]
    u = (x0[1] - target[0]) / np.linalg.norm(x0[1] - target[0])
    assert abs(np.linalg.norm(d) - 1.4) < 1e-8 / 20
    assert np.abs(d / np.linalg.norm(d) - u).max() < 1e-9
    free = O.fire_batch(B, spec, [m], [0], x0[2:], 3000, f_conv=1e-8)
    assert np.array_equal(out["pos"][2:], free["pos"])


def test_fire_restraint_at_the_minimum_is_inactive():
    """Holding one atom where the free relaxation put it leaves that minimum a minimum: a
    perturbed start relaxes back to the same energy and geometry."""
    spec = dict(nx=8, ny=8, nz=12, x0=0.0, y0=0.0, z0=1.0, dx=0.5, dy=0.5, dz=0.5)
    B = O.fit_bspline(RNG.normal(size=(3, 8, 8, 12)) * 0.01)
    mol = S.mol_chain24()
    x0 = mol.pos + [2.0, 2.0, 4.0]
    free = O.fire_batch(B, spec, [mol], [0], x0, 20000, f_conv=1e-7)
    assert (free["status"] & 1).all()
    xs = free["pos"]
    j = 5
    start = xs + np.random.default_rng(3).normal(0, 0.02, xs.shape)
    held = O.fire_batch(B, spec, [mol], [0], start, 20000, f_conv=1e-7, fixed_atom=np.array([j]),
                        fixed_pos=xs[j][None])
    assert (held["status"] & 1).all()
    assert np.array_equal(held["pos"][j], xs[j])
    assert abs(held["E"][0] - free["E"][0]) < 1e-9
    assert np.abs(held["pos"] - xs).max() < 1e-4


def test_fire_resume_equals_continuous():
    sub_spec = dict(nx=8, ny=8, nz=12, x0=0.0, y0=0.0, z0=1.0, dx=0.5, dy=0.5, dz=0.5)
    B = O.fit_bspline(RNG.normal(size=(3, 8, 8, 12)) * [[[[0.01]]], [[[0.01]]], [[[0.01]]]])
    mol = S.mol_chain24()
    x0 = mol.pos + [2.0, 2.0, 4.0]
    a = O.fire_batch(B, sub_spec, [mol], [0], x0, 40, f_conv=0.0)
    b1 = O.fire_batch(B, sub_spec, [mol], [0], x0, 20, f_conv=0.0)
    b2 = O.fire_batch(B, sub_spec, [mol], [0], b1["pos"], 20, vel=b1["vel"],
                      state=dict(dt=b1["dt"], alpha=b1["alpha"], npos=b1["npos"], status=b1["status"]),
                      f_conv=0.0)
    assert np.array_equal(a["pos"], b2["pos"]) and np.array_equal(a["vel"], b2["vel"])
    assert a["E"][0] < O.intra(mol, x0)[0]   # relaxation lowered the energy


# ------------------------------------------------------------------ P9: NVE
def test_p9_nve_energy_fluctuation_scales_dt2():
    mol = S.mol_chain24()
    spec = dict(nx=4, ny=4, nz=4, x0=0.0, y0=0.0, z0=-50.0, dx=1.0, dy=1.0, dz=1.0)
    B = np.zeros((3, 4, 4, 4))
    x0 = mol.pos.copy()
    v0 = S.mb_velocities(mol.mass, 1, 300.0, 7000)[0]
    fl = []
    for dt in (0.5, 0.25):
        n = int(round(200 / dt))
        out = O.nve_batch(B, spec, [mol], [0], x0, v0, n, dt=dt, drift_every=1)
        fl.append(out["drift"][0, 2])
    assert 3.0 < fl[0] / fl[1] < 5.0


# ------------------------------------------------------------------ RNG and proposals
def load_philox_kat():
    import os
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(t, 16) for t in line.split()]
                rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answer_vectors():
    for ctr, key, out in load_philox_kat():
        assert O.philox4x32_10(ctr, key) == out


def test_uniform_proposals_and_pose():
    mol = S.mol_chain24()
    T = len(mol.rot_quads)
    dof = O.propose_uniform(2000, T, S.SEED_PHILOX, 0)
    assert (dof[:, :2] >= 0).all() and (dof[:, :2] < 1).all()
    assert (dof[:, 2] >= 3).all() and (dof[:, 2] <= 5).all()
    assert np.allclose(np.linalg.norm(dof[:, 3:7], axis=1), 1, atol=1e-12)
    # Shoemake quaternions are uniform on S^3: each component has E[q^2] = 1/4
    assert np.allclose((dof[:, 3:7] ** 2).mean(0), 0.25, atol=0.03)
    Lx = Ly = 11.28
    P = O.pose(mol, dof[:20], Lx, Ly, 0.0)
    for r in range(20):
        x = P[r]
        for k in range(T):
            q = mol.rot_quads[k]
            phi = O.dihedral(x[q])
            dphi = (phi - dof[r, 7 + k] + np.pi) % (2 * np.pi) - np.pi
            assert abs(dphi) < 1e-9
        for (i, j), r0 in zip(mol.bonds, np.linalg.norm(mol.pos[mol.bonds[:, 0]] - mol.pos[mol.bonds[:, 1]], axis=1)):
            assert abs(np.linalg.norm(x[i] - x[j]) - r0) < 1e-9
        assert abs(x[:, 2].min() - dof[r, 2]) < 1e-12
        assert np.allclose(x[:, :2].mean(0), dof[r, :2] * [Lx, Ly], atol=1e-12)


# ------------------------------------------------------------------ Langevin (BAOAB)
KB = 8.617333262e-5
AMU = 103.6426965268


def test_langevin_without_friction_is_velocity_verlet():
    """gamma = 0 removes the O step (c1 = 1, c2 = 0): BAOAB is then velocity Verlet."""
    spec = dict(nx=8, ny=8, nz=12, x0=0.0, y0=0.0, z0=1.0, dx=0.5, dy=0.5, dz=0.5)
    B = O.fit_bspline(RNG.normal(size=(3, 8, 8, 12)) * 0.01)
    mol = S.mol_chain24()
    x0 = mol.pos + [2.0, 2.0, 4.0]
    v0 = S.mb_velocities(mol.mass, 1, 300.0, 7001)[0]
    a = O.nve_batch(B, spec, [mol], [0], x0, v0, 60, dt=0.5)
    b = O.langevin_batch(B, spec, [mol], [0], x0, v0, 60, dt=0.5, gamma=0.0, seed=3)
    assert np.abs(a["pos"] - b["pos"]).max() < 1e-10
    assert np.abs(a["vel"] - b["vel"]).max() < 1e-10
    assert abs(a["E"][0] - b["E"][0]) < 1e-9


def test_langevin_noise_keyed_by_replica_id_seed_and_round():
    spec = dict(nx=8, ny=8, nz=12, x0=0.0, y0=0.0, z0=1.0, dx=0.5, dy=0.5, dz=0.5)
    B = O.fit_bspline(RNG.normal(size=(3, 8, 8, 12)) * 0.01)
    mol = S.mol_chain24()
    xa, xb = mol.pos + [2.0, 2.0, 4.0], mol.pos + [2.5, 1.0, 4.2]
    v = np.zeros((2 * mol.n, 3))
    run = lambda x, ids, **kw: O.langevin_batch(B, spec, [mol], [0, 0], x, v, 30, gamma=0.05, rep_id=ids, **kw)
    r1 = run(np.concatenate([xa, xb]), [5, 9], seed=11, rnd=2)
    r2 = run(np.concatenate([xb, xa]), [9, 5], seed=11, rnd=2)     # same ids, other batch order
    assert np.array_equal(r1["pos"], np.concatenate([r2["pos"][mol.n:], r2["pos"][:mol.n]]))
    r3 = run(np.concatenate([xa, xb]), [5, 9], seed=11, rnd=3)
    r4 = run(np.concatenate([xa, xb]), [5, 9], seed=12, rnd=2)
    assert np.abs(r3["pos"] - r1["pos"]).max() > 1e-4 and np.abs(r4["pos"] - r1["pos"]).max() > 1e-4


def test_batch_wrappers_accept_strided_coordinates():
    """Coordinates handed over as transposed views (as a [3][N] layout yields) give the same
    trajectories as contiguous copies."""
    spec = dict(nx=8, ny=8, nz=12, x0=0.0, y0=0.0, z0=1.0, dx=0.5, dy=0.5, dz=0.5)
    B = O.fit_bspline(RNG.normal(size=(3, 8, 8, 12)) * 0.01)
    mol = S.mol_chain24()
    x = np.ascontiguousarray((mol.pos + [2.0, 2.0, 4.0]).T).T       # (n, 3) view of a (3, n) array
    v = np.ascontiguousarray(S.mb_velocities(mol.mass, 1, 300.0, 7002)[0].T).T
    assert not x.flags.c_contiguous
    xc, vc = np.ascontiguousarray(x), np.ascontiguousarray(v)
    for f in (lambda p, u: O.fire_batch(B, spec, [mol], [0], p, 20, vel=u),
              lambda p, u: O.nve_batch(B, spec, [mol], [0], p, u, 20),
              lambda p, u: O.langevin_batch(B, spec, [mol], [0], p, u, 20, gamma=0.05, rep_id=np.array([3, 9])[::2])):
        assert np.array_equal(f(x, v)["pos"], f(xc, vc)["pos"])


def test_langevin_harmonic_stationary_moments():
    """One-atom molecules (q = 1) in a Coulomb channel whose B-spline model is exactly
    k (z - zc)^2 and flat laterally.  For a quadratic potential BAOAB samples positions
    with the exact variance kT/K (K = 2k) at any stable step, and velocities along z with
    variance (kT/m)(1 - (w dt/2)^2), w^2 = K/m (the stationary solution of the scheme's
    linear recurrence); the force-free lateral velocities are an exact Ornstein-Uhlenbeck
    process with variance kT/m.  A wrong splitting order or a dropped half kick moves these
    moments by 25 % or more for the light atom (w dt = 1)."""
    d, nz, zc = 0.5, 16, 3.75
    z = np.arange(nz) * d
    T, dt, gamma = 300.0, 1.0, 0.2
    kT = KB * T
    m_h, m_c = 1.008, 12.011
    K = m_h * AMU * 1.0 ** 2                  # w dt = 1 for the light atom
    B = np.zeros((3, 6, 6, nz))
    B[2] = (0.5 * K * ((z - zc) ** 2 - d * d / 3))[None, None, :]
    spec = dict(nx=6, ny=6, nz=nz, x0=0.0, y0=0.0, z0=0.0, dx=d, dy=d, dz=d)
    mols = []
    for m in (m_h, m_c):
        a = _one_atom(); a.q = np.array([1.0]); a.mass = np.array([m]); mols.append(a)
    nr = 300
    rep_type = np.repeat([0, 1], nr)
    x = np.zeros((2 * nr, 3)); x[:, :2] = np.random.default_rng(5).random((2 * nr, 2)) * 3.0; x[:, 2] = zc
    v = np.zeros((2 * nr, 3))
    zz, vz, vl = [], [], []
    for rnd in range(260):
        out = O.langevin_batch(B, spec, mols, rep_type, x, v, 10, dt=dt, T=T, gamma=gamma, seed=77, rnd=rnd,
                               intra_on=False)
        x, v = out["pos"], out["vel"]
        assert (out["status"] == 0).all()
        if rnd >= 20:
            zz.append((x[:, 2] - zc) ** 2); vz.append(v[:, 2] ** 2); vl.append(0.5 * (v[:, 0] ** 2 + v[:, 1] ** 2))
    zz, vz, vl = np.array(zz), np.array(vz), np.array(vl)
    for t, m in enumerate((m_h, m_c)):
        sel = rep_type == t
        w = np.sqrt(K / (m * AMU))
        assert zz[:, sel].mean() / (kT / K) == pytest.approx(1.0, abs=0.03)
        assert vz[:, sel].mean() / (kT / (m * AMU) * (1 - (w * dt / 2) ** 2)) == pytest.approx(1.0, abs=0.03)
        assert vl[:, sel].mean() / (kT / (m * AMU)) == pytest.approx(1.0, abs=0.03)


def test_direct_image_sum_pins():
    """The all-atom comparison's image sum (Section "Configuration sampling on GPU"):
    its Pauli/London part equals the pinned Morse image sums where the atoms beyond the 3x3
    cell block lie more than 15 A away (tail below 1e-8 relative); its Coulomb part
    converges to the 2D Ewald sum of the neutral zero-dipole slab as the square block of
    images grows (error falling about 8x per doubling); F = -grad E by central differences."""
    sub = S.rocksalt_slab(2, 3)
    rng = np.random.default_rng(0)
    pts = np.stack([rng.uniform(0.4, 0.6, 6) * sub.Lx, rng.uniform(0.4, 0.6, 6) * sub.Ly,
                    rng.uniform(2.5, 5.0, 6)], 1)
    plq = np.tile([0.7, -1.3, 0.0], (6, 1))
    VP, VL, gP, gL = O.morse_direct(sub, pts, 1.6, 40.0)
    E, F = O.direct_images(sub, pts, plq, nimg=1)
    ref = 0.7 * VP - 1.3 * VL
    assert np.abs(E - ref).max() < 1e-8 * np.abs(ref).max()
    assert np.abs(F + (0.7 * gP - 1.3 * gL)).max() < 1e-8 * np.abs(0.7 * gP - 1.3 * gL).max()
    plq = np.tile([0.0, 0.0, 1.0], (6, 1))
    VC, gC = O.coulomb_ewald2d(sub, pts)
    err = [np.abs(O.direct_images(sub, pts, plq, nimg=k)[0] - VC).max() for k in (10, 20, 40)]
    assert err[2] < 1e-6 and err[0] / err[1] > 6 and err[1] / err[2] > 6
    Ec, Fc = O.direct_images(sub, pts, plq, nimg=40)
    assert np.abs(Fc + gC).max() < 1e-6
    # force = -grad E, all channels together
    plq = np.tile([0.7, -1.3, 0.4], (6, 1))
    E0, F0 = O.direct_images(sub, pts, plq, nimg=1)
    h = 1e-5
    for c in range(3):
        d = np.zeros(3); d[c] = h
        fd = -(O.direct_images(sub, pts + d, plq)[0] - O.direct_images(sub, pts - d, plq)[0]) / (2 * h)
        assert np.abs(fd - F0[:, c]).max() < 1e-6 * max(1.0, np.abs(F0).max())
