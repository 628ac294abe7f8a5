"""Pins of the oracle's sampling rows (proposals, pose encoding, dedupe, proposer MLP)."""
import numpy as np
import pytest

import oracle as O
from oracle import sampling as OS
from paper_2508_15522_amd import synth as S


def test_horn_quaternion_matches_svd_kabsch():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(20, 3)); X -= X.mean(0)
    R = S.random_rotations(1, rng)[0]
    Y = X @ R.T + rng.normal(scale=0.01, size=X.shape); Y -= Y.mean(0)
    q = OS.horn_quaternion(X, Y)
    U, s, Vt = np.linalg.svd(X.T @ Y)
    D = np.diag([1, 1, np.sign(np.linalg.det(Vt.T @ U.T))])
    Rk = Vt.T @ D @ U.T
    assert np.allclose(OS.quat_to_matrix(q), Rk, atol=1e-12)
    assert q[0] >= 0


@pytest.mark.parametrize("mk", [S.mol_chain24, lambda: S.mol_size(52, 6)])
def test_encode_inverts_pose(mk):
    mol = mk()
    T = len(mol.rot_quads)
    dof = O.propose_uniform(30, T, 77, 3)
    dof[:, 3:7] *= np.where(dof[:, 3:4] < 0, -1, 1)          # canonical sign (w >= 0)
    P = O.pose(mol, dof, 11.28, 11.28, 0.0)
    for r in range(30):
        e = OS.encode_pose(mol, P[r], 11.28, 11.28, 0.0)
        d = OS.decode_dof(e, T, 0.0, 10.0)
        assert np.allclose(d[:3], dof[r, :3], atol=1e-9)
        assert np.allclose(d[3:7], dof[r, 3:7], atol=1e-9)
        ang = (d[7:] - dof[r, 7:] + np.pi) % (2 * np.pi) - np.pi
        assert np.abs(ang).max() < 1e-9
        # decoding then posing reproduces the pose
        assert np.abs(O.pose(mol, d, 11.28, 11.28, 0.0)[0] - P[r]).max() < 1e-9


def test_dedupe_semantics():
    E = np.array([-1.0, -1.005, -1.02, -1.0149, -2.0, np.nan, -1.0])
    t = np.array([0, 0, 0, 0, 0, 0, 1])
    new, arch = OS.dedupe_energy(E, t, None, 0.01)
    # -1.005 matches -1.0; -1.02 is new; -1.0149 matches -1.02 (|d| < 0.01); NaN never counts;
    # the same energy in another type is new
    assert list(new) == [1, 0, 1, 0, 1, 0, 1]
    new2, _ = OS.dedupe_energy(np.array([-1.0, -3.0]), np.array([0, 0]), None, 0.01, arch)
    assert list(new2) == [0, 1]


def test_rmsd_lattice_closed_forms():
    mol = S.mol_chain24()
    A = mol.pos + [2.0, 3.0, 4.0]
    Lx, Ly = 11.28, 8.46
    assert OS.rmsd_lattice(A, A, Lx, Ly) == 0.0
    assert OS.rmsd_lattice(A + [3 * Lx, -2 * Ly, 0.0], A, Lx, Ly) < 1e-12
    # a rigid shift s: the distance from s to the nearest lattice vector, here (Lx, 0, 0)
    s = np.array([0.7 * Lx, -0.2 * Ly, 0.15])
    want = np.sqrt((0.3 * Lx) ** 2 + (0.2 * Ly) ** 2 + 0.15 ** 2)
    assert abs(OS.rmsd_lattice(A + s, A, Lx, Ly) - want) < 1e-12
    assert abs(OS.rmsd_lattice(A, A + s, Lx, Ly) - want) < 1e-12
    # a rotation by th about the vertical axis through the centroid is not fitted away:
    # |R r - r|^2 = 2 rho^2 (1 - cos th), rho the distance from the axis
    th = 0.3
    c = A.mean(0)
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    Arot = (A - c) @ R.T + c
    rho2 = ((A - c)[:, :2] ** 2).sum(1)
    assert abs(OS.rmsd_lattice(Arot, A, Lx, Ly) - np.sqrt(np.mean(2 * rho2 * (1 - np.cos(th))))) < 1e-12
    # nor is a permutation: swapping atoms i and j moves two atoms by |x_i - x_j|
    P = A.copy(); P[[3, 10]] = P[[10, 3]]
    assert abs(OS.rmsd_lattice(P, A, Lx, Ly) - np.sqrt(2 * ((A[3] - A[10]) ** 2).sum() / len(A))) < 1e-12


def test_dedupe_rmsd_discovery_order():
    mol = S.mol_chain24()
    A = mol.pos + [2.0, 3.0, 4.0]
    Lx = Ly = 11.28
    s = np.array([0.08, 0.0, 0.0])
    B, Cc = A + s, A + 2 * s                  # rmsd(A,B) = rmsd(B,C) = 0.08, rmsd(A,C) = 0.16
    new, arch = OS.dedupe_rmsd([A, B, Cc], [0, 0, 0], None, 0.1, Lx, Ly)
    assert list(new) == [1, 0, 1]             # C is compared with the accepted A only
    new, _ = OS.dedupe_rmsd([B, A, Cc], [0, 0, 0], None, 0.1, Lx, Ly)
    assert list(new) == [1, 0, 0]
    N = A.copy(); N[5, 1] = np.nan
    new, _ = OS.dedupe_rmsd([A, A, N, A + [Lx, 0, 0], A], [0, 1, 0, 0, 0], [1, 1, 1, 1, 0], 0.1, Lx, Ly)
    assert list(new) == [1, 1, 0, 0, 0]       # another type is new; NaN, lattice image, ok=0 are not
    new2, arch2 = OS.dedupe_rmsd([Cc + [0, Ly, 0], A + [0, 0, 0.5]], [0, 0], None, 0.1, Lx, Ly, arch)
    assert list(new2) == [0, 1] and len(arch2) == 3


def test_mlp_backward_matches_finite_differences():
    """P12: the FP64 oracle's gradient against central differences of its own loss."""
    n_types = 3
    rng = np.random.default_rng(1)
    p = S.mlp_init_params(n_types).astype(np.float64)
    B = 6
    noise = rng.normal(size=(B, 64))
    types = rng.integers(0, n_types, B)
    target = rng.normal(size=(B, 41)) * 0.5
    ntors = rng.integers(0, 17, B)
    # BF16 rounding is piecewise constant in the weights, so differentiate with respect to
    # parameters through a model whose weights are already BF16 values: perturb biases and
    # the embedding's effect exactly, weights by BF16-representable steps is not smooth --
    # use the bias and final-layer entries, and a smooth surrogate for the rest below
    L, g, _ = OS.loss_and_grad(p, n_types, noise, types, target, ntors)
    idx = []
    o = 0
    for l in range(4):
        nW = OS.DIMS[l + 1] * OS.DIMS[l]
        idx += [o + nW + k for k in (0, 5, OS.DIMS[l + 1] - 1)]     # biases
        o += nW + OS.DIMS[l + 1]
    for i in idx:
        h = 1e-6
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (OS.loss_and_grad(pp, n_types, noise, types, target, ntors)[0] -
              OS.loss_and_grad(pm, n_types, noise, types, target, ntors)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])
    # weights: with the BF16 rounding switched off the analytic gradient matches FD too
    orig = OS.bf16
    try:
        OS.bf16 = lambda a: np.asarray(a, dtype=np.float64)
        L, g, _ = OS.loss_and_grad(p, n_types, noise, types, target, ntors)
        o = 0
        for l in range(4):
            for i in (o, o + 7, o + OS.DIMS[l] + 3):
                h = 1e-6
                pp = p.copy(); pp[i] += h
                pm = p.copy(); pm[i] -= h
                fd = (OS.loss_and_grad(pp, n_types, noise, types, target, ntors)[0] -
                      OS.loss_and_grad(pm, n_types, noise, types, target, ntors)[0]) / (2 * h)
                assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (l, i, fd, g[i])
            o += OS.DIMS[l + 1] * OS.DIMS[l] + OS.DIMS[l + 1]
        for i in range(o, o + 5):                                           # embedding
            h = 1e-6
            pp = p.copy(); pp[i] += h
            pm = p.copy(); pm[i] -= h
            fd = (OS.loss_and_grad(pp, n_types, noise, types, target, ntors)[0] -
                  OS.loss_and_grad(pm, n_types, noise, types, target, ntors)[0]) / (2 * h)
            assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])
    finally:
        OS.bf16 = orig


def test_bf16_rounding_rule():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 1e-30])
    r = OS.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0                 # tie to even
    assert r[2] == 1.0 + 2 ** -7                       # tie to even (odd mantissa rounds up)
    assert abs(r[3] + 3.14159) <= 2 ** -8 * 3.15
    assert (np.abs(r - x) <= np.abs(x) * 2 ** -8).all()


def test_normal_philox_moments():
    z = OS.normal_philox(40000, 9, 2)
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1) < 0.02
    assert abs((z ** 4).mean() - 3) < 0.1


def test_mlp_forward_path_closed_form():
    """One live path through the four layers (input 0 -> unit 0 -> unit 0 -> unit 0 -> output
    3, weights exactly representable in BF16, everything else zero): the output is the
    composition silu(silu(silu(s x0 + b1) + b2) + b3) w4 + b4 of the scalar SiLU x/(1+e^-x);
    with all weights zero the output is the last bias."""
    n_types = 2
    sizes = [(OS.DIMS[l + 1], OS.DIMS[l]) for l in range(4)]
    n = sum(a * b + a for a, b in sizes) + n_types * 32
    p = np.zeros(n)
    o = 0
    Ws, bs = [], []
    for a, b in sizes:
        Ws.append(o); o += a * b
        bs.append(o); o += a
    s, b1, b2, b3, w4, b4 = 1.5, 0.25, -0.5, 0.75, -2.0, 0.125
    p[Ws[0] + 0 * 96 + 0] = s
    p[bs[0] + 0] = b1
    p[Ws[1] + 0] = 1.0; p[bs[1] + 0] = b2
    p[Ws[2] + 0] = 1.0; p[bs[2] + 0] = b3
    p[Ws[3] + 3 * 256 + 0] = w4; p[bs[3] + 3] = b4
    noise = np.array([[0.7] + [0.3] * 63, [-1.9] + [5.0] * 63])
    Y, _ = OS.forward(p, n_types, noise, np.array([0, 1]))
    f = lambda z: z / (1.0 + np.exp(-z))
    for r in range(2):
        want = f(f(f(s * noise[r, 0] + b1) + b2) + b3) * w4 + b4
        assert abs(Y[r, 3] - want) < 1e-14
        others = np.delete(Y[r], 3)
        assert np.abs(others).max() == 0.0
    q = np.zeros(n); q[bs[3]:bs[3] + 41] = np.arange(41) * 0.5
    Y0, _ = OS.forward(q, n_types, noise, np.array([1, 0]))
    assert np.array_equal(Y0, np.tile(np.arange(41) * 0.5, (2, 1)))


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are exact (m_hat = g,
    v_hat = g^2) at every step, so each Adam step moves a parameter by lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, -1.0, 0.5, 2.0])
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    lr = 1e-2
    for step in range(1, 51):
        p, m, v = OS.adam(p, g, m, v, step, lr)
        assert np.allclose(p, p0 - step * lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-13)


def test_imle_select_brute_force_cases():
    """The nearest candidate under the encoding distance: an exact copy of the target wins;
    the quaternion block is compared up to sign (q and -q are one rotation); angle pairs
    beyond the molecule's torsion count are ignored; ties go to the lowest index."""
    rng = np.random.default_rng(2)
    t = rng.normal(size=(3, 41))
    cand = rng.normal(size=(3, 5, 41)) * 3.0
    cand[0, 3] = t[0]                                    # exact copy
    flip = t[1].copy(); flip[5:9] *= -1; cand[1, 2] = flip     # quaternion sign flipped
    junk = t[2].copy(); junk[9 + 2 * 2:] += 50.0         # differs only beyond 2 torsions
    cand[2, 1] = junk; cand[2, 4] = junk                 # tie: lowest index
    best, d = OS.imle_select(cand, t, np.array([16, 16, 2]))
    assert list(best) == [3, 2, 1]
    assert d[0] == 0.0 and d[1] < 1e-24 and d[2] == 0.0
