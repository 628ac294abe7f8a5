"""Closed-form pins of the oracle's intramolecular field and FIRE update order.

The finite-difference, zero-net-force and rigid-motion pins of the intramolecular field
would pass a misread term (a different angle form, a dropped factor in the Morse
attraction, 1-4 pairs excluded); the quadratic-bowl pin of FIRE would pass a different
update order.  These tests fix each against a value worked out by hand:

* non-bonded pair (Section "Principles", Eqs. E_Morse and E_Coulomb, with the product
  depth eps_i eps_j at separation R_i + R_j): at s = r - R_i - R_j = 0 the Morse part is
  -eps_i eps_j with zero slope; at e^{-alpha s} = 1/2 it is -3/4 eps_i eps_j with slope
  +alpha/2 eps_i eps_j;
* angle 1/2 k (cos th - cos th0)^2, torsion 1/2 V (1 - cos(n phi - phi0)) with the IUPAC
  sign of phi, and the force each puts on the outer atoms (lever arm closed forms);
* exclusions: exactly the pairs one or two bonds apart are excluded, 1-4 pairs count;
* FIRE (Bitzek et al. 2006, as used in Section "Accuracy and performance tests on CPU"):
  per move P = F.v, mix with the current alpha, adapt (on P > 0 the streak grows, and
  beyond N_min dt grows and alpha shrinks; otherwise dt halves, alpha resets, v = 0),
  kick with the adapted dt, move by v dt capped per atom.  A three-move trajectory in an
  anisotropic quadratic bowl is worked out by hand below.
No GPU.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2508_15522_amd import synth as S

K_E = 14.3996454784
ALPHA = 1.6


def _mol(pos, bonds=(), angles=(), tors=(), eps=None, R=None, q=None, angle_k=5.0, cos0=None, tors_V=None,
         tors_n=None, tors_phi0=None):
    """A molecule with explicit terms; bond force constants are zero so that only the
    terms under test contribute (the bonds still define the exclusions)."""
    n = len(pos)
    bonds = np.array(bonds, np.int32).reshape(-1, 2)
    angles = np.array(angles, np.int32).reshape(-1, 3)
    tors = np.array(tors, np.int32).reshape(-1, 4)
    return S.Molecule(
        name="pin", elem=["C"] * n, pos=np.array(pos, float), q=np.zeros(n) if q is None else np.array(q, float),
        eps=np.zeros(n) if eps is None else np.array(eps, float), R=np.zeros(n) if R is None else np.array(R, float),
        mass=np.full(n, 12.011), bonds=bonds, bond_k=np.zeros(len(bonds)), bond_r0=np.ones(len(bonds)),
        angles=angles, angle_k=np.full(len(angles), angle_k),
        angle_cos0=np.zeros(len(angles)) if cos0 is None else np.full(len(angles), cos0),
        tors=tors, tors_V=np.zeros(len(tors)) if tors_V is None else np.array(tors_V, float),
        tors_n=np.ones(len(tors), np.int32) if tors_n is None else np.array(tors_n, np.int32),
        tors_phi0=np.zeros(len(tors)) if tors_phi0 is None else np.array(tors_phi0, float))


# ------------------------------------------------------------------ non-bonded pair
@pytest.mark.parametrize("which", ["C-O", "H-C"])
def test_pair_morse_minimum_and_coulomb(which):
    """Two unbonded atoms at r = R_i + R_j: the Morse term sits at its minimum, depth
    eps_i eps_j, slope zero, so the whole force is the Coulomb force k_e Q_i Q_j / r^2."""
    eps, R, q = {"C-O": ([0.07, 0.08], [1.90, 1.75], [0.31, -0.22]),
                 "H-C": ([0.04, 0.07], [1.45, 1.90], [-0.17, -0.09])}[which]
    r = R[0] + R[1]
    u = np.array([2.0, -1.0, 2.0]) / 3.0                       # unit vector from atom 1 to atom 0
    x = np.array([[0.4, 0.1, -0.3], [0.4, 0.1, -0.3]]); x[0] += r * u
    E, F = O.intra(_mol(x, eps=eps, R=R, q=q), x)
    coul = K_E * q[0] * q[1] / r
    assert E == pytest.approx(-eps[0] * eps[1] + coul, abs=1e-13)
    np.testing.assert_allclose(F[0], K_E * q[0] * q[1] / r ** 2 * u, atol=1e-13)
    np.testing.assert_allclose(F[1], -F[0], atol=1e-15)


def test_pair_morse_at_half_attraction():
    """At e^{-alpha s} = 1/2 the Morse factor e^{-2 alpha s} - 2 e^{-alpha s} is
    1/4 - 1 = -3/4 and its r-derivative -2 alpha/4 + 2 alpha/2 = alpha/2: the pair pulls
    with -dE/dr = -alpha/2 eps_i eps_j (no charges)."""
    eps, R = [0.15, 0.05], [2.0, 1.5]
    r = R[0] + R[1] + math.log(2.0) / ALPHA
    x = np.array([[0.0, 0.0, 0.0], [0.0, r, 0.0]])
    E, F = O.intra(_mol(x, eps=eps, R=R), x)
    ee = eps[0] * eps[1]
    assert E == pytest.approx(-0.75 * ee, abs=1e-14)
    # atom 1 sits at +r along y and is pulled back towards atom 0
    np.testing.assert_allclose(F[1], [0.0, -0.5 * ALPHA * ee, 0.0], atol=1e-14)
    np.testing.assert_allclose(F[0], [0.0, 0.5 * ALPHA * ee, 0.0], atol=1e-14)


# ------------------------------------------------------------------ angle
@pytest.mark.parametrize("theta_deg", [90.0, 120.0, 75.0])
def test_angle_cosine_harmonic_closed_form(theta_deg):
    """Vertex at the origin, arms of 1.3 and 1.1 A: E = 1/2 k (cos th - cos th0)^2.  The
    force on an outer atom is -dE/dth / arm along the direction that opens the angle,
    dE/dth = -k (cos th - cos th0) sin th; the vertex takes the balance."""
    k, th0 = 5.0, math.radians(109.5)
    th = math.radians(theta_deg)
    x = np.array([[1.3, 0.0, 0.0], [0.0, 0.0, 0.0], [1.1 * math.cos(th), 1.1 * math.sin(th), 0.0]])
    mol = _mol(x, bonds=[(0, 1), (1, 2)], angles=[(0, 1, 2)], angle_k=k, cos0=math.cos(th0))
    E, F = O.intra(mol, x)
    assert E == pytest.approx(0.5 * k * (math.cos(th) - math.cos(th0)) ** 2, abs=1e-14)
    dEdth = -k * (math.cos(th) - math.cos(th0)) * math.sin(th)
    # moving atom 0 along +y closes the angle; moving atom 2 along e_th = (-sin, cos) opens it
    np.testing.assert_allclose(F[0], [0.0, dEdth / 1.3, 0.0], atol=1e-13)
    np.testing.assert_allclose(F[2], -dEdth / 1.1 * np.array([-math.sin(th), math.cos(th), 0.0]), atol=1e-13)
    np.testing.assert_allclose(F[1], -(F[0] + F[2]), atol=1e-13)


# ------------------------------------------------------------------ torsion
TORSION_VARIANTS = [
    (0.1, 3, math.pi),     # soft sp3 torsion: minima at the staggered angles
    (1.0, 2, 0.0),         # stiff planar torsion: minima at 0 and 180 degrees
    (1.0, 1, math.pi),     # stiff trans torsion
    (1.0, 1, 1.0),         # stiff torsion with its reference dihedral: fixes the sign of phi
]


@pytest.mark.parametrize("V,n,phi0", TORSION_VARIANTS)
@pytest.mark.parametrize("phi_deg", [-150.0, -60.0, 35.0, 60.0, 100.0, 180.0])
def test_torsion_closed_form_and_iupac_sign(V, n, phi0, phi_deg):
    """j at the origin, k on +z, i - j = 1.3 x, l - k = 1.4 (cos phi, sin phi, 0): looking
    from j to k, the i-j bond turns clockwise by phi to eclipse k-l, so this is the IUPAC
    dihedral phi.  E = 1/2 V (1 - cos(n phi - phi0)); the force on l is -dE/dphi / 1.4 along
    e_phi = (-sin phi, cos phi, 0), the force on i is +dE/dphi / 1.3 along +y (moving i
    towards +y lowers phi).  Charges and Morse factors are zero, so the 1-4 pair is silent."""
    phi = math.radians(phi_deg)
    x = np.array([[1.3, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 1.5],
                  [1.4 * math.cos(phi), 1.4 * math.sin(phi), 1.5]])
    mol = _mol(x, bonds=[(0, 1), (1, 2), (2, 3)], tors=[(0, 1, 2, 3)], tors_V=[V], tors_n=[n], tors_phi0=[phi0])
    E, F = O.intra(mol, x)
    assert E == pytest.approx(0.5 * V * (1 - math.cos(n * phi - phi0)), abs=1e-14)
    dEdphi = 0.5 * V * n * math.sin(n * phi - phi0)
    np.testing.assert_allclose(F[3], -dEdphi / 1.4 * np.array([-math.sin(phi), math.cos(phi), 0.0]), atol=1e-13)
    np.testing.assert_allclose(F[0], [0.0, dEdphi / 1.3, 0.0], atol=1e-13)
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-13)


# ------------------------------------------------------------------ exclusions
def _coulomb_over(x, q, pairs):
    return sum(K_E * q[i] * q[j] / np.linalg.norm(x[i] - x[j]) for i, j in pairs)


def _ring(m, r):
    a = 2 * np.pi * np.arange(m) / m
    return np.stack([r * np.cos(a), r * np.sin(a), 0.05 * np.sin(3 * a)], 1)


EXCLUSION_CASES = {
    # zig-zag chain of 7: pairs |i - j| >= 3 are at least three bonds apart
    "chain7": (np.array([[1.25 * i, 0.7 * (i % 2), 0.1 * i * i] for i in range(7)]),
               [(i, i + 1) for i in range(6)],
               [(i, j) for i in range(7) for j in range(i + 3, 7)]),
    # six-ring: only the three para pairs are three bonds apart (both ways round)
    "ring6": (_ring(6, 1.4), [(i, (i + 1) % 6) for i in range(6)], [(0, 3), (1, 4), (2, 5)]),
    # five-ring: every pair is within two bonds
    "ring5": (_ring(5, 1.2), [(i, (i + 1) % 5) for i in range(5)], []),
    # six-ring with a substituent 6 on atom 0: 6 is 1-2 to 0, 1-3 to 1 and 5, 1-4 to 2 and 4,
    # and four bonds from 3
    "ring6+1": (np.vstack([_ring(6, 1.4), [[2.8, 0.0, 0.3]]]),
                [(i, (i + 1) % 6) for i in range(6)] + [(0, 6)],
                [(0, 3), (1, 4), (2, 5), (6, 2), (6, 4), (6, 3)]),
}


@pytest.mark.parametrize("case", sorted(EXCLUSION_CASES))
def test_exclusions_are_exactly_the_one_two_and_one_three_pairs(case):
    """With only charges switched on, the field is the Coulomb sum over the non-excluded
    pairs.  The expected pair lists are written out by hand from the bond graphs."""
    x, bonds, included = EXCLUSION_CASES[case]
    n = len(x)
    q = np.random.default_rng(len(case)).normal(0.0, 0.3, n)
    E, _ = O.intra(_mol(x, bonds=bonds, q=q), x)
    assert E == pytest.approx(_coulomb_over(x, q, included), abs=1e-12)
    # the same set governs the Morse part: one included pair, Morse minimum depth at s = 0
    if included:
        i, j = included[0]
        eps = np.zeros(n); eps[i], eps[j] = 0.1, 0.2
        R = np.zeros(n); R[i] = R[j] = 0.5 * np.linalg.norm(x[i] - x[j])
        E2, _ = O.intra(_mol(x, bonds=bonds, eps=eps, R=R), x)
        assert E2 == pytest.approx(-0.02, abs=1e-13)
    # and an excluded pair set up the same way contributes nothing
    i, j = bonds[0]
    eps = np.zeros(n); eps[i], eps[j] = 0.1, 0.2
    E3, _ = O.intra(_mol(x, bonds=bonds, eps=eps, R=np.ones(n)), x)
    assert E3 == 0.0


# ------------------------------------------------------------------ FIRE update order
def _bowl_grid():
    """B-spline coefficients whose model is exactly E = 1/2 (dx^2 + 2 dy^2), d = r - r*
    (the quadratic-exactness construction: per axis b = p - h^2/6 p''), constant in z."""
    h, n = 0.25, 24
    t = np.arange(n) * h
    rs = np.array([2.61, 3.07, 2.83])
    gx = 0.5 * (t - rs[0]) ** 2 - h * h / 6 * 1.0
    gy = (t - rs[1]) ** 2 - h * h / 6 * 2.0
    B = np.zeros((3, n, n, n))
    B[2] = gx[:, None, None] + gy[None, :, None]
    spec = dict(nx=n, ny=n, nz=n, x0=0.0, y0=0.0, z0=0.0, dx=h, dy=h, dz=h)
    return B, spec, rs


def _charge():
    return _mol(np.zeros((1, 3)), q=[1.0])


# Hand-worked trajectory, N_min = 0 (so the first positive move already adapts), dt0 = 0.05,
# alpha0 = 0.1, f_inc = 1.1, f_alpha = 0.99, f_dec = 0.5, dt_max = 0.1, unit mass.
# Start d0 = (0.3, 0.2), v0 = (0.206, -0.142); F = -(dx, 2 dy).
# Move 1: F = (-0.3, -0.4), |F| = 0.5; P = -0.0618 + 0.0568 = -0.005 <= 0.  (Mixing first
#   would give P = 0.9 (-0.005) + 0.1 |v0| |F| = +0.0080 and no restart.)  Restart: dt = 0.025,
#   alpha = 0.1, v = 0; kick v = F dt = (-0.0075, -0.01); move d1 = d0 + v dt
#   = (0.2998125, 0.19975).
# Move 2: F = (-0.2998125, -0.3995), P = 0.00224859375 + 0.003995 > 0; mix with alpha = 0.1:
#   v = 0.9 v + 0.1 |v| F/|F| (|v| = 0.0125); streak 1 > N_min: dt = 0.0275, alpha = 0.099;
#   kick v += F 0.0275; move d2 = d1 + v 0.0275.
# Move 3: P > 0 again; mix with alpha = 0.099, then dt = 0.03025, alpha = 0.09801; kick; move.
# Values of moves 2 and 3 evaluated in 40-digit decimal arithmetic from these steps.
FIRE_HAND = [
    (np.array([-7.5e-3, -1.0e-2]), np.array([0.2998125, 0.19975]), 0.025, 0.1, 0),
    (np.array([-1.57451440239826761e-02, -2.09860247240561335e-02]),
     np.array([2.99379508539340478e-01, 1.99172884320088450e-01]), 0.0275, 0.099, 1),
    (np.array([-2.48030858585900592e-02, -3.30346988879069922e-02]),
     np.array([2.98629215192118103e-01, 1.98173584678729281e-01]), 0.03025, 0.09801, 2),
]


@pytest.mark.parametrize("moves", [1, 2, 3])
def test_fire_update_order_hand_worked(moves):
    B, spec, rs = _bowl_grid()
    x0 = rs + np.array([0.3, 0.2, 0.0])
    v0 = np.array([[0.206, -0.142, 0.0]])
    out = O.fire_batch(B, spec, [_charge()], [0], x0[None], moves, vel=v0, intra_on=False, f_conv=1e-9, nmin=0)
    v, d, dt, a, npos = FIRE_HAND[moves - 1]
    np.testing.assert_allclose(out["pos"][0, :2] - rs[:2], d, rtol=0, atol=1e-13)
    assert out["pos"][0, 2] == x0[2]
    np.testing.assert_allclose(out["vel"][0, :2], v, rtol=0, atol=1e-14)
    assert out["dt"][0] == pytest.approx(dt, abs=1e-16) and out["alpha"][0] == pytest.approx(a, abs=1e-16)
    assert out["npos"][0] == npos and out["steps"][0] == moves
    # the state is evaluated once more after the last move
    assert out["E"][0] == pytest.approx(0.5 * (d[0] ** 2 + 2 * d[1] ** 2), abs=1e-13)
    assert out["fnorm"][0] == pytest.approx(math.hypot(d[0], 2 * d[1]), abs=1e-13)


def test_fire_displacement_cap_hand_worked():
    """Move 1 of the trajectory above with max_disp = 2e-4: the step v dt = (-1.875e-4,
    -2.5e-4) of length 3.125e-4 is scaled to length 2e-4 along itself, (-1.2e-4, -1.6e-4);
    the velocity is not rescaled."""
    B, spec, rs = _bowl_grid()
    x0 = rs + np.array([0.3, 0.2, 0.0])
    out = O.fire_batch(B, spec, [_charge()], [0], x0[None], 1, vel=np.array([[0.206, -0.142, 0.0]]),
                       intra_on=False, f_conv=1e-9, nmin=0, max_disp=2e-4)
    np.testing.assert_allclose(out["pos"][0, :2] - rs[:2], [0.3 - 1.2e-4, 0.2 - 1.6e-4], rtol=0, atol=1e-14)
    np.testing.assert_allclose(out["vel"][0, :2], [-7.5e-3, -1.0e-2], rtol=0, atol=1e-16)


def test_fire_convergence_test_precedes_the_move():
    """A replica whose |F| is already below f_conv is flagged converged and not moved, and
    its velocity is left as it came in."""
    B, spec, rs = _bowl_grid()
    x0 = rs + np.array([1e-7, 0.0, 0.0])
    out = O.fire_batch(B, spec, [_charge()], [0], x0[None], 5, vel=np.array([[0.3, 0.1, 0.0]]), intra_on=False,
                       f_conv=1e-6)
    assert out["status"][0] & 1 and out["steps"][0] == 0
    assert np.array_equal(out["pos"][0], x0) and np.array_equal(out["vel"][0], [0.3, 0.1, 0.0])


# ------------------------------------------------------------------ FP16 storage
def test_fp16_quantize_hand_worked():
    """Per-channel scale s_c = 2^(ceil(log2 max|b_c|) - 15); each coefficient stored as the
    RNE half h of b / s_c; the Pauli channel also stores the RNE half l of b / s_c - h.
    Values worked out by hand (FP16 has 10 fraction bits, so the ulp at 1 is 2^-10)."""
    B = np.zeros((3, 4, 4, 4))
    B[0, 3, 3, 3] = B[1, 3, 3, 3] = 4.3          # ceil(log2 4.3) = 3: s = 2^-12
    B[2, 3, 3, 3] = -4.0                         # an exact power of two: ceil(log2 4) = 2, s = 2^-13
    s = 2.0 ** -12
    cases = [  # b / s, decoded Pauli / s, decoded London / s
        (1 + 2 ** -11, 1 + 2 ** -11, 1.0),                        # tie: h = 1 (even), l = 2^-11
        (1 + 3 * 2 ** -11, 1 + 3 * 2 ** -11, 1 + 2 ** -9),        # tie: h = 1 + 2^-9 (even), l = -2^-11
        (1 + 2 ** -11 + 2 ** -25, 1 + 2 ** -11, 1 + 2 ** -10),    # h = 1 + 2^-10; l = -2^-11 (1 - 2^-14 rounds to 1)
        (3.0, 3.0, 3.0),
    ]
    for k, (r, _, _) in enumerate(cases):
        B[0, 0, 0, k] = B[1, 0, 0, k] = r * s
    Bq, sc = O.fp16_quantize(B)
    assert list(sc) == [2.0 ** -12, 2.0 ** -12, 2.0 ** -13]
    for k, (_, p, l) in enumerate(cases):
        assert Bq[0, 0, 0, k] == p * s and Bq[1, 0, 0, k] == l * s, k
    assert Bq[2, 3, 3, 3] == -4.0 and Bq[0, 3, 3, 3] != 4.3   # 4.3 / 2^-12 needs more than 22 bits
    assert abs(Bq[0, 3, 3, 3] - 4.3) <= 2.0 ** -22 * 4.3 and abs(Bq[1, 3, 3, 3] - 4.3) <= 2.0 ** -11 * 4.3
    # an all-zero channel keeps scale 1
    _, sc0 = O.fp16_quantize(np.zeros((3, 4, 4, 4)))
    assert list(sc0) == [1.0, 1.0, 1.0]


# ------------------------------------------------------------------ NVE drift record
def test_nve_drift_record_follows_its_definition():
    """The drift record {E(0), E(last sample), max |E(s) - E(0)|, sum dE, sum s dE, samples}
    over the samples s = 0, k, 2k, ... <= n, recomputed from E_tot(s) = E_pot + sum m v^2 / 2
    at the states of separate runs of s steps (E_pot from the model evaluation, the kinetic
    energy in eV from amu A^2/fs^2)."""
    mol = S.mol_size(10, 2)
    nx, ny, nz = 16, 16, 40
    spec = dict(nx=nx, ny=ny, nz=nz, x0=0.0, y0=0.0, z0=1.0, dx=0.4, dy=0.4, dz=0.25)
    B = S.random_coefficients(nx, ny, nz, 5, (1e-3, 1e-2, 1e-1))
    sub = S.rocksalt_slab(1, 1)
    x0 = S.place_replicas(mol, 1, sub, 31, (3.0, 3.5))[0]
    v0 = S.mb_velocities(mol.mass, 1, 600.0, 32)[0]
    n, k = 11, 3
    rec = O.nve_batch(B, spec, [mol], [0], x0, v0, n, dt=0.5, drift_every=k)["drift"][0]
    E = {}
    for s_ in range(0, n + 1, k):
        st = O.nve_batch(B, spec, [mol], [0], x0, v0, s_, dt=0.5, drift_every=k)
        Ep = O.eval_batch(B, spec, [mol], [0], st["pos"])[1][0]
        ke = 0.5 * (mol.mass[:, None] * st["vel"] ** 2).sum() * O.AMU_A2_FS2_EV
        E[s_] = Ep + ke
    s_ = np.array(sorted(E))
    dE = np.array([E[t] - E[0] for t in s_])
    want = [E[0], E[s_[-1]], np.abs(dE).max(), dE.sum(), (s_ * dE).sum(), len(s_)]
    np.testing.assert_allclose(rec, want, rtol=1e-12, atol=1e-12)
    assert rec[5] == 4 and s_[-1] == 9


def test_fire_check_cadence_hand_worked():
    """With replica-wide decisions every second move (the paper's GPU form checks every 100
    steps), move 1 is the restart of the trajectory above and move 2 a plain kick and move
    with the unchanged dt = 0.025: F = -(d1x, 2 d1y) = (-0.2998125, -0.3995),
    v2 = v1 + F dt = (-0.0149953125, -0.0199875), d2 = d1 + v2 dt = (0.2994376171875,
    0.1992503125); alpha and the streak are untouched.  Move 3 is a full FIRE step again."""
    B, spec, rs = _bowl_grid()
    x0 = rs + np.array([0.3, 0.2, 0.0])
    v0 = np.array([[0.206, -0.142, 0.0]])
    kw = dict(vel=v0, intra_on=False, f_conv=1e-9, nmin=0, check_every=2)
    out = O.fire_batch(B, spec, [_charge()], [0], x0[None], 2, **kw)
    np.testing.assert_allclose(out["pos"][0, :2] - rs[:2], [0.2994376171875, 0.1992503125], rtol=0, atol=1e-13)
    np.testing.assert_allclose(out["vel"][0, :2], [-0.0149953125, -0.0199875], rtol=0, atol=1e-14)
    assert out["dt"][0] == 0.025 and out["alpha"][0] == 0.1 and out["npos"][0] == 0 and out["steps"][0] == 2
    # move 3 (a check): P = F.v > 0 at d2, so the streak grows and dt, alpha adapt (N_min = 0)
    out3 = O.fire_batch(B, spec, [_charge()], [0], x0[None], 3, **kw)
    assert out3["npos"][0] == 1 and out3["dt"][0] == pytest.approx(0.0275, abs=1e-16)
    assert out3["alpha"][0] == pytest.approx(0.099, abs=1e-16) and out3["steps"][0] == 3
    # cadence 1 is the plain form
    a = O.fire_batch(B, spec, [_charge()], [0], x0[None], 3, vel=v0, intra_on=False, f_conv=1e-9, nmin=0)
    b = O.fire_batch(B, spec, [_charge()], [0], x0[None], 3, vel=v0, intra_on=False, f_conv=1e-9, nmin=0,
                     check_every=1)
    assert np.array_equal(a["pos"], b["pos"])
