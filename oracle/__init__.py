"""FP64 CPU oracle for the GridFF hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never imports, links or
calls it, and the two share no code: the only common inputs come from
``paper_2508_15522_amd.synth`` (seeded input generation, none of the method's
arithmetic).

The C part (``gridff_oracle.c``) holds the numerics; this module is ctypes
marshalling plus small glue (grid node lists, batching of molecule types).
Parity status of every function is listed in ``PINS`` below; a function with no
independent pin is marked "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "gridff_oracle.c")

K_E = 14.3996454784       # Coulomb constant [eV A / e^2]
AMU_A2_FS2_EV = 103.6426965268

# what pins each oracle function (see tests/test_oracle_*.py)
PINS = {
    "bspline_B": "closed form at nodes, partition of unity (P1)",
    "fit_bspline": "periodic cosine closed form (P3), node residual (P4)",
    "bspline_eval": "cubic-polynomial exactness (P2), FD gradient (P5), special case vs direct (P8)",
    "morse_direct": "single-atom analytic case, FD gradient, lattice symmetry (P6)",
    "coulomb_ewald2d": "eta independence, Fourier form above slab, corrugation decay (P7)",
    "intra": "FD gradient, zero net force/torque, rigid-motion invariance (P11); closed forms of each term: "
             "Morse minimum depth and slope, half-attraction point, Coulomb pair force, cosine-harmonic "
             "angle and torsion (four (V, n, phi0) variants, IUPAC sign) with their lever-arm forces; "
             "hand-listed exclusion sets on a chain and on 5-, 6- and substituted 6-rings",
    "fire_batch": "quadratic-bowl convergence (P10); hand-worked three-move trajectory fixing the update "
                  "order (restart decided before mixing, mix then adapt, kick with the adapted dt), the "
                  "displacement cap and the convergence test before the move; restraint: held atom, "
                  "bond-length and inactive-restraint cases; check cadence: hand-worked plain kick between "
                  "checks",
    "nve_batch": "dt^2 scaling of the energy fluctuation (P9); drift record recomputed from its definition "
                 "at the states of separate runs (sampling cadence 3)",
    "fp16_quantize": "hand-worked scales and round-to-nearest-even ties, the Pauli residual half",
    "philox4x32_10": "published known-answer vectors",
    "pose": "torsion set to target, rigid-body invariants",
    "mlp": "FD gradient check (P12); one-path forward closed form; Adam constant-gradient closed form; "
           "IMLE selection brute-force cases",
    "direct_images": "Morse image sums, 2D Ewald convergence, FD gradient",
    "langevin_batch": "velocity Verlet at zero friction, exact BAOAB harmonic moments",
    "sampling.dedupe_energy": "hand-worked discovery-order cases",
    "sampling.rmsd_lattice": "lattice/continuous shift, rotation and permutation closed forms",
    "trilinear_eval": "nodal values, exactness on multilinear fields, domain rules",
    "sampling.dedupe_rmsd": "hand-worked discovery-order chain, type, NaN and carried-archive cases",
}


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", LIB, SRC, "-lm"])
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(LIB)
        _lib.orc_bspline_B.restype = C.c_double
        _lib.orc_bspline_dB.restype = C.c_double
        _lib.orc_erfcx.restype = C.c_double
        _lib.orc_dihedral.restype = C.c_double
        _lib.orc_intra.restype = C.c_double
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def set_threads(n):
    """Thread count of the oracle's OpenMP loops (n <= 0: the initial count); returns the
    previous count.  For timing only: no result depends on it."""
    return lib().orc_set_threads(C.c_int(n))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int))


def _nullable(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


# ------------------------------------------------------------------ substrate channels
def morse_direct(sub, pts, alpha=1.6, rcut=30.0):
    pts, pp = _d(pts)
    n = len(pts)
    VP, VL = np.zeros(n), np.zeros(n)
    gP, gL = np.zeros((n, 3)), np.zeros((n, 3))
    sp, spp = _d(sub.pos)
    se, sep = _d(sub.eps)
    sr, srp = _d(sub.R)
    lib().orc_morse_direct(C.c_int(sub.n), spp, sep, srp, C.c_double(sub.Lx), C.c_double(sub.Ly),
                           C.c_double(alpha), C.c_double(rcut), C.c_int(n), pp,
                           _nullable(VP), _nullable(VL), _nullable(gP), _nullable(gL))
    return VP, VL, gP, gL


def coulomb_ewald2d(sub, pts, eta=0.35, ke=K_E):
    pts, pp = _d(pts)
    n = len(pts)
    V, g = np.zeros(n), np.zeros((n, 3))
    sp, spp = _d(sub.pos)
    sq, sqp = _d(sub.q)
    lib().orc_coulomb_ewald2d(C.c_int(sub.n), spp, sqp, C.c_double(sub.Lx), C.c_double(sub.Ly),
                              C.c_double(ke), C.c_double(eta), C.c_int(n), pp, _nullable(V), _nullable(g))
    return V, g


def coulomb_fourier_above(sub, pts, ke=K_E):
    pts, pp = _d(pts)
    n = len(pts)
    V, g = np.zeros(n), np.zeros((n, 3))
    sp, spp = _d(sub.pos)
    sq, sqp = _d(sub.q)
    lib().orc_coulomb_fourier_above(C.c_int(sub.n), spp, sqp, C.c_double(sub.Lx), C.c_double(sub.Ly),
                                    C.c_double(ke), C.c_int(n), pp, _nullable(V), _nullable(g))
    return V, g


def direct_images(sub, pts, plq, alpha=1.6, ke=K_E, nimg=1):
    """All-atom molecule-substrate energy and force at points (mixing plq [n][3]) summed over
    the cell and its lateral images |a|, |b| <= nimg: (E [n], F [n][3])."""
    pts, pp = _d(pts)
    plq, qp = _d(plq)
    n = len(pts)
    E, F = np.zeros(n), np.zeros((n, 3))
    sp, spp = _d(sub.pos)
    sq, sqp = _d(sub.q)
    se, sep = _d(sub.eps)
    sr, srp = _d(sub.R)
    lib().orc_direct_images(C.c_int(sub.n), spp, sqp, sep, srp, C.c_double(sub.Lx), C.c_double(sub.Ly),
                            C.c_double(alpha), C.c_double(ke), C.c_int(nimg), C.c_int(n), pp, qp,
                            _nullable(E), _nullable(F))
    return E, F


def channels_direct(sub, pts, alpha=1.6, rcut=30.0, eta=0.35):
    """Exact V^P, V^L, V^C and gradients at points: (V[3][n], g[3][n][3])."""
    VP, VL, gP, gL = morse_direct(sub, pts, alpha, rcut)
    VC, gC = coulomb_ewald2d(sub, pts, eta)
    return np.stack([VP, VL, VC]), np.stack([gP, gL, gC])


def node_coords(spec, idx):
    """Cartesian coordinates of grid nodes idx (m,3) = (i,j,k)."""
    idx = np.asarray(idx)
    return np.stack([spec["x0"] + idx[:, 0] * spec["dx"], spec["y0"] + idx[:, 1] * spec["dy"],
                     spec["z0"] + idx[:, 2] * spec["dz"]], axis=1)


def grid_values(sub, spec, idx=None, alpha=1.6, rcut=30.0, eta=0.35):
    """Channel values V[3][...] at grid nodes (all nodes if idx is None, else the listed
    (i,j,k) nodes).  Node (i,j,k) sits at (x0 + i dx, y0 + j dy, z0 + k dz)."""
    nx, ny, nz = spec["nx"], spec["ny"], spec["nz"]
    if idx is None:
        I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        idx = np.stack([I.ravel(), J.ravel(), K.ravel()], 1)
        V, _ = channels_direct(sub, node_coords(spec, idx), alpha, rcut, eta)
        return V.reshape(3, nx, ny, nz)
    V, _ = channels_direct(sub, node_coords(spec, idx), alpha, rcut, eta)
    return V


# ------------------------------------------------------------------ B-spline
def bspline_B(t):
    return lib().orc_bspline_B(C.c_double(t))


def bspline_dB(t):
    return lib().orc_bspline_dB(C.c_double(t))


def fit_bspline(V):
    """Exact coefficients for V[..., nx, ny, nz] (leading channel axes allowed)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    nx, ny, nz = V.shape[-3:]
    flat = V.reshape(-1, nx, ny, nz)
    out = np.empty_like(flat)
    for c in range(flat.shape[0]):
        src, sp = _d(flat[c])
        dst = np.empty_like(src)
        lib().orc_fit_bspline(C.c_int(nx), C.c_int(ny), C.c_int(nz), sp,
                              dst.ctypes.data_as(C.POINTER(C.c_double)))
        out[c] = dst
    return out.reshape(V.shape)


def bspline_eval(B, spec, pos, plq, chan=False):
    """Model energy/force at points: B[3][nx][ny][nz], plq (n,3) = (P, L, Q).
    Returns E (n,), F (n,3), flags (n,) [, channel values (n,3)]."""
    B, bp = _d(B)
    pos, pp = _d(pos)
    plq, qp = _d(plq)
    n = len(pos)
    E, F, fl = np.zeros(n), np.zeros((n, 3)), np.zeros(n, np.int32)
    ch = np.zeros((n, 3)) if chan else None
    lib().orc_bspline_eval(C.c_int(spec["nx"]), C.c_int(spec["ny"]), C.c_int(spec["nz"]),
                           C.c_double(spec["x0"]), C.c_double(spec["y0"]), C.c_double(spec["z0"]),
                           C.c_double(spec["dx"]), C.c_double(spec["dy"]), C.c_double(spec["dz"]),
                           bp, C.c_int(n), pp, qp, _nullable(E), _nullable(F),
                           fl.ctypes.data_as(C.POINTER(C.c_int)), _nullable(ch))
    return (E, F, fl, ch) if chan else (E, F, fl)


def trilinear_nodes(B, spec):
    """Nodal (E, Fx, Fy, Fz) per channel of the B-spline model B: [3][nx][ny][nz][4], the
    table the trilinear scheme stores (energies and forces of the same model at the nodes)."""
    nx, ny, nz = spec["nx"], spec["ny"], spec["nz"]
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pts = np.stack([spec["x0"] + ii * spec["dx"], spec["y0"] + jj * spec["dy"], spec["z0"] + kk * spec["dz"]],
                   -1).reshape(-1, 3)
    out = np.zeros((3, nx * ny * nz, 4))
    for c in range(3):
        plq = np.zeros((len(pts), 3)); plq[:, c] = 1.0
        E, F, _ = bspline_eval(B, spec, pts, plq)
        out[c, :, 0] = E; out[c, :, 1:] = F
    return out.reshape(3, nx, ny, nz, 4)


def trilinear_eval(N, spec, pos, plq):
    """Trilinear interpolation of stored nodal (E, F) N[3][nx][ny][nz][4]: E (n,), F (n,3), flags."""
    N, np_ = _d(N)
    pos, pp = _d(pos)
    plq, qp = _d(plq)
    n = len(pos)
    E, F, fl = np.zeros(n), np.zeros((n, 3)), np.zeros(n, np.int32)
    lib().orc_trilinear_eval(C.c_int(spec["nx"]), C.c_int(spec["ny"]), C.c_int(spec["nz"]),
                             C.c_double(spec["x0"]), C.c_double(spec["y0"]), C.c_double(spec["z0"]),
                             C.c_double(spec["dx"]), C.c_double(spec["dy"]), C.c_double(spec["dz"]),
                             np_, C.c_int(n), pp, qp, _nullable(E), _nullable(F),
                             fl.ctypes.data_as(C.POINTER(C.c_int)))
    return E, F, fl


def mixing(eps, R, q, alpha=1.6):
    eps, ep = _d(eps)
    R, rp = _d(R)
    q, qp = _d(q)
    out = np.zeros((len(eps), 3))
    lib().orc_mixing(C.c_int(len(eps)), ep, rp, qp, C.c_double(alpha), _nullable(out))
    return out


def fp16_quantize(B):
    """Per-channel power-of-two scale s_c = 2^(ceil(log2 max|b_c|) - 15) and the
    round-to-nearest-even FP16 value h of b/s_c; the Pauli channel also keeps the FP16
    value l of its residual b/s_c - h, so that it is stored as h + l.  Returned decoded in
    FP64, (h [+ l]) s_c: (Bq, s)."""
    B = np.asarray(B, dtype=np.float64)
    s = np.empty(3)
    out = np.empty_like(B)
    for c in range(3):
        m = np.abs(B[c]).max()
        s[c] = 2.0 ** (int(np.ceil(np.log2(m))) - 15) if m > 0 else 1.0
        r = B[c] / s[c]
        h = r.astype(np.float16).astype(np.float64)
        if c == 0:
            h = h + (r - h).astype(np.float16).astype(np.float64)
        out[c] = h * s[c]
    return out, s


# ------------------------------------------------------------------ molecules / batches
class _Mol(C.Structure):
    _fields_ = [("n", C.c_int), ("eps", C.POINTER(C.c_double)), ("R", C.POINTER(C.c_double)),
                ("q", C.POINTER(C.c_double)),
                ("nb", C.c_int), ("bonds", C.POINTER(C.c_int)), ("bk", C.POINTER(C.c_double)),
                ("br0", C.POINTER(C.c_double)),
                ("na", C.c_int), ("angles", C.POINTER(C.c_int)), ("ak", C.POINTER(C.c_double)),
                ("acos0", C.POINTER(C.c_double)),
                ("nt", C.c_int), ("tors", C.POINTER(C.c_int)), ("tV", C.POINTER(C.c_double)),
                ("tn", C.POINTER(C.c_int)), ("tphi0", C.POINTER(C.c_double)),
                ("alpha", C.c_double), ("ke", C.c_double)]


class _Types(C.Structure):
    _fields_ = [("n_types", C.c_int), ("natoms", C.POINTER(C.c_int)), ("atom_off", C.POINTER(C.c_int)),
                ("eps", C.POINTER(C.c_double)), ("R", C.POINTER(C.c_double)), ("q", C.POINTER(C.c_double)),
                ("mass", C.POINTER(C.c_double)),
                ("bond_off", C.POINTER(C.c_int)), ("angle_off", C.POINTER(C.c_int)),
                ("tors_off", C.POINTER(C.c_int)),
                ("bonds", C.POINTER(C.c_int)), ("bk", C.POINTER(C.c_double)), ("br0", C.POINTER(C.c_double)),
                ("angles", C.POINTER(C.c_int)), ("ak", C.POINTER(C.c_double)), ("acos0", C.POINTER(C.c_double)),
                ("tors", C.POINTER(C.c_int)), ("tV", C.POINTER(C.c_double)), ("tn", C.POINTER(C.c_int)),
                ("tphi0", C.POINTER(C.c_double)),
                ("alpha", C.c_double), ("ke", C.c_double)]


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("B", C.POINTER(C.c_double)), ("N", C.POINTER(C.c_double))]


class _Fire(C.Structure):
    _fields_ = [("n_steps", C.c_int), ("dt0", C.c_double), ("f_conv", C.c_double),
                ("max_disp", C.c_double), ("finc", C.c_double), ("fdec", C.c_double),
                ("alpha0", C.c_double), ("falpha", C.c_double), ("dtmax", C.c_double),
                ("nmin", C.c_int), ("intra", C.c_int), ("check_every", C.c_int)]


class MolView:
    """Keeps numpy buffers alive behind an orc_mol struct."""

    def __init__(self, mol, alpha=1.6, ke=K_E, q=None):
        self.keep = []

        def d(a):
            a, p = _d(a)
            self.keep.append(a)
            return p

        def i(a):
            a, p = _i(a)
            self.keep.append(a)
            return p
        self.s = _Mol(mol.n, d(mol.eps), d(mol.R), d(mol.q if q is None else q),
                      len(mol.bonds), i(mol.bonds), d(mol.bond_k), d(mol.bond_r0),
                      len(mol.angles), i(mol.angles), d(mol.angle_k), d(mol.angle_cos0),
                      len(mol.tors), i(mol.tors), d(mol.tors_V), i(mol.tors_n), d(mol.tors_phi0),
                      alpha, ke)


def intra(mol, x, alpha=1.6, ke=K_E):
    """Intramolecular energy and forces of one molecule at positions x (n,3)."""
    mv = MolView(mol, alpha, ke)
    x, xp = _d(x)
    F = np.zeros((mol.n, 3))
    E = lib().orc_intra(C.byref(mv.s), xp, _nullable(F), None)
    return E, F


class TypesView:
    def __init__(self, mols, alpha=1.6, ke=K_E):
        self.keep = []
        cat = lambda key: np.concatenate([np.asarray(getattr(m, key)) for m in mols])
        natoms = np.array([m.n for m in mols], np.int32)
        off = lambda arr: np.concatenate([[0], np.cumsum([len(getattr(m, arr)) for m in mols])]).astype(np.int32)

        def d(a):
            a, p = _d(a)
            self.keep.append(a)
            return p

        def i(a):
            a, p = _i(a)
            self.keep.append(a)
            return p
        self.mols = mols
        self.s = _Types(len(mols), i(natoms), i(np.concatenate([[0], np.cumsum(natoms)])),
                        d(cat("eps")), d(cat("R")), d(cat("q")), d(cat("mass")),
                        i(off("bonds")), i(off("angles")), i(off("tors")),
                        i(np.concatenate([m.bonds.reshape(-1, 2) for m in mols])), d(cat("bond_k")), d(cat("bond_r0")),
                        i(np.concatenate([m.angles.reshape(-1, 3) for m in mols])), d(cat("angle_k")),
                        d(cat("angle_cos0")),
                        i(np.concatenate([m.tors.reshape(-1, 4) for m in mols])), d(cat("tors_V")),
                        i(cat("tors_n")), d(cat("tors_phi0")), alpha, ke)


class GridView:
    """B: B-spline coefficients [3][nx][ny][nz], or a trilinear nodal table [3][nx][ny][nz][4]
    (trilinear_nodes), which the batch functions then interpolate instead."""

    def __init__(self, B, spec):
        self.B, bp = _d(B)
        tri = self.B.ndim == 5
        self.s = _Grid(spec["nx"], spec["ny"], spec["nz"], spec["x0"], spec["y0"], spec["z0"],
                       spec["dx"], spec["dy"], spec["dz"], None if tri else bp, bp if tri else None)


def _batch_arrays(mols, rep_type):
    rep_type = np.asarray(rep_type, np.int32)
    nat = np.array([mols[t].n for t in rep_type], np.int32)
    off = np.concatenate([[0], np.cumsum(nat)]).astype(np.int32)
    return rep_type, off


def eval_batch(B, spec, mols, rep_type, pos, intra_on=True, alpha=1.6):
    """pos (n_atoms_total,3) -> F (n_atoms_total,3), E_rep, E_atom (grid part), status."""
    tv, gv = TypesView(mols, alpha), GridView(B, spec)
    rep_type, off = _batch_arrays(mols, rep_type)
    pos, pp = _d(pos)
    F = np.zeros_like(pos)
    Er, Ea = np.zeros(len(rep_type)), np.zeros(len(pos))
    st = np.zeros(len(rep_type), np.int32)
    lib().orc_eval_batch(C.byref(gv.s), C.byref(tv.s), C.c_int(int(intra_on)), C.c_int(len(rep_type)),
                         _i(rep_type)[1], _i(off)[1], pp, _nullable(F), _nullable(Er), _nullable(Ea),
                         st.ctypes.data_as(C.POINTER(C.c_int)))
    return F, Er, Ea, st


# dt_max = 0.1: the stiffest bond modes (unit masses, k = 20 eV/A^2, up to three bonds per
# atom) put the semi-implicit Euler stability limit near 0.18; larger steps keep FIRE
# resetting and it stalls
FIRE_DEFAULTS = dict(dt0=0.05, f_conv=1e-4, max_disp=0.1, finc=1.1, fdec=0.5, alpha0=0.1,
                     falpha=0.99, dtmax=0.1, nmin=5, check_every=1)


def fire_batch(B, spec, mols, rep_type, pos, n_steps, vel=None, state=None, intra_on=True,
               alpha=1.6, fixed_atom=None, fixed_pos=None, **kw):
    """FIRE relaxation; returns dict with pos, vel, dt, alpha, npos, status, E, fnorm, steps.
    fixed_atom [n_rep] (index in the molecule, -1 none) with fixed_pos [n_rep][3]: one
    restrained atom per replica."""
    p = dict(FIRE_DEFAULTS)
    p.update(kw)
    tv, gv = TypesView(mols, alpha), GridView(B, spec)
    rep_type, off = _batch_arrays(mols, rep_type)
    nr = len(rep_type)
    pos = np.array(pos, dtype=np.float64, order="C")
    vel = np.zeros_like(pos) if vel is None else np.array(vel, dtype=np.float64, order="C")
    st = state or {}
    fdt = np.array(st.get("dt", np.full(nr, p["dt0"])), np.float64)
    fal = np.array(st.get("alpha", np.full(nr, p["alpha0"])), np.float64)
    fnp = np.array(st.get("npos", np.zeros(nr)), np.int32)
    status = np.array(st.get("status", np.zeros(nr)), np.int32)
    E, fn, steps = np.zeros(nr), np.zeros(nr), np.zeros(nr, np.int32)
    prm = _Fire(n_steps, p["dt0"], p["f_conv"], p["max_disp"], p["finc"], p["fdec"], p["alpha0"],
                p["falpha"], p["dtmax"], p["nmin"], int(intra_on), p["check_every"])
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
    lib().orc_fire_batch(C.byref(gv.s), C.byref(tv.s), C.byref(prm), C.c_int(nr), _i(rep_type)[1],
                         _i(off)[1], _nullable(pos), _nullable(vel), _nullable(fdt), _nullable(fal),
                         ip(fnp), ip(status), _nullable(E), _nullable(fn), ip(steps),
                         None if fixed_atom is None else _i(fixed_atom)[1],
                         None if fixed_atom is None else _d(fixed_pos)[1])
    return dict(pos=pos, vel=vel, dt=fdt, alpha=fal, npos=fnp, status=status, E=E, fnorm=fn, steps=steps)


def nve_batch(B, spec, mols, rep_type, pos, vel, n_steps, dt=0.5, drift_every=1, intra_on=True,
              alpha=1.6, status=None):
    tv, gv = TypesView(mols, alpha), GridView(B, spec)
    rep_type, off = _batch_arrays(mols, rep_type)
    nr = len(rep_type)
    pos = np.array(pos, dtype=np.float64, order="C")
    vel = np.array(vel, dtype=np.float64, order="C")
    st = np.zeros(nr, np.int32) if status is None else np.array(status, np.int32, order="C")
    E, drift = np.zeros(nr), np.zeros((nr, 6))
    lib().orc_nve_batch(C.byref(gv.s), C.byref(tv.s), C.c_int(n_steps), C.c_double(dt),
                        C.c_int(int(intra_on)), C.c_int(drift_every), C.c_int(nr), _i(rep_type)[1],
                        _i(off)[1], _nullable(pos), _nullable(vel), st.ctypes.data_as(C.POINTER(C.c_int)),
                        _nullable(E), _nullable(drift))
    return dict(pos=pos, vel=vel, status=st, E=E, drift=drift)


def langevin_batch(B, spec, mols, rep_type, pos, vel, n_steps, dt=0.5, T=300.0, gamma=0.01, seed=0, rnd=0,
                   rep_id=None, intra_on=True, alpha=1.6, status=None):
    """BAOAB Langevin dynamics (Philox normals keyed by the replica ids rep_id)."""
    tv, gv = TypesView(mols, alpha), GridView(B, spec)
    rep_type, off = _batch_arrays(mols, rep_type)
    nr = len(rep_type)
    rid = np.arange(nr, dtype=np.int32) if rep_id is None else np.ascontiguousarray(rep_id, np.int32)
    pos = np.array(pos, dtype=np.float64, order="C")
    vel = np.array(vel, dtype=np.float64, order="C")
    st = np.zeros(nr, np.int32) if status is None else np.array(status, np.int32, order="C")
    E = np.zeros(nr)
    kT = 8.617333262e-5 * T
    lib().orc_langevin_batch(C.byref(gv.s), C.byref(tv.s), C.c_int(n_steps), C.c_double(dt), C.c_double(kT),
                             C.c_double(gamma), C.c_uint64(seed), C.c_uint32(rnd), C.c_int(int(intra_on)),
                             C.c_int(nr), _i(rep_type)[1], rid.ctypes.data_as(C.POINTER(C.c_int)), _i(off)[1],
                             _nullable(pos), _nullable(vel), st.ctypes.data_as(C.POINTER(C.c_int)), _nullable(E))
    return dict(pos=pos, vel=vel, status=st, E=E)


# ------------------------------------------------------------------ RNG / proposals
def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def propose_uniform(n_rep, T, seed, rnd, hlo=3.0, hhi=5.0):
    dof = np.zeros((n_rep, 7 + T))
    lib().orc_propose_uniform(C.c_int(n_rep), C.c_int(T), C.c_uint64(seed), C.c_uint32(rnd),
                              C.c_double(hlo), C.c_double(hhi), _nullable(dof))
    return dof


def pose(mol, dof, Lx, Ly, z_top=0.0):
    ref, rp = _d(mol.pos)
    T = len(mol.rot_quads)
    quad, qp = _i(mol.rot_quads.reshape(-1, 4) if T else np.zeros((1, 4)))
    mask = np.ascontiguousarray(mol.rot_masks.reshape(T, mol.n) if T else np.zeros((1, mol.n)), np.uint8)
    dof = np.atleast_2d(dof)
    out = np.zeros((len(dof), mol.n, 3))
    for r in range(len(dof)):
        d, dp = _d(dof[r])
        o = np.zeros((mol.n, 3))
        lib().orc_pose(C.c_int(mol.n), rp, C.c_int(T), qp, mask.ctypes.data_as(C.POINTER(C.c_ubyte)),
                       dp, C.c_double(Lx), C.c_double(Ly), C.c_double(z_top), _nullable(o))
        out[r] = o
    return out


def dihedral(p4):
    p4, pp = _d(p4)
    return lib().orc_dihedral(pp)
