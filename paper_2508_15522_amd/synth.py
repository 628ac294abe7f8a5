"""Seeded synthetic inputs for the GridFF hot path.

This module only *generates inputs*: rock-salt slab coordinates and charges,
molecule geometries with their topology and force-field parameters, lateral
placements, Maxwell-Boltzmann velocities, random coefficient grids and random
evaluation points.  It computes none of the method's quantities (no grid
values, no B-spline weights, no energies or forces, no mixing coefficients),
so the HIP library and the FP64 oracle can both consume it without sharing any
of the method's arithmetic.

Every per-atom value that reaches the GPU in FP32 is produced here already
rounded to FP32 (and stored as float64), so both sides see identical inputs.

Units: energy eV, length Angstrom, charge e, mass amu, time fs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

# Synthetic Morse table (R in Angstrom, eps in sqrt(eV)); pair depth eps_i*eps_j
# at separation R_i + R_j (the product/sum mixing written in the paper's Morse
# factorisation, Section "Principles", Eq. E_Morse).  Values are synthetic.
MORSE_R = {"cation": 1.50, "anion": 2.00, "C": 1.90, "O": 1.75, "H": 1.45}
MORSE_EPS = {"cation": 0.05, "anion": 0.15, "C": 0.07, "O": 0.08, "H": 0.04}
MASS = {"C": 12.011, "O": 15.999, "H": 1.008, "cation": 22.990, "anion": 35.453}
ALPHA = 1.6            # Morse alpha [1/A], shared by all pairs
SLAB_A = 5.64          # rock-salt conventional lattice constant [A]
SLAB_Q = 0.7           # ionic charge magnitude [e]

SEED_MOL = 100         # molecule type k uses SEED_MOL + k
SEED_PLACE = 1000      # placements: SEED_PLACE * config + round
SEED_NVE = 7000
SEED_MLP = 9000
SEED_PHILOX = 4242

# bonded parameters (synthetic, explicit)
K_BOND = 20.0          # eV/A^2
K_ANGLE = 5.0          # eV
V_STIFF = 1.0          # eV
V_SOFT = 0.1           # eV


def f32(a):
    """Round to the nearest FP32 value, keep as float64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------- substrate
@dataclass
class Substrate:
    pos: np.ndarray          # (n,3) float64
    q: np.ndarray            # (n,)
    eps: np.ndarray          # (n,)
    R: np.ndarray            # (n,)
    kind: list               # "cation"/"anion"
    Lx: float
    Ly: float
    z_top: float
    a: float
    n_cells: int
    n_planes: int

    @property
    def n(self):
        return len(self.q)


def rocksalt_slab(n_cells: int, n_planes: int, a: float = SLAB_A, q: float = SLAB_Q,
                  vacancy: list | None = None) -> Substrate:
    """Rock-salt (001) slab: atomic plane p at z = -p*a/2 (top plane z = 0), sites
    (i*a/2, j*a/2) for 0 <= i, j < 2*n_cells, cation where i+j+p is even.
    `vacancy` is a list of (i, j, p) sites to remove."""
    h = a / 2.0
    pos, qq, kind = [], [], []
    vac = set(tuple(v) for v in (vacancy or []))
    for p in range(n_planes):
        for i in range(2 * n_cells):
            for j in range(2 * n_cells):
                if (i, j, p) in vac:
                    continue
                cat = (i + j + p) % 2 == 0
                pos.append((i * h, j * h, -p * h))
                qq.append(q if cat else -q)
                kind.append("cation" if cat else "anion")
    pos = np.array(pos, dtype=np.float64)
    return Substrate(pos=pos, q=np.array(qq), eps=np.array([MORSE_EPS[k] for k in kind]),
                     R=np.array([MORSE_R[k] for k in kind]), kind=kind,
                     Lx=n_cells * a, Ly=n_cells * a, z_top=0.0, a=a,
                     n_cells=n_cells, n_planes=n_planes)


# ----------------------------------------------------------------------------- molecules
@dataclass
class Molecule:
    name: str
    elem: list
    pos: np.ndarray                 # (n,3) reference geometry, FP32-representable
    q: np.ndarray
    eps: np.ndarray
    R: np.ndarray
    mass: np.ndarray
    bonds: np.ndarray               # (nb,2) int32
    bond_k: np.ndarray
    bond_r0: np.ndarray
    angles: np.ndarray              # (na,3) int32, middle index is the vertex
    angle_k: np.ndarray
    angle_cos0: np.ndarray
    tors: np.ndarray                # (nt,4) int32
    tors_V: np.ndarray
    tors_n: np.ndarray              # int32
    tors_phi0: np.ndarray
    # rotatable torsions used by pose construction: defining quadruple and the
    # mask of atoms on the (k) side of the rotatable (j,k) bond
    rot_quads: np.ndarray = field(default_factory=lambda: np.zeros((0, 4), np.int32))
    rot_masks: np.ndarray = field(default_factory=lambda: np.zeros((0, 0), bool))

    @property
    def n(self):
        return len(self.elem)


def _dihedral(p0, p1, p2, p3):
    # generator-side helper used only to assign reference torsion offsets
    b0, b1, b2 = p1 - p0, p2 - p1, p3 - p2
    m, nn = np.cross(b0, b1), np.cross(b1, b2)
    return np.arctan2(np.linalg.norm(b1) * np.dot(b0, nn), np.dot(m, nn))


def _place_zmat(a, b, c, r, theta, phi):
    """Position of atom d with |cd| = r, angle bcd = theta, dihedral abcd = phi."""
    bc = c - b
    bc /= np.linalg.norm(bc)
    nrm = np.cross(b - a, bc)
    nn = np.linalg.norm(nrm)
    if nn < 1e-8:
        tmp = np.array([0.0, 0.0, 1.0]) if abs(bc[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
        nrm = np.cross(tmp, bc)
        nn = np.linalg.norm(nrm)
    nrm /= nn
    m = np.cross(nrm, bc)
    d2 = np.array([-r * np.cos(theta), r * np.sin(theta) * np.cos(phi), r * np.sin(theta) * np.sin(phi)])
    return c + d2[0] * bc + d2[1] * m + d2[2] * nrm


def _topology(n, bonds):
    adj = [set() for _ in range(n)]
    for i, j in bonds:
        adj[i].add(j)
        adj[j].add(i)
    angles = []
    for j in range(n):
        nb = sorted(adj[j])
        for x in range(len(nb)):
            for y in range(x + 1, len(nb)):
                angles.append((nb[x], j, nb[y]))
    tors = []
    for j, k in bonds:
        for i in sorted(adj[j] - {k}):
            for l in sorted(adj[k] - {j}):
                if i != l:
                    tors.append((i, j, k, l))
    return adj, angles, tors


def _side_mask(n, adj, j, k):
    """Atoms reachable from k without crossing the j-k bond."""
    seen = {k}
    st = [k]
    while st:
        a = st.pop()
        for b in adj[a]:
            if (a == k and b == j) or b in seen:
                continue
            seen.add(b)
            st.append(b)
    m = np.zeros(n, bool)
    m[list(seen)] = True
    return m


def _finish(name, elem, pos, bonds, soft_bonds, soft_n, rng, planar_n2=False):
    """Assign parameters from the reference geometry: r0/cos0 from the geometry,
    stiff torsions keep the reference dihedral as their minimum, soft torsions
    (around `soft_bonds`) get V_SOFT with multiplicity soft_n."""
    n = len(elem)
    pos = f32(pos - pos.mean(0))
    bonds = np.array(sorted(tuple(sorted(b)) for b in bonds), dtype=np.int32)
    adj, angles, tors = _topology(n, [tuple(b) for b in bonds])
    r0 = np.array([np.linalg.norm(pos[i] - pos[j]) for i, j in bonds])
    cos0 = []
    for i, j, k in angles:
        a, b = pos[i] - pos[j], pos[k] - pos[j]
        cos0.append(np.dot(a, b) / np.linalg.norm(a) / np.linalg.norm(b))
    soft = set(tuple(sorted(b)) for b in soft_bonds)
    tV, tn, tphi = [], [], []
    for (i, j, k, l) in tors:
        phi = _dihedral(pos[i], pos[j], pos[k], pos[l])
        if tuple(sorted((j, k))) in soft:
            tV.append(V_SOFT)
            tn.append(soft_n)
            # soft multiplicity-3 wells at the staggered angles, multiplicity-2 wells in plane
            tphi.append(np.pi if soft_n == 3 else 0.0)
        elif planar_n2:
            tV.append(V_STIFF); tn.append(2); tphi.append(0.0)
        else:
            tV.append(V_STIFF); tn.append(1); tphi.append(phi)
    q = rng.normal(0.0, 0.2, n)
    q = q - q.mean()
    rq, rm = [], []
    for (j, k) in sorted(soft):
        quad = next(t for t in tors if (t[1], t[2]) in ((j, k), (k, j)))
        rq.append(quad)
        rm.append(_side_mask(n, adj, quad[1], quad[2]))
    return Molecule(
        name=name, elem=list(elem), pos=pos, q=f32(q),
        eps=f32([MORSE_EPS[e] for e in elem]), R=f32([MORSE_R[e] for e in elem]),
        mass=f32([MASS[e] for e in elem]),
        bonds=bonds, bond_k=f32(np.full(len(bonds), K_BOND)), bond_r0=f32(r0),
        angles=np.array(angles, np.int32).reshape(-1, 3),
        angle_k=f32(np.full(len(angles), K_ANGLE)), angle_cos0=f32(cos0),
        tors=np.array(tors, np.int32).reshape(-1, 4), tors_V=f32(tV),
        tors_n=np.array(tn, np.int32), tors_phi0=f32(tphi),
        rot_quads=np.array(rq, np.int32).reshape(-1, 4),
        rot_masks=np.array(rm, bool).reshape(len(rq), n))


def mol_chain(n: int, seed: int, n_soft: int, name: str, branched: bool) -> Molecule:
    """Zig-zag sp3 chain (all trans) with bonds 1.4 +- 0.05 A, angle 109.5 deg.
    If `branched`, the backbone holds about 60 % of the atoms and the rest are
    single-atom side branches on consecutive interior backbone atoms, on
    alternating sides (tetrahedral positions)."""
    rng = np.random.default_rng(seed)
    th = np.deg2rad(109.5)
    nb_main = int(np.ceil(0.6 * n)) if branched else n
    assert n - nb_main <= nb_main - 2
    pos = []
    for k in range(nb_main):
        r = rng.normal(1.4, 0.05)
        if k == 0:
            pos.append(np.zeros(3))
        elif k == 1:
            pos.append(np.array([r, 0.0, 0.0]))
        elif k == 2:
            pos.append(pos[1] + r * np.array([-np.cos(th), np.sin(th), 0.0]))
        else:
            pos.append(_place_zmat(pos[k - 3], pos[k - 2], pos[k - 1], r, th, np.pi))
    bonds = [(k - 1, k) for k in range(1, nb_main)]
    side = 1.0
    for k in range(1, 1 + n - nb_main):
        r = rng.normal(1.4, 0.05)
        pos.append(_place_zmat(pos[k + 1], pos[k - 1], pos[k], r, th, side * 2 * np.pi / 3))
        bonds.append((k, len(pos) - 1))
        side = -side
    pos = np.array(pos)
    d = np.linalg.norm(pos[:, None] - pos[None], axis=-1)
    np.fill_diagonal(d, 9.0)
    assert d.min() > 1.2, (name, d.min())
    deg = np.zeros(n, int)
    for i, j in bonds:
        deg[i] += 1
        deg[j] += 1
    elem = []
    for i in range(n):
        u = rng.random()
        if deg[i] == 1 and u < 0.4:
            elem.append("H")
        elif u < 0.8:
            elem.append("C")
        else:
            elem.append("O")
    interior = [b for b in bonds if deg[b[0]] >= 2 and deg[b[1]] >= 2]
    pick = rng.choice(len(interior), size=min(n_soft, len(interior)), replace=False)
    soft = [interior[i] for i in sorted(pick)]
    return _finish(name, elem, pos, bonds, soft, 3, rng)


_HEX_B = 1.42
_A1 = np.array([1.5 * _HEX_B, np.sqrt(3) / 2 * _HEX_B])
_A2 = np.array([1.5 * _HEX_B, -np.sqrt(3) / 2 * _HEX_B])
_NBR = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, -1), (-1, 1)]
# a 6-ring honeycomb patch with 24 C and 14 two-coordinated rim atoms (C24 core of
# the same size as the paper's 38-atom planar adsorbate)
_PAH24 = [(0, 0), (-1, 0), (-2, 0), (-2, -1), (-3, 0), (-3, -1)]


def _hex_patch(centers):
    pts = []
    for (i, j) in centers:
        c = i * _A1 + j * _A2
        for k in range(6):
            v = c + _HEX_B * np.array([np.cos(np.pi / 3 * k), np.sin(np.pi / 3 * k)])
            if not any(np.linalg.norm(v - p) < 0.1 for p in pts):
                pts.append(v)
    return np.array(pts)


def _compact_centers(h):
    cent = [(0, 0)]
    while len(cent) < h:
        cand = set()
        for (i, j) in cent:
            for di, dj in _NBR:
                c = (i + di, j + dj)
                if c not in cent:
                    cand.add(c)
        best = None
        for c in sorted(cand):
            k = sum(((c[0] + di, c[1] + dj) in cent) for di, dj in _NBR)
            r = np.hypot(*(c[0] * _A1 + c[1] * _A2))
            key = (-k, round(r, 6), c)
            if best is None or key < best[0]:
                best = (key, c)
        cent.append(best[1])
    return cent


def mol_pah(name: str, centers, n_total: int, n_O: int, n_OH: int, seed: int) -> Molecule:
    """Planar fused-hexagon carbon patch; two-coordinated rim carbons carry H
    (1.09 A), carbonyl O (1.23 A) or a hydroxyl O-H (1.36 A, 0.97 A, soft
    torsion about C-O).  Bonds are pairs closer than 1.6 A."""
    rng = np.random.default_rng(seed)
    c2 = _hex_patch(centers)
    nC = len(c2)
    d = np.linalg.norm(c2[:, None] - c2[None], axis=-1)
    cc = (d < 1.6) & (d > 0.1)
    rim = np.where(cc.sum(1) == 2)[0]
    n_sub_sites = n_total - nC - n_OH
    assert 0 <= n_sub_sites <= len(rim), (name, nC, len(rim), n_total, n_OH)
    order = rng.permutation(rim)[:n_sub_sites]
    n_O = min(n_O, n_sub_sites - n_OH)
    kinds = (["OH"] * n_OH + ["O"] * n_O)
    kinds += ["H"] * (n_sub_sites - len(kinds))
    kinds = [kinds[i] for i in rng.permutation(len(kinds))]
    pos = [np.array([p[0], p[1], 0.0]) for p in c2]
    elem = ["C"] * nC
    bonds = [(i, j) for i in range(nC) for j in range(i + 1, nC) if cc[i, j]]
    soft = []
    for site, kd in zip(order, kinds):
        nbrs = np.where(cc[site])[0]
        out = 2 * c2[site] - c2[nbrs].sum(0)
        out = out / np.linalg.norm(out)
        base = np.array([c2[site][0], c2[site][1], 0.0])
        o3 = np.array([out[0], out[1], 0.0])
        if kd == "H":
            pos.append(base + 1.09 * o3); elem.append("H")
            bonds.append((site, len(pos) - 1))
        elif kd == "O":
            pos.append(base + 1.23 * o3); elem.append("O")
            bonds.append((site, len(pos) - 1))
        else:
            po = base + 1.36 * o3
            pos.append(po); elem.append("O")
            io = len(pos) - 1
            bonds.append((site, io))
            hpos = _place_zmat(np.array([*c2[nbrs[0]], 0.0]), base, po, 0.97, np.deg2rad(109.5), np.pi)
            pos.append(hpos); elem.append("H")
            bonds.append((io, len(pos) - 1))
            soft.append((site, io))
    return _finish(name, elem, np.array(pos), bonds, soft, 2, rng, planar_n2=True)


def mol_chain24(k: int = 0) -> Molecule:
    """M-chain24: linear 24-atom chain, 3 soft torsions (config 1's molecule)."""
    return mol_chain(24, SEED_MOL + k, 3, "chain24", branched=False)


def mol_pah38(k: int = 0) -> Molecule:
    """M-pah38: planar C24 patch with 6 O and 8 H on the rim (38 atoms, rigid)."""
    return mol_pah("pah38", _PAH24, 38, 6, 0, SEED_MOL + k)


SIZE_SERIES = (10, 18, 24, 38, 52, 70, 96, 120)


def mol_size(n: int, k: int) -> Molecule:
    """M-size{n}: branched chains below 38 atoms, fused-ring patches from 38 up,
    with about 10 % of the bonds carrying soft torsions."""
    if n < 38:
        return mol_chain(n, SEED_MOL + k, max(1, round(0.1 * n)), f"size{n}", branched=True)
    n_oh_target = max(1, round(0.1 * n))
    best = None
    for h in range(2, 40):
        c2 = _hex_patch(_compact_centers(h))
        nC = len(c2)
        d = np.linalg.norm(c2[:, None] - c2[None], axis=-1)
        nrim = int((((d < 1.6) & (d > 0.1)).sum(1) == 2).sum())
        for n_oh in range(0, nrim + 1):
            sites = n - nC - n_oh
            if 0 <= sites <= nrim and n_oh <= sites:
                key = (abs(n_oh - n_oh_target), -nC)
                if best is None or key < best[0]:
                    best = (key, h, n_oh)
    _, h, n_oh = best
    return mol_pah(f"size{n}", _compact_centers(h), n, max(0, round(0.15 * n) - n_oh), n_oh, SEED_MOL + k)


def molecule_types(kind: str):
    if kind == "chain24":
        return [mol_chain24(0)]
    if kind == "pah38":
        return [mol_pah38(1)]
    if kind == "sizes":
        return [mol_size(n, 2 + i) for i, n in enumerate(SIZE_SERIES)]
    raise ValueError(kind)


# ----------------------------------------------------------------------------- placements
def random_rotations(n: int, rng) -> np.ndarray:
    """Haar-uniform rotation matrices from the QR factorisation of Gaussian matrices."""
    g = rng.normal(size=(n, 3, 3))
    qm, rm = np.linalg.qr(g)
    s = np.sign(np.diagonal(rm, axis1=1, axis2=2))
    qm = qm * s[:, None, :]
    det = np.linalg.det(qm)
    qm[:, :, 2] *= det[:, None]
    return qm


def place_replicas(mol: Molecule, n_rep: int, sub: Substrate, seed: int,
                   h_range=(3.0, 5.0)) -> np.ndarray:
    """Replica start geometries: the reference geometry, randomly rotated, lateral
    centroid uniform over the cell, lowest atom at z_top + U[h_range].
    Returns (n_rep, n, 3) FP32-representable float64."""
    rng = np.random.default_rng(seed)
    rot = random_rotations(n_rep, rng)
    out = np.einsum("rij,nj->rni", rot, mol.pos)
    out -= out.mean(1, keepdims=True)
    lat = rng.random((n_rep, 2)) * np.array([sub.Lx, sub.Ly])
    h = rng.uniform(h_range[0], h_range[1], n_rep)
    out[:, :, 0] += lat[:, 0:1]
    out[:, :, 1] += lat[:, 1:2]
    out[:, :, 2] += (sub.z_top + h - out[:, :, 2].min(1))[:, None]
    return f32(out)


def mb_velocities(mass: np.ndarray, n_rep: int, T: float, seed: int) -> np.ndarray:
    """Maxwell-Boltzmann velocities [A/fs] at temperature T [K]; (n_rep, n, 3)."""
    rng = np.random.default_rng(seed)
    kT = 8.617333262e-5 * T                # eV
    sig = np.sqrt(kT / (mass * 103.6426965))  # 1 amu A^2/fs^2 = 103.64 eV
    return f32(rng.normal(size=(n_rep, len(mass), 3)) * sig[None, :, None])


def random_points(n: int, Lx: float, Ly: float, z_lo: float, z_hi: float, seed: int,
                  lateral_span: float = 1.0) -> np.ndarray:
    """Random evaluation points: x,y uniform over `lateral_span` cells (may exceed
    one period to exercise the wrap), z uniform in [z_lo, z_hi]."""
    rng = np.random.default_rng(seed)
    p = np.empty((n, 3))
    p[:, 0] = (rng.random(n) * lateral_span - 0.5 * (lateral_span - 1)) * Lx
    p[:, 1] = (rng.random(n) * lateral_span - 0.5 * (lateral_span - 1)) * Ly
    p[:, 2] = rng.uniform(z_lo, z_hi, n)
    return f32(p)


def random_coefficients(nx: int, ny: int, nz: int, seed: int, scale=(1.0, 1.0, 1.0)) -> np.ndarray:
    """FP32-representable random B-spline coefficients, layout [3][nx][ny][nz]."""
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((3, nx, ny, nz)) * np.asarray(scale)[:, None, None, None]
    return f32(b)


def mlp_init_params(n_types: int, seed: int = SEED_MLP) -> np.ndarray:
    """Initial proposer parameters (flat FP32, layout of the library's MLP): weights
    U(-1/sqrt(fan_in), 1/sqrt(fan_in)), zero biases, N(0, 1) type embeddings."""
    rng = np.random.default_rng(seed)
    dims = [96, 256, 256, 256, 41]
    parts = []
    for l in range(4):
        a = 1.0 / np.sqrt(dims[l])
        parts.append(rng.uniform(-a, a, (dims[l + 1], dims[l])).ravel())
        parts.append(np.zeros(dims[l + 1]))
    parts.append(rng.normal(size=(n_types, 32)).ravel())
    return np.concatenate(parts).astype(np.float32)


def mlp_noise(n: int, seed: int) -> np.ndarray:
    """Standard-normal noise rows [n][64] (FP32-representable)."""
    return f32(np.random.default_rng(seed).normal(size=(n, 64)))
