"""FP64 oracle for the sampling rows -- TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* pose encoding (the inverse of pose construction): torsions measured, the reference
  re-posed with them, the best rigid rotation by Horn's quaternion method;
* deduplication in discovery order, by energy and by the lattice-translated RMSD;
* the proposer MLP (4 layers, SiLU) forward and backward in FP64 on BF16-rounded weights,
  IMLE nearest-candidate selection, Adam;
* standard normals from Philox4x32-10 by Box-Muller.
"""
from __future__ import annotations

import numpy as np

from . import dihedral, philox4x32_10, pose

N_ENC = 41
DIMS = [96, 256, 256, 256, 41]


# ------------------------------------------------------------------ pose encoding
def horn_quaternion(X, Y):
    """Unit quaternion (w >= 0) of the rotation R minimising sum |R x_i - y_i|^2 for centred
    point sets X, Y (n, 3) (Horn 1987: top eigenvector of the 4x4 matrix built from S = X^T Y)."""
    S = X.T @ Y
    N = np.array([
        [S[0, 0] + S[1, 1] + S[2, 2], S[1, 2] - S[2, 1], S[2, 0] - S[0, 2], S[0, 1] - S[1, 0]],
        [S[1, 2] - S[2, 1], S[0, 0] - S[1, 1] - S[2, 2], S[0, 1] + S[1, 0], S[2, 0] + S[0, 2]],
        [S[2, 0] - S[0, 2], S[0, 1] + S[1, 0], -S[0, 0] + S[1, 1] - S[2, 2], S[1, 2] + S[2, 1]],
        [S[0, 1] - S[1, 0], S[2, 0] + S[0, 2], S[1, 2] + S[2, 1], -S[0, 0] - S[1, 1] + S[2, 2]]])
    w, V = np.linalg.eigh(N)
    q = V[:, -1]
    return q if q[0] >= 0 else -q


def quat_to_matrix(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def encode_pose(mol, x, Lx, Ly, z_top=0.0):
    """Encoding [41] of pose x (n, 3): (cos 2pi u, sin 2pi u, cos 2pi v, sin 2pi v, h,
    quaternion (w >= 0), (cos phi_k, sin phi_k) for k < 16)."""
    T = len(mol.rot_quads)
    phis = np.array([dihedral(x[q]) for q in mol.rot_quads])
    dof = np.concatenate([[0.0, 0.0, 3.0, 1.0, 0.0, 0.0, 0.0], phis])
    ref = pose(mol, dof, Lx, Ly, z_top)[0]
    X = ref - ref.mean(0)
    c = x.mean(0)
    q = horn_quaternion(X, x - c)
    u = (c[0] / Lx) % 1.0
    v = (c[1] / Ly) % 1.0
    e = np.zeros(N_ENC)
    e[:5] = [np.cos(2 * np.pi * u), np.sin(2 * np.pi * u), np.cos(2 * np.pi * v), np.sin(2 * np.pi * v),
             x[:, 2].min() - z_top]
    e[5:9] = q
    for k in range(T):
        e[9 + 2 * k] = np.cos(phis[k])
        e[10 + 2 * k] = np.sin(phis[k])
    return e


def decode_dof(e, T, hlo, hhi):
    d = np.zeros(7 + T)
    d[0] = (np.arctan2(e[1], e[0]) / (2 * np.pi)) % 1.0
    d[1] = (np.arctan2(e[3], e[2]) / (2 * np.pi)) % 1.0
    d[2] = min(max(e[4], hlo), hhi)
    q = e[5:9]
    nq = np.linalg.norm(q)
    d[3:7] = q / nq if nq > 1e-6 else [1.0, 0.0, 0.0, 0.0]
    for k in range(T):
        d[7 + k] = np.arctan2(e[10 + 2 * k], e[9 + 2 * k])
    return d


# ------------------------------------------------------------------ dedupe
def dedupe_energy(E, types, ok, tol, archive=None):
    """Discovery-order energy dedupe: returns (is_new flags, archive list of (E, type))."""
    arch = list(archive or [])
    new = np.zeros(len(E), np.int32)
    for c in range(len(E)):
        if ok is not None and not ok[c]:
            continue
        if not np.isfinite(E[c]):
            continue
        if all(not (t == types[c] and abs(e - E[c]) <= tol) for e, t in arch):
            arch.append((E[c], types[c]))
            new[c] = 1
    return new, arch


def rmsd_lattice(A, B, Lx, Ly):
    """RMSD of two minima of one molecule type (same atom order), minimised over the lateral
    lattice translations (a Lx, b Ly) of the substrate: adsorption site and orientation
    count, with no rotation fit and no atom permutation (Section "Configuration sampling on
    GPU").  The mean square over atoms equals |t - m|^2 + const with m the mean difference,
    so its minimum lies at a lattice vector within one cell of m; all lattice vectors within
    two cells of m are tried."""
    D = np.asarray(A, np.float64) - np.asarray(B, np.float64)
    m = D.mean(0)
    a = np.arange(int(np.floor(m[0] / Lx)) - 2, int(np.floor(m[0] / Lx)) + 4)
    b = np.arange(int(np.floor(m[1] / Ly)) - 2, int(np.floor(m[1] / Ly)) + 4)
    T = np.zeros((len(a), len(b), 1, 3))
    T[..., 0] = a[:, None, None] * Lx
    T[..., 1] = b[None, :, None] * Ly
    return float(np.sqrt(np.mean(np.sum((D - T) ** 2, axis=-1), axis=-1)).min())


def dedupe_rmsd(pos, types, ok, tol, Lx, Ly, archive=None):
    """Discovery-order RMSD dedupe: candidate c is new when rmsd_lattice > tol against every
    archived minimum of its type, including those accepted earlier in the batch; candidates
    with ok[c] == 0 or non-finite coordinates are never new.  pos: list of (n_c, 3) arrays.
    Returns (is_new flags, archive list of (coordinates, type))."""
    arch = list(archive or [])
    new = np.zeros(len(pos), np.int32)
    for c, x in enumerate(pos):
        if ok is not None and not ok[c]:
            continue
        if not np.isfinite(x).all():
            continue
        if all(not (t == types[c] and rmsd_lattice(x, y, Lx, Ly) <= tol) for y, t in arch):
            arch.append((np.array(x, np.float64), types[c]))
            new[c] = 1
    return new, arch


# ------------------------------------------------------------------ MLP
def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params, n_types):
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for l in range(4):
        W = p[o:o + DIMS[l + 1] * DIMS[l]].reshape(DIMS[l + 1], DIMS[l]); o += W.size
        b = p[o:o + DIMS[l + 1]]; o += DIMS[l + 1]
        out.append((W, b))
    emb = p[o:o + n_types * 32].reshape(n_types, 32)
    return out, emb


def silu(z):
    return z / (1 + np.exp(-z))


def forward(params, n_types, noise, types):
    """FP64 forward with BF16-rounded weights and embedding; returns (Y, cache)."""
    layers, emb = unpack(params, n_types)
    X = np.concatenate([noise, bf16(emb)[types]], 1)
    cache = [X]
    H = X
    for l in range(4):
        W, b = layers[l]
        Z = H @ bf16(W).T + b
        H = silu(Z) if l < 3 else Z
        cache.append((Z, H))
    return H, cache


def enc_dist(y, t, T):
    d = ((y[:5] - t[:5]) ** 2).sum()
    dp, dm = ((y[5:9] - t[5:9]) ** 2).sum(), ((y[5:9] + t[5:9]) ** 2).sum()
    d += min(dp, dm)
    d += ((y[9:9 + 2 * T] - t[9:9 + 2 * T]) ** 2).sum()
    return d, (-1.0 if dm < dp else 1.0)


def loss_and_grad(params, n_types, noise, types, target, ntors):
    """Batch mean of the masked squared distance and its gradient (flat, parameter layout)."""
    Y, cache = forward(params, n_types, noise, types)
    B = len(Y)
    dY = np.zeros_like(Y)
    L = 0.0
    for b in range(B):
        d, s = enc_dist(Y[b], target[b], ntors[b])
        L += d / B
        t = target[b].copy(); t[5:9] *= s
        m = np.zeros(N_ENC); m[:9 + 2 * ntors[b]] = 1
        dY[b] = 2.0 / B * m * (Y[b] - t)
    layers, emb = unpack(params, n_types)
    grads = [None] * 4
    dH = dY
    for l in range(3, -1, -1):
        W, b = layers[l]
        Z, H = cache[l + 1]
        Hin = cache[0] if l == 0 else cache[l][1]
        dZ = dH if l == 3 else dH * (lambda s: s * (1 + Z * (1 - s)))(1 / (1 + np.exp(-Z)))
        grads[l] = (dZ.T @ Hin, dZ.sum(0))
        dH = dZ @ bf16(W)
    gemb = np.zeros((n_types, 32))
    for b in range(B):
        gemb[types[b]] += dH[b, 64:96]
    flat = np.concatenate([np.concatenate([g[0].ravel(), g[1]]) for g in grads] + [gemb.ravel()])
    return L, flat, Y


def imle_select(cand, target, ntors):
    """cand [n][K][41]: index of the nearest candidate per row (ties: lowest k) and distances."""
    n, K = cand.shape[:2]
    best = np.zeros(n, np.int32)
    bd = np.zeros(n)
    for i in range(n):
        ds = [enc_dist(cand[i, k], target[i], ntors[i])[0] for k in range(K)]
        best[i] = int(np.argmin(ds))
        bd[i] = ds[best[i]]
    return best, bd


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    return p, m, v


def normal_philox(n, seed, rnd):
    out = np.zeros(n)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for q in range((n + 3) // 4):
        o = philox4x32_10([q & 0xFFFFFFFF, rnd, 1, q >> 32], key)
        u = [((x >> 8) + 0.5) / 16777216.0 for x in o]
        z = []
        for p in range(2):
            r = np.sqrt(-2 * np.log(u[2 * p]))
            z += [r * np.cos(2 * np.pi * u[2 * p + 1]), r * np.sin(2 * np.pi * u[2 * p + 1])]
        for k in range(4):
            if 4 * q + k < n:
                out[4 * q + k] = z[k]
    return out
