"""Shared helpers of the GPU parity tests (inputs from the seeded generator or the
oracle only; nothing here computes the method)."""
import functools
import os

import numpy as np

import oracle as O
from paper_2508_15522_amd import synth as S

# realistic magnitudes for random coefficient grids: |P b^P|, |L b^L|, |Q b^C| ~ 0.03 eV
COEF_SCALE = (1e-3, 1e-2, 1e-1)


def drift_tolerances(eps, steps):
    """Bounds on the drift-record fields {E(0), E(last), max |dE|, sum dE, sum s dE, samples}
    that follow from a per-sample error |E_gpu(s) - E_oracle(s)| <= eps: each dE(s) =
    E(s) - E(0) is within 2 eps, so max |dE| is within 2 eps, sum dE within 2 eps per sample
    after the first and sum s dE within 2 eps sum s; the sample count is exact."""
    s = np.asarray(steps[1:], dtype=np.float64)
    return np.array([eps, eps, 2 * eps, 2 * eps * len(s), 2 * eps * s.sum(), 0.0])


# per-sample energy error of one 38-atom replica after 50 steps: FP32 evaluation at the same
# positions (64 grid terms per atom of |P b| <~ 0.05 eV, ~600 pair terms of <~ 1 eV, each
# rounded at 2^-24, give <~ 5e-5 eV) plus the energy difference of the two trajectories,
# which is second order in their 1e-5 A separation because both conserve E_tot
NVE_EPS = 1e-4


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def mixing_for(mols, rep_type):
    return np.concatenate([O.mixing(mols[t].eps, mols[t].R, mols[t].q) for t in rep_type])


@functools.lru_cache(maxsize=None)
def oracle_relax_grid():
    """A coarse physical grid built entirely by the oracle (direct Morse sums, 2D Ewald,
    exact fit), rounded to FP32: the model both sides relax on.  2x2 cells, 3 planes,
    40 x 40 x 27 nodes at ~0.28 x 0.28 x 0.25 A, z from 1.5 to 8.0 A."""
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), "gff_oracle_relax_grid_v1.npz")
    sub = S.rocksalt_slab(2, 3)
    spec = dict(nx=40, ny=40, nz=27, x0=0.0, y0=0.0, z0=1.5, dx=sub.Lx / 40, dy=sub.Ly / 40, dz=0.25)
    if os.path.exists(cache):
        B = np.load(cache)["B"]
    else:
        V = O.grid_values(sub, spec, rcut=20.0)
        B = S.f32(O.fit_bspline(V))
        tmp = cache + ".tmp.npz"
        np.savez(tmp, B=B)
        os.replace(tmp, cache)
    # geometry exactly as the FP32 descriptor will carry it
    g = {k: (float(np.float32(v)) if isinstance(v, float) else v) for k, v in spec.items()}
    return sub, g, B
