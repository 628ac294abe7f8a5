"""Device-buffer helpers around the C ABI (torch tensors for memory, nothing else).

Every numerical step runs inside libgridff; these helpers only allocate tensors,
copy inputs to the device and fill the argument structs.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gridff as G


def require_gpu():
    if not torch.cuda.is_available():
        raise G.GffError("no ROCm GPU visible: the GridFF path runs only on the GPU")
    G.lib()


def spec_for(cfg, Lx=None, Ly=None):
    return G.grid_spec(cfg.nx, cfg.ny, cfg.nz, 0.0, 0.0, cfg.z0, cfg.dz, cfg.alpha, cfg.rcut)


class DeviceGrid:
    """A packed grid on the device plus its descriptor."""

    def __init__(self, spec, storage, Lx, Ly, coef, scale, V=None, B=None):
        self.spec, self.storage, self.Lx, self.Ly = spec, storage, Lx, Ly
        self.coef, self.scale, self.V, self.B = coef, scale, V, B
        self.desc = G.grid(spec, storage, coef, scale, Lx, Ly)

    @property
    def geometry(self):
        """Geometry as the FP32 values the kernels use, promoted to float64."""
        d = self.desc
        f = lambda v: float(np.float32(v))
        return dict(nx=d.nx, ny=d.ny, nz=d.nz, x0=f(d.x0), y0=f(d.y0), z0=f(d.z0), dx=f(d.dx), dy=f(d.dy),
                    dz=f(d.dz))


def pack_from_coefficients(B, spec, storage, Lx, Ly, stream=None):
    """Upload FP64 coefficients B[3][nx][ny][nz] and pack them on the GPU."""
    dev = torch.device("cuda")
    dB = torch.from_numpy(np.ascontiguousarray(B, dtype=np.float64)).to(dev)
    nbytes = G.grid_bytes(spec, storage)
    coef = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    scale = torch.empty(4, dtype=torch.float32, device=dev)
    G.pack_grid(spec, dB, storage, coef, scale, stream)
    return DeviceGrid(spec, storage, Lx, Ly, coef, scale, B=dB)


def build_physical_grid(sub, spec, storage=G.STORE_F32, keep_fp64=False, stream=None):
    """Substrate -> V (FP64 build) -> B (FP64 exact fit) -> packed grid, all on the GPU."""
    dev = torch.device("cuda")
    n = spec.nx * spec.ny * spec.nz
    V = torch.empty(3 * n, dtype=torch.float64, device=dev)
    wb = G.build_grid_workspace_bytes(spec, sub)
    work = torch.empty(max(wb, 1), dtype=torch.uint8, device=dev)
    G.build_grid(sub, spec, V, work, stream)
    del work
    B = torch.empty_like(V)
    fw = torch.empty(max(G.fit_workspace_bytes(spec), 1), dtype=torch.uint8, device=dev)
    G.fit_bspline(spec, V, B, fw, stream)
    coef = torch.empty(G.grid_bytes(spec, storage), dtype=torch.uint8, device=dev)
    scale = torch.empty(4, dtype=torch.float32, device=dev)
    G.pack_grid(spec, B, storage, coef, scale, stream)
    if not keep_fp64:
        V = B = None
    return DeviceGrid(spec, storage, sub.Lx, sub.Ly, coef, scale, V=V, B=B)


def soa(plan, per_rep):
    """list/array of per-replica (n,3) arrays in replica order -> float32 [3][N] tensor."""
    N = plan.n_atoms
    out = np.zeros((3, N), np.float32)
    for r, x in enumerate(per_rep):
        a, b = plan.atom_off[r], plan.atom_off[r + 1]
        out[:, a:b] = np.asarray(x, np.float32).T
    return torch.from_numpy(out).cuda()


def unsoa(plan, t):
    a = t.detach().cpu().numpy().astype(np.float64)
    return [np.ascontiguousarray(a[:, plan.atom_off[r]:plan.atom_off[r + 1]].T) for r in range(plan.n_rep)]


def fire_state(plan, pos_per_rep, dt0=0.05, alpha0=0.1, vel_per_rep=None):
    dev = torch.device("cuda")
    st = dict(pos=soa(plan, pos_per_rep),
              vel=soa(plan, vel_per_rep) if vel_per_rep is not None else torch.zeros(3, plan.n_atoms, device=dev),
              fire_dt=torch.full((plan.n_rep,), dt0, dtype=torch.float32, device=dev),
              fire_alpha=torch.full((plan.n_rep,), alpha0, dtype=torch.float32, device=dev),
              fire_npos=torch.zeros(plan.n_rep, dtype=torch.int32, device=dev),
              status=torch.zeros(plan.n_rep, dtype=torch.int32, device=dev))
    return st


def outputs(plan):
    dev = torch.device("cuda")
    return dict(E=torch.zeros(plan.n_rep, dtype=torch.float64, device=dev),
                fnorm=torch.zeros(plan.n_rep, dtype=torch.float32, device=dev),
                steps=torch.zeros(plan.n_rep, dtype=torch.int32, device=dev),
                drift=torch.zeros(plan.n_rep, 6, dtype=torch.float64, device=dev))
