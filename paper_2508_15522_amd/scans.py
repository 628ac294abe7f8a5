"""Rigid and restrained (relaxed) scans of a molecule over the substrate, batched (host
orchestration only; every numerical step is a libgridff call).

Sections "Rigid scans", "Relaxed detachment" and "Dragging" of the paper scan one molecule at
a time.  Here every scan point (rigid scans) or every path (restrained scans) is a replica:

* rigid_scan: the molecule translated rigidly by each offset; all energies from one
  evaluation launch.
* restrained_scan: n_paths paths of a held atom with n_points targets each.  At point k the
  held atom of every path is placed at its k-th target and the rest of the molecule relaxes
  with FIRE from the configuration of point k-1 (the continuation the paper's scans use),
  all paths in one launch per point.
* restrained_scan_fused: the same scans in one launch, each path advancing to its next point
  as soon as the current one is relaxed.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import device as D, gridff as G


def rigid_scan(grid, topo, mol_type, base_pos, offsets, include_intra=False, block=256):
    """Energy of the molecule (type index mol_type of topo, geometry base_pos (n,3)) at
    base_pos + offset for every offset (m,3): host float64 [m] (FP64 per-replica sums of the
    FP32 per-atom energies) and status flags [m]."""
    offsets = np.asarray(offsets, np.float64)
    m = len(offsets)
    plan = G.Plan(topo, np.full(m, mol_type, np.int32), block_threads=block)
    pos = D.soa(plan, [np.asarray(base_pos, np.float64) + o for o in offsets])
    F = torch.empty_like(pos)
    E = torch.empty(m, dtype=torch.float64, device="cuda")
    st = torch.empty(m, dtype=torch.int32, device="cuda")
    G.eval_forces(grid.desc, topo, plan, include_intra, pos, F, None, E, st)
    torch.cuda.synchronize()
    return E.cpu().numpy(), st.cpu().numpy()


def restrained_scan_fused(grid, topo, plan, start_pos, held_atom, targets, f_conv=1e-3, max_steps=5000,
                          keep_pos=False, dt0=0.05):
    """The same scan as restrained_scan in a single launch (gff_relax_scan): every replica
    advances to its next point as soon as the current one is relaxed.  Same returns, with the
    per-point energies as FP32 sums."""
    n = plan.n_rep
    targets = np.asarray(targets, np.float32)
    n_pts = targets.shape[1]
    st = D.fire_state(plan, start_pos, dt0=dt0)
    st["fixed_atom"] = torch.from_numpy(np.ascontiguousarray(held_atom, np.int32)).cuda()
    path = torch.from_numpy(np.ascontiguousarray(targets)).cuda()                      # [n_rep][n_points][3]
    E = torch.empty(n, n_pts, dtype=torch.float64, device="cuda")
    steps = torch.empty(n, n_pts, dtype=torch.int32, device="cuda")
    status = torch.empty(n, n_pts, dtype=torch.int32, device="cuda")
    pos = torch.empty(n_pts, 3, plan.n_atoms, device="cuda") if keep_pos else None
    out = D.outputs(plan)
    prm = G.relax_params(G.MODE_FIRE, 0, True, f_conv=f_conv)
    torch.cuda.synchronize()
    t0 = time.time()
    G.relax_scan(grid.desc, topo, plan, prm, st, path, n_pts, max_steps, dt0, E, steps, status, pos, out["E"],
                 out["fnorm"], out["steps"])
    torch.cuda.synchronize()
    res = dict(E=E.cpu().numpy(), steps=steps.cpu().numpy(), status=status.cpu().numpy(), seconds=time.time() - t0)
    if keep_pos:
        res["pos"] = [pos[k] for k in range(n_pts)]
    return res


def restrained_scan(grid, topo, plan, start_pos, held_atom, targets, f_conv=1e-3, max_steps=5000, keep_pos=False,
                    log=None):
    """Restrained scans of all replicas of `plan` at once.

    start_pos: per-replica (n,3) start geometries; held_atom [n_rep]: index of the held atom
    in each molecule; targets [n_rep][n_points][3]: where it is held at each point.  Each
    point relaxes with FIRE to |F|_2 < f_conv (the held atom's force excluded) in at most
    max_steps moves, from the previous point's relaxed state with FIRE restarted (zero
    velocities, dt0, alpha0).  Returns host arrays E [n_rep][n_points] (energy of the whole
    replica), steps and status [n_rep][n_points], the wall time, and with keep_pos the relaxed
    positions [n_points] of [3][N] device tensors."""
    say = log or (lambda s: None)
    n = plan.n_rep
    targets = np.asarray(targets, np.float32)
    assert targets.shape[0] == n and targets.shape[2] == 3
    n_pts = targets.shape[1]
    st = D.fire_state(plan, start_pos)
    st["fixed_atom"] = torch.from_numpy(np.ascontiguousarray(held_atom, np.int32)).cuda()
    st["fixed_pos"] = torch.empty(n, 3, device="cuda")
    tg = torch.from_numpy(np.ascontiguousarray(targets.transpose(1, 0, 2))).cuda()     # [n_points][n_rep][3]
    all1 = torch.ones(n, dtype=torch.int32, device="cuda")
    out = D.outputs(plan)
    prm = G.relax_params(G.MODE_FIRE, max_steps, True, f_conv=f_conv)
    E = torch.empty(n_pts, n, dtype=torch.float64, device="cuda")
    steps = torch.empty(n_pts, n, dtype=torch.int32, device="cuda")
    status = torch.empty(n_pts, n, dtype=torch.int32, device="cuda")
    kept = []
    torch.cuda.synchronize()
    t0 = time.time()
    for k in range(n_pts):
        st["fixed_pos"].copy_(tg[k])
        G.refill(plan, all1, st["pos"], st)                 # restart FIRE from the current positions
        G.relax_batch(grid.desc, topo, plan, prm, st, out["E"], out["fnorm"], out["steps"])
        E[k].copy_(out["E"]); steps[k].copy_(out["steps"]); status[k].copy_(st["status"])
        if keep_pos:
            kept.append(st["pos"].clone())
        if k % 50 == 0:
            say(f"scan point {k}/{n_pts}")
    torch.cuda.synchronize()
    secs = time.time() - t0
    res = dict(E=E.cpu().numpy().T, steps=steps.cpu().numpy().T, status=status.cpu().numpy().T, seconds=secs)
    if keep_pos:
        res["pos"] = kept
    return res


def detachment_targets(start_pos, held_atom, z_values):
    """Targets lifting each replica's held atom vertically from its start (x, y) through
    z_values (the relaxed detachment scan)."""
    n = len(start_pos)
    t = np.zeros((n, len(z_values), 3))
    for r in range(n):
        t[r, :, :2] = start_pos[r][held_atom[r], :2]
        t[r, :, 2] = z_values
    return t


def drag_targets(start_pos, held_atom, direction, step, n_points, height=None):
    """Targets dragging each replica's held atom along `direction` (unit vector in the xy
    plane) in steps of `step` from its start position, at its start height or `height`."""
    d = np.asarray(direction, np.float64)
    d = d / np.linalg.norm(d)
    n = len(start_pos)
    t = np.zeros((n, n_points, 3))
    for r in range(n):
        p0 = np.array(start_pos[r][held_atom[r]], np.float64)
        if height is not None:
            p0[2] = height
        t[r] = p0[None, :] + np.arange(n_points)[:, None] * step * np.array([d[0], d[1], 0.0])[None, :]
    return t
