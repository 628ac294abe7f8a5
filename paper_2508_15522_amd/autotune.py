"""Autotuned launch shapes, cached in JSON.

The measurement itself is libgridff's gff_autotune; this module only keys and stores the
result (per device name, mode, storage and the batch's per-type replica counts)."""
from __future__ import annotations

import json
import os

import numpy as np

from . import gridff as G


def cache_path():
    return os.environ.get("GRIDFF_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gridff", "autotune.json"))


def _key(topo, rep_type, params, storage):
    import torch
    counts = np.bincount(np.asarray(rep_type), minlength=len(topo.mols))
    sizes = [m.n for m in topo.mols]
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    return json.dumps([dev, int(params.mode), int(storage), sizes, counts.tolist(), int(params.n_steps)])


def launch_for(grid, topo, rep_type, params, st, use_cache=True):
    """(block_threads, reps_per_block, grid_blocks, lanes_per_atom) for this batch, measured
    once per key."""
    path = cache_path()
    key = _key(topo, rep_type, params, grid.storage)
    db = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
    if key in db and "lanes_per_atom" in db[key]:
        v = db[key]
        return (v["block_threads"], v["reps_per_block"], v["grid_blocks"], v["lanes_per_atom"]), v["rate"]
    best, rate = G.autotune(grid.desc, topo, rep_type, params, st)
    v = dict(block_threads=best.block_threads, reps_per_block=best.reps_per_block, grid_blocks=best.grid_blocks,
             lanes_per_atom=best.lanes_per_atom, rate=rate)
    if use_cache:
        db[key] = v
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, path)
    return (v["block_threads"], v["reps_per_block"], v["grid_blocks"], v["lanes_per_atom"]), rate
