"""The allocation-free RMSD dedupe (static device scratch) against the workspace entry point:
two calls in a row, the second with fewer candidates, each on its own archive, compared bit
for bit (new-minimum flags, archive count, entries, centroids and types); the size limit is
refused before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_2508_15522_amd import device as D, gridff as G, synth as S
from tests.gpu_common import announce

pytestmark = pytest.mark.gpu


def _candidates(mols, n, seed, Lx, Ly):
    """Relaxed-looking candidates: a few base poses per type with small shifts, lattice
    translations and rotations, so that both new and repeated minima occur."""
    rng = np.random.default_rng(seed)
    types = rng.integers(0, len(mols), n).astype(np.int32)
    base = {t: [S.f32(S.place_replicas(mols[t], 1, S.rocksalt_slab(2, 3), seed * 10 + t * 3 + k)[0])
                for k in range(3)] for t in range(len(mols))}
    pos = []
    for t in types:
        x = base[t][rng.integers(0, 3)].copy()
        kind = rng.integers(0, 3)
        if kind == 1:
            x[:, 0] += 0.02                         # within tolerance: the same minimum
        elif kind == 2:
            x[:, 2] += 0.5                          # a different minimum
        x[:, :2] += [rng.integers(-1, 2) * Lx, rng.integers(-1, 2) * Ly]
        pos.append(S.f32(x))
    return types, pos


def _archive(cap, max_atoms):
    return dict(pos=torch.zeros(cap, max_atoms, 3, device="cuda"),
                cen=torch.zeros(cap, 3, dtype=torch.float64, device="cuda"),
                type=torch.zeros(cap, dtype=torch.int32, device="cuda"),
                n=torch.zeros(1, dtype=torch.int32, device="cuda"))


def test_noalloc_dedupe_equals_workspace_dedupe():
    D.require_gpu()
    mols = [S.mol_chain24(), S.mol_pah38()]
    topo = G.Topology(mols)
    Lx = Ly = 2 * S.SLAB_A
    cap, max_atoms = 5000, 38
    A, B = _archive(cap, max_atoms), _archive(cap, max_atoms)
    for call, (n, seed) in enumerate(((3000, 41), (700, 42))):
        announce(f"no-alloc dedupe call {call}: {n} candidates")
        types, pos = _candidates(mols, n, seed, Lx, Ly)
        plan = G.Plan(topo, types)
        dpos = D.soa(plan, pos)
        ok = torch.from_numpy((np.random.default_rng(seed).random(n) < 0.9).astype(np.int32)).cuda()
        new_a = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        new_b = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        G.dedupe_rmsd(plan, dpos, ok, 0.1, Lx, Ly, cap, max_atoms, A["pos"], A["cen"], A["type"], A["n"], new_a)
        G.dedupe_rmsd_noalloc(plan, dpos, ok, 0.1, Lx, Ly, cap, max_atoms, B["pos"], B["cen"], B["type"], B["n"],
                              new_b)
        torch.cuda.synchronize()
        announce(f"  new minima {int(new_a.sum())} / {int(new_b.sum())}, archive {A['n'].item()} / {B['n'].item()}")
        assert torch.equal(new_a, new_b)
        assert int(new_a.sum()) > 0 and int(new_a.sum()) < n
        for k in ("n", "pos", "cen", "type"):
            assert torch.equal(A[k], B[k]), k


def test_noalloc_dedupe_refuses_more_than_its_scratch():
    D.require_gpu()
    topo = G.Topology([S.mol_size(10, 1)])
    n = G.DEDUPE_NOALLOC_MAX_REP + 1
    plan = G.Plan(topo, np.zeros(n, np.int32))
    arch = _archive(4, 10)
    isn = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    dpos = torch.zeros(3, plan.n_atoms, device="cuda")
    with pytest.raises(G.GffError, match="workspace"):
        G.dedupe_rmsd_noalloc(plan, dpos, None, 0.1, 11.28, 11.28, 4, 10, arch["pos"], arch["cen"], arch["type"],
                              arch["n"], isn)
    torch.cuda.synchronize()
    assert (isn == 7).all() and arch["n"].item() == 0     # nothing was enqueued
