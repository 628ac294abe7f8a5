"""GPU tests of the graph-captured relaxation launch and the autotuner."""
import numpy as np
import pytest
import torch

from paper_2508_15522_amd import device as D, gridff as G, synth as S
from tests.gpu_common import announce, oracle_relax_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def world():
    D.require_gpu()
    sub, geo, B = oracle_relax_grid()
    spec = G.grid_spec(geo["nx"], geo["ny"], geo["nz"], 0.0, 0.0, geo["z0"], geo["dz"])
    grid = D.pack_from_coefficients(B, spec, G.STORE_F32, sub.Lx, sub.Ly)
    mols = S.molecule_types("sizes") + [S.mol_chain24(), S.mol_pah38()]
    return dict(sub=sub, grid=grid, mols=mols, topo=G.Topology(mols))


def _state(w, plan, rep_type, seed):
    pos = [S.place_replicas(w["mols"][t], 1, w["sub"], seed + r, (2.8, 4.0))[0] for r, t in enumerate(rep_type)]
    return D.fire_state(plan, pos)


def test_graph_replays_equal_eager_launches(world):
    w = world
    announce("graph replay")
    rep_type = np.repeat(np.arange(len(w["mols"])), 5)
    plan = G.Plan(w["topo"], rep_type, block_threads=256)
    prm = G.relax_params(G.MODE_FIRE, 40, True, f_conv=1e-4)
    st_e = _state(w, plan, rep_type, 300)
    st_g = {k: v.clone() for k, v in st_e.items()}
    out_e, out_g = D.outputs(plan), D.outputs(plan)
    graph = G.RelaxGraph(w["grid"].desc, w["topo"], plan, prm, st_g, out_g["E"], out_g["fnorm"], out_g["steps"])
    for rep in range(4):
        G.relax_batch(w["grid"].desc, w["topo"], plan, prm, st_e, out_e["E"], out_e["fnorm"], out_e["steps"])
        graph.launch()
        junk = torch.randn(1 << 20, device="cuda").sum()     # eager work between replays
        torch.cuda.synchronize()
        for k in st_e:
            assert torch.equal(st_e[k], st_g[k]), (rep, k)
        assert torch.equal(out_e["E"], out_g["E"]), rep
        del junk


def test_autotune_choice_is_launchable_and_result_invariant(world):
    w = world
    announce("autotune")
    rng = np.random.default_rng(4)
    rep_type = rng.integers(0, len(w["mols"]), 600)
    prm = G.relax_params(G.MODE_FIRE, 20, True, f_conv=1e-4)
    plan0 = G.Plan(w["topo"], rep_type, block_threads=256)
    st0 = _state(w, plan0, rep_type, 700)
    ref = {k: v.clone() for k, v in st0.items()}
    best, rate = G.autotune(w["grid"].desc, w["topo"], rep_type, prm, st0)
    announce(f"  best block {best.block_threads}, replicas per block {best.reps_per_block}, grid {best.grid_blocks}: "
             f"{rate:.3e} replica-steps/s")
    assert rate > 0 and best.block_threads % 64 == 0
    for k in st0:                                   # the caller's state is untouched
        assert torch.equal(st0[k], ref[k])
    plan1 = G.Plan(w["topo"], rep_type, best.block_threads, best.reps_per_block, best.grid_blocks)
    outs = []
    for plan in (plan0, plan1):
        st = {k: v.clone() for k, v in ref.items()}
        o = D.outputs(plan)
        G.relax_batch(w["grid"].desc, w["topo"], plan, prm, st, o["E"], o["fnorm"], o["steps"])
        torch.cuda.synchronize()
        outs.append((st["pos"].clone(), o["E"].clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
