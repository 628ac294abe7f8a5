"""Parity at the workloads' full sizes, in the launch shapes the benchmark times.

The replica kernel runs every replica of a workload (16 384 x 38 atoms NVE and Langevin
on the 112 x 112 x 150 grid in 192-thread blocks; 65 536 x 38 atoms FIRE on the 452 x 452 x 200
grid in 192-thread blocks; 4096 replicas of eight sizes FIRE with the autotuned launch), on
seeded random coefficients of the workload's
grid size; a sample of replicas is then re-run one by one by the FP64 oracle on the same
FP32-rounded coefficients and inputs.  Tolerances as in the short-run parity tests: FP32
trajectories within 2e-4 A of the FP64 ones, identical step counts and status flags.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2508_15522_amd import autotune as AT, configs, device as D, gridff as G, synth as S
from tests.gpu_common import COEF_SCALE, NVE_EPS, announce, drift_tolerances

pytestmark = pytest.mark.gpu


def _grid(cfg, seed, storage=G.STORE_F32):
    """The packed grid and the coefficients the oracle evaluates (FP16: the quantised ones)."""
    B = S.random_coefficients(cfg.nx, cfg.ny, cfg.nz, seed, COEF_SCALE)     # FP32-representable
    L = cfg.n_cells * S.SLAB_A
    grid = D.pack_from_coefficients(B, D.spec_for(cfg), storage, L, L)
    return grid, (O.fp16_quantize(B)[0] if storage == G.STORE_F16 else B)


def _sample(n, extra=()):
    return np.unique(np.array([0, 1, n // 3, n // 2 + 7, n - 2, n - 1, *extra]))


@pytest.mark.parametrize("storage", [G.STORE_F32, G.STORE_F16])
def test_c2_nve_full_size_sampled(storage):
    D.require_gpu()
    announce(f"full size: 16384 x pah38 NVE, block 192, storage {storage}")
    cfg = configs.GRID_SMALL
    grid, Bref = _grid(cfg, 21, storage)
    mol = S.mol_pah38()
    n_rep = configs.C2_PAH_NVE.n_rep
    sub = cfg.substrate()
    pos = S.f32(S.place_replicas(mol, n_rep, sub, S.SEED_PLACE * 2))
    vel = S.f32(S.mb_velocities(mol.mass, n_rep, 300.0, S.SEED_NVE))
    topo = G.Topology([mol])
    plan = G.Plan(topo, np.zeros(n_rep, np.int32), block_threads=192)
    st = D.fire_state(plan, list(pos), vel_per_rep=list(vel))
    out = D.outputs(plan)
    n = 20
    G.relax_batch(grid.desc, topo, plan, G.relax_params(G.MODE_NVE, n, True, dt=0.5, drift_every=1), st,
                  out["E"], out["fnorm"], out["steps"], out["drift"])
    torch.cuda.synchronize()
    idx = _sample(n_rep)
    xg = D.unsoa(plan, st["pos"])
    ref = O.nve_batch(Bref, grid.geometry, [mol], np.zeros(len(idx), np.int32), np.concatenate(pos[idx]),
                      np.concatenate(vel[idx]), n, dt=0.5, drift_every=1)
    dx = np.abs(np.concatenate([xg[i] for i in idx]) - ref["pos"]).max()
    dr = out["drift"].cpu().numpy()[idx]
    err = np.abs(dr - ref["drift"]).max(axis=0)
    tol = drift_tolerances(NVE_EPS, range(n + 1))
    announce(f"  max |dx| = {dx:.3e} A; drift-record diffs {err}; tolerances {tol}")
    assert dx < 2e-4
    assert (err <= tol).all()
    assert np.array_equal(dr[:, 5], ref["drift"][:, 5])
    assert (out["steps"].cpu().numpy() == n).all()
    assert np.isfinite(out["E"].cpu().numpy()).all()


def test_c2_langevin_full_size_sampled():
    """The thermal perturbation on the same workload: sampled replicas re-run by the oracle
    with their batch indices as Philox replica ids."""
    D.require_gpu()
    announce("full size: 16384 x pah38 Langevin, block 192")
    cfg = configs.GRID_SMALL
    grid, Bref = _grid(cfg, 24)
    mol = S.mol_pah38()
    n_rep = configs.C2_PAH_NVE.n_rep
    pos = S.f32(S.place_replicas(mol, n_rep, cfg.substrate(), S.SEED_PLACE * 5))
    vel = S.f32(S.mb_velocities(mol.mass, n_rep, 300.0, S.SEED_NVE + 1))
    topo = G.Topology([mol])
    plan = G.Plan(topo, np.zeros(n_rep, np.int32), block_threads=192)
    st = D.fire_state(plan, list(pos), vel_per_rep=list(vel))
    out = D.outputs(plan)
    n, seed, rnd = 20, 0xC0FFEE, 11
    G.relax_batch(grid.desc, topo, plan, G.relax_params(G.MODE_LANGEVIN, n, True, dt=0.5, T=300.0, gamma=0.01,
                                                        seed=seed, rnd=rnd), st, out["E"], out["fnorm"], out["steps"])
    torch.cuda.synchronize()
    idx = _sample(n_rep)
    xg = D.unsoa(plan, st["pos"])
    ref = O.langevin_batch(Bref, grid.geometry, [mol], np.zeros(len(idx), np.int32), np.concatenate(pos[idx]),
                           np.concatenate(vel[idx]), n, dt=0.5, T=300.0, gamma=0.01, seed=seed, rnd=rnd,
                           rep_id=idx)
    dx = np.abs(np.concatenate([xg[i] for i in idx]) - ref["pos"]).max()
    dE = np.abs(out["E"].cpu().numpy()[idx] - ref["E"]).max()
    announce(f"  max |dx| = {dx:.3e} A, max |dE| = {dE:.3e} eV")
    assert dx < 2e-4
    assert dE < 2e-5 * mol.n
    assert (out["steps"].cpu().numpy() == n).all()
    assert (st["status"].cpu().numpy()[idx] == ref["status"]).all()


def _fire_check(grid, Bref, mols, rep_type, pos, plan, topo, n, idx):
    st = D.fire_state(plan, pos)
    out = D.outputs(plan)
    G.relax_batch(grid.desc, topo, plan, G.relax_params(G.MODE_FIRE, n, True, f_conv=1e-4), st, out["E"],
                  out["fnorm"], out["steps"])
    torch.cuda.synchronize()
    xg = D.unsoa(plan, st["pos"])
    ref = O.fire_batch(Bref, grid.geometry, mols, rep_type[idx], np.concatenate([pos[i] for i in idx]), n)
    dx = np.abs(np.concatenate([xg[i] for i in idx]) - ref["pos"]).max()
    nat = np.array([mols[t].n for t in rep_type[idx]])
    dE = np.abs(out["E"].cpu().numpy()[idx] - ref["E"])
    announce(f"  max |dx| = {dx:.3e} A, max |dE|/atom = {(dE / nat).max():.3e} eV")
    assert dx < 2e-4
    assert (dE < 2e-5 * nat + 1e-6 * np.abs(ref["E"])).all()
    assert np.array_equal(out["steps"].cpu().numpy()[idx], ref["steps"])
    assert np.array_equal(st["status"].cpu().numpy()[idx], ref["status"])


def test_c5_fire_large_grid_full_size_sampled():
    D.require_gpu()
    announce("full size: 65536 x pah38 FIRE on the 452 x 452 x 200 grid, block 192")
    cfg = configs.GRID_LARGE
    grid, Bref = _grid(cfg, 22)
    mol = S.mol_pah38()
    n_rep = configs.C5_PAH_FIRE_LARGE.n_rep
    pos = list(S.f32(S.place_replicas(mol, n_rep, cfg.substrate(), S.SEED_PLACE)))
    topo = G.Topology([mol])
    rep_type = np.zeros(n_rep, np.int32)
    plan = G.Plan(topo, rep_type, block_threads=192)
    _fire_check(grid, Bref, [mol], rep_type, pos, plan, topo, 10, _sample(n_rep))


@pytest.mark.parametrize("forced", [None, (256, 0, 0, 2)])
def test_c3_sizes_autotuned_full_size_sampled(forced):
    """The uneven-size workload in its autotuned launch shape and, explicitly, in the shape the
    autotuner picks for it on this GPU (256-thread blocks, two lanes per atom); sampled
    replicas of every size against the oracle."""
    D.require_gpu()
    announce(f"full size: 4096 replicas of 8 sizes FIRE, {'autotuned launch' if forced is None else forced}")
    cfg = configs.GRID_SMALL
    grid, Bref = _grid(cfg, 23)
    mols = S.molecule_types("sizes")
    n_rep = configs.C3_SIZES_FIRE.n_rep
    rep_type = (np.arange(n_rep) % len(mols)).astype(np.int32)
    sub = cfg.substrate()
    per_type = [iter(S.f32(S.place_replicas(m, int((rep_type == t).sum()), sub, S.SEED_PLACE * 3 + t)))
                for t, m in enumerate(mols)]
    pos = [next(per_type[t]) for t in rep_type]
    topo = G.Topology(mols)
    if forced is None:
        st0 = D.fire_state(G.Plan(topo, rep_type), pos)
        launch, _ = AT.launch_for(grid, topo, rep_type, G.relax_params(G.MODE_FIRE, 20, True, f_conv=1e-4), st0,
                                  use_cache=False)
    else:
        launch = forced
    announce(f"  launch {launch}")
    plan = G.Plan(topo, rep_type, *launch)
    idx = _sample(n_rep, extra=range(8, 16))                   # every molecule size
    _fire_check(grid, Bref, mols, rep_type, pos, plan, topo, 10, idx)


def test_c1_chain_autotuned_full_size_sampled():
    """The chain workload (256 x 24 atoms, far too few to fill the GPU) in its autotuned launch
    shape, which may use several lanes per atom; sampled replicas against the oracle."""
    D.require_gpu()
    announce("full size: 256 x chain24 FIRE, autotuned launch")
    cfg = configs.GRID_SMALL
    grid, Bref = _grid(cfg, 25)
    mol = S.mol_chain24()
    n_rep = configs.C1_CHAIN_FIRE.n_rep
    rep_type = np.zeros(n_rep, np.int32)
    pos = list(S.f32(S.place_replicas(mol, n_rep, cfg.substrate(), S.SEED_PLACE)))
    topo = G.Topology([mol])
    st0 = D.fire_state(G.Plan(topo, rep_type), pos)
    launch, rate = AT.launch_for(grid, topo, rep_type, G.relax_params(G.MODE_FIRE, 50, True, f_conv=1e-4), st0,
                                 use_cache=False)
    announce(f"  launch {launch} ({rate:.3e} replica-steps/s)")
    plan = G.Plan(topo, rep_type, *launch)
    _fire_check(grid, Bref, [mol], rep_type, pos, plan, topo, 20, _sample(n_rep))
