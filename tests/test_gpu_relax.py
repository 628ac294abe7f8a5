"""GPU parity of the fused relaxation / dynamics path (a5-a8, a14) against the oracle.

Both sides run on the same model: a physical grid built, fitted and FP32-rounded by
the oracle (direct Morse sums + 2D Ewald), packed into the GPU layout by the library.
FP32 and FP64 trajectories separate slowly, so parity is checked over short runs
from identical seeded starts: positions within 2e-4 A after 25 FIRE moves or 50 NVE
steps, energies within 2e-5 eV per atom.  Long runs are checked through properties
(energy lowered, convergence flags consistent with the reported force norm,
determinism, resumability, batch-composition independence).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2508_15522_amd import device as D, gridff as G, synth as S
from tests.gpu_common import NVE_EPS, announce, drift_tolerances, oracle_relax_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def world():
    D.require_gpu()
    sub, geo, B = oracle_relax_grid()
    spec = G.grid_spec(geo["nx"], geo["ny"], geo["nz"], 0.0, 0.0, geo["z0"], geo["dz"])
    grid = D.pack_from_coefficients(B, spec, G.STORE_F32, sub.Lx, sub.Ly)
    assert grid.geometry == geo
    # the same coefficients in FP16 storage; the oracle runs on their quantised values
    grid16 = D.pack_from_coefficients(B, spec, G.STORE_F16, sub.Lx, sub.Ly)
    B16, _ = O.fp16_quantize(B)
    mols = S.molecule_types("sizes") + [S.mol_chain24(), S.mol_pah38()]
    topo = G.Topology(mols)
    return dict(sub=sub, geo=geo, B=B, grid=grid, grid16=grid16, B16=B16, mols=mols, topo=topo)


def _grid(w, storage):
    return w["grid16"] if storage == G.STORE_F16 else w["grid"]


def _B(w, storage):
    return w["B16"] if storage == G.STORE_F16 else w["B"]


def _plan_or_skip(topo, rep_type, block):
    try:
        return G.Plan(topo, rep_type, block_threads=block)
    except G.GffError as e:
        if "unsupported" in str(e):
            pytest.skip(f"{block}-thread blocks exceed this device's LDS per block")
        raise


def _positions(w, rep_type, seed, h=(2.8, 4.0)):
    return [S.place_replicas(w["mols"][t], 1, w["sub"], seed + r, h)[0] for r, t in enumerate(rep_type)]


def _fire(w, plan, pos, n_steps, f_conv=1e-4, st=None, storage=G.STORE_F32, **kw):
    st = st or D.fire_state(plan, pos)
    out = D.outputs(plan)
    prm = G.relax_params(G.MODE_FIRE, n_steps, True, f_conv=f_conv, **kw)
    G.relax_batch(_grid(w, storage).desc, w["topo"], plan, prm, st, out["E"], out["fnorm"], out["steps"])
    torch.cuda.synchronize()
    return st, out


# FP32 storage; FP16 storage with the register stencil cache (blocks of <= 512 threads) and
# without it (1024-thread blocks gather every step)
@pytest.mark.parametrize("storage,block", [(G.STORE_F32, 256), (G.STORE_F16, 256), (G.STORE_F16, 1024)])
@pytest.mark.parametrize("n_steps", [0, 1, 25])
def test_fire_short_run_parity(world, n_steps, storage, block):
    w = world
    announce(f"fire parity n_steps={n_steps} storage={storage} block={block}")
    rng = np.random.default_rng(3)
    rep_type = rng.integers(0, len(w["mols"]), 40)
    plan = _plan_or_skip(w["topo"], rep_type, block)
    pos = _positions(w, rep_type, 500)
    st, out = _fire(w, plan, pos, n_steps, storage=storage)
    ref = O.fire_batch(_B(w, storage), w["geo"], w["mols"], rep_type, np.concatenate(pos), n_steps)
    xg = np.concatenate(D.unsoa(plan, st["pos"]))
    dx = np.abs(xg - ref["pos"]).max()
    nat = np.array([w["mols"][t].n for t in rep_type])
    dE = np.abs(out["E"].cpu().numpy() - ref["E"])
    announce(f"  max |dx| = {dx:.3e} A, max |dE|/atom = {(dE / nat).max():.3e} eV")
    assert dx < 2e-4
    assert (dE < 2e-5 * nat + 1e-6 * np.abs(ref["E"])).all()
    assert np.allclose(out["fnorm"].cpu().numpy(), ref["fnorm"], rtol=1e-3, atol=1e-4)
    assert np.array_equal(out["steps"].cpu().numpy(), ref["steps"])
    assert np.array_equal(st["status"].cpu().numpy(), ref["status"])
    assert np.array_equal(st["fire_npos"].cpu().numpy(), ref["npos"])
    assert np.allclose(st["fire_dt"].cpu().numpy(), ref["dt"], rtol=1e-6)


def test_fire_check_cadence_parity(world):
    """The paper's form: replica-wide decisions (convergence test, P, mixing, adaptation,
    restart) every 7th move, plain kicks in between; 40 moves against the oracle."""
    w = world
    announce("fire check cadence 7")
    rng = np.random.default_rng(4)
    rep_type = rng.integers(0, len(w["mols"]), 30)
    plan = G.Plan(w["topo"], rep_type, block_threads=256)
    pos = _positions(w, rep_type, 800)
    st, out = _fire(w, plan, pos, 40, check_every=7)
    ref = O.fire_batch(w["B"], w["geo"], w["mols"], rep_type, np.concatenate(pos), 40, check_every=7)
    dx = np.abs(np.concatenate(D.unsoa(plan, st["pos"])) - ref["pos"]).max()
    nat = np.array([w["mols"][t].n for t in rep_type])
    dE = np.abs(out["E"].cpu().numpy() - ref["E"])
    announce(f"  max |dx| = {dx:.3e} A, max |dE|/atom = {(dE / nat).max():.3e} eV")
    assert dx < 2e-4
    assert (dE < 2e-5 * nat + 1e-6 * np.abs(ref["E"])).all()
    assert np.array_equal(out["steps"].cpu().numpy(), ref["steps"])
    assert np.array_equal(st["status"].cpu().numpy(), ref["status"])
    assert np.array_equal(st["fire_npos"].cpu().numpy(), ref["npos"])


def test_fire_long_run_properties_and_determinism(world):
    w = world
    announce("fire long run")
    rep_type = np.repeat(np.arange(len(w["mols"])), 6)
    plan = G.Plan(w["topo"], rep_type, block_threads=256)
    pos = _positions(w, rep_type, 900)
    st1, o1 = _fire(w, plan, pos, 4000, f_conv=1e-3)
    st2, o2 = _fire(w, plan, pos, 4000, f_conv=1e-3)
    for k in st1:
        assert torch.equal(st1[k], st2[k]), k
    for k in ("E", "fnorm", "steps"):
        assert torch.equal(o1[k], o2[k]), k
    E0 = O.eval_batch(w["B"], w["geo"], w["mols"], rep_type, np.concatenate(pos))[1]
    E = o1["E"].cpu().numpy()
    status = st1["status"].cpu().numpy()
    fn = o1["fnorm"].cpu().numpy()
    steps = o1["steps"].cpu().numpy()
    assert (E < E0).all()
    conv = (status & G.REP_CONVERGED) != 0
    assert (fn[conv] < 1e-3).all() and (steps[conv] <= 4000).all()
    assert ((status[~conv] & G.REP_MAXSTEPS) != 0).all()
    announce(f"  converged {conv.sum()}/{len(conv)}; mean steps {steps[conv].mean() if conv.any() else 0:.0f}")
    assert conv.mean() > 0.5


def test_fire_resume_equals_continuous(world):
    w = world
    announce("fire resume")
    rep_type = np.array([9, 8, 3, 9, 0, 7])
    plan = G.Plan(w["topo"], rep_type)
    pos = _positions(w, rep_type, 40)
    stA, oA = _fire(w, plan, pos, 60, f_conv=0.0)
    stB, _ = _fire(w, plan, pos, 30, f_conv=0.0)
    stB, oB = _fire(w, plan, None, 30, f_conv=0.0, st=stB)
    for k in stA:
        assert torch.equal(stA[k], stB[k]), k
    assert torch.equal(oA["E"], oB["E"])


def test_batch_composition_and_launch_shape_do_not_change_results(world):
    """A replica's result does not depend on the other replicas in the batch or on the
    block size: the mixed (uneven) batch equals per-type batches bit for bit."""
    w = world
    announce("batch composition")
    rng = np.random.default_rng(8)
    rep_type = rng.integers(0, len(w["mols"]), 50)
    pos = _positions(w, rep_type, 1200)
    ref = None
    for bt in (128, 320, 512):
        plan = G.Plan(w["topo"], rep_type, block_threads=bt)
        st, out = _fire(w, plan, pos, 40)
        x = D.unsoa(plan, st["pos"])
        if ref is None:
            ref = (x, out["E"].cpu().numpy())
        else:
            assert all(np.array_equal(a, b) for a, b in zip(x, ref[0]))
            assert np.array_equal(out["E"].cpu().numpy(), ref[1])
    for t in np.unique(rep_type):
        idx = np.where(rep_type == t)[0]
        plan = G.Plan(w["topo"], rep_type[idx], block_threads=256)
        st, out = _fire(w, plan, [pos[i] for i in idx], 40)
        x = D.unsoa(plan, st["pos"])
        for k, i in enumerate(idx):
            assert np.array_equal(x[k], ref[0][i])


def test_status_flags_nonfinite_and_out_of_domain(world):
    w = world
    announce("status flags")
    rep_type = np.array([9, 9, 9, 9])
    plan = G.Plan(w["topo"], rep_type)
    pos = _positions(w, rep_type, 70)
    pos[1] = pos[1].copy(); pos[1][3, 0] = np.nan                      # one NaN coordinate
    pos[2] = pos[2].copy(); pos[2][:, 2] -= pos[2][:, 2].min() - 1.2  # an atom below z0
    st, out = _fire(w, plan, pos, 5)
    s = st["status"].cpu().numpy()
    ref = O.fire_batch(w["B"], w["geo"], w["mols"], rep_type, np.concatenate(pos), 5)
    assert s[1] & G.REP_NONFINITE and not (s[0] & G.REP_NONFINITE) and not (s[3] & G.REP_NONFINITE)
    assert s[2] & G.REP_OUT_OF_DOMAIN and not (s[0] & G.REP_OUT_OF_DOMAIN)
    assert np.isnan(out["E"].cpu().numpy()[1])
    assert np.array_equal(s, ref["status"])
    # the healthy replicas equal a run without the faulty ones
    plan2 = G.Plan(w["topo"], rep_type[[0, 3]])
    st2, _ = _fire(w, plan2, [pos[0], pos[3]], 5)
    x = D.unsoa(plan, st["pos"]); x2 = D.unsoa(plan2, st2["pos"])
    assert np.array_equal(x[0], x2[0]) and np.array_equal(x[3], x2[1])
    # the NaN replica is frozen: its coordinates are returned unchanged
    assert np.array_equal(np.isnan(x[1]), np.isnan(pos[1]))




@pytest.mark.parametrize("storage,drift_every", [(G.STORE_F32, 1), (G.STORE_F32, 7), (G.STORE_F16, 1)])
def test_nve_short_run_parity_and_drift(world, storage, drift_every):
    w = world
    announce(f"nve parity storage={storage} drift_every={drift_every}")
    pah = len(w["mols"]) - 1
    rep_type = np.full(24, pah)
    plan = G.Plan(w["topo"], rep_type, block_threads=256)
    pos = _positions(w, rep_type, 2000)
    vel = list(S.mb_velocities(w["mols"][pah].mass, len(rep_type), 300.0, S.SEED_NVE))
    st = D.fire_state(plan, pos, vel_per_rep=vel)
    out = D.outputs(plan)
    n = 50
    prm = G.relax_params(G.MODE_NVE, n, True, dt=0.5, drift_every=drift_every)
    G.relax_batch(_grid(w, storage).desc, w["topo"], plan, prm, st, out["E"], out["fnorm"], out["steps"],
                  out["drift"])
    torch.cuda.synchronize()
    ref = O.nve_batch(_B(w, storage), w["geo"], w["mols"], rep_type, np.concatenate(pos), np.concatenate(vel), n,
                      dt=0.5, drift_every=drift_every)
    xg = np.concatenate(D.unsoa(plan, st["pos"]))
    dx = np.abs(xg - ref["pos"]).max()
    dr = out["drift"].cpu().numpy()
    err = np.abs(dr - ref["drift"]).max(axis=0)
    tol = drift_tolerances(NVE_EPS, range(0, n + 1, drift_every))
    announce(f"  max |dx| = {dx:.3e}; drift-record diffs {err}; tolerances {tol}; "
             f"max|dE| gpu {dr[:, 2].max():.3e} oracle {ref['drift'][:, 2].max():.3e}")
    assert dx < 2e-4
    assert (err <= tol).all()
    assert np.array_equal(dr[:, 5], ref["drift"][:, 5])
    assert (dr[:, 5] == n // drift_every + 1).all()
    assert (out["steps"].cpu().numpy() == n).all()
    # FP32 forces with FP64 accounting: the energy error stays far below the thermal scale
    assert dr[:, 2].max() < 5e-3


def test_nve_grid_only_without_drift_record(world):
    """NVE on the grid alone (no intramolecular field) and no drift record: the launch
    shape with no block barrier between two steps' position exchanges."""
    w = world
    announce("nve grid only, no drift record")
    rng = np.random.default_rng(12)
    rep_type = rng.integers(0, len(w["mols"]), 30)
    plan = G.Plan(w["topo"], rep_type, block_threads=256)
    pos = _positions(w, rep_type, 2600)
    vel = [S.mb_velocities(w["mols"][t].mass, 1, 300.0, S.SEED_NVE + 1 + r)[0] for r, t in enumerate(rep_type)]
    st = D.fire_state(plan, pos, vel_per_rep=vel)
    out = D.outputs(plan)
    n = 60
    prm = G.relax_params(G.MODE_NVE, n, False, dt=0.5)
    G.relax_batch(w["grid"].desc, w["topo"], plan, prm, st, out["E"], out["fnorm"], out["steps"])
    torch.cuda.synchronize()
    ref = O.nve_batch(w["B"], w["geo"], w["mols"], rep_type, np.concatenate(pos), np.concatenate(vel), n, dt=0.5,
                      intra_on=False)
    dx = np.abs(np.concatenate(D.unsoa(plan, st["pos"])) - ref["pos"]).max()
    nat = np.array([w["mols"][t].n for t in rep_type])
    dE = np.abs(out["E"].cpu().numpy() - ref["E"])
    announce(f"  max |dx| = {dx:.3e} A, max |dE|/atom = {(dE / nat).max():.3e} eV")
    assert dx < 2e-4
    assert (dE < 2e-5 * nat).all()
    assert (out["steps"].cpu().numpy() == n).all()
    assert np.array_equal(st["status"].cpu().numpy(), ref["status"])


def test_fire_teacher_forced_steps_and_final_certificate(world):
    """Long runs cannot be compared step for step (FP32 and FP64 trajectories separate), so
    (i) teacher forcing: the GPU state after 1500 moves (positions, velocities, FIRE dt,
    alpha, count, flags) is handed to the oracle, and both sides take 5 more moves from it;
    (ii) a final-state certificate: the oracle's FP64 |F|_2 and energy at the GPU's final
    positions agree with the convergence the GPU reported."""
    w = world
    announce("fire teacher forcing + certificate")
    rep_type = np.repeat(np.arange(len(w["mols"])), 4)
    plan = G.Plan(w["topo"], rep_type, block_threads=256)
    pos = _positions(w, rep_type, 1700)
    st, out = _fire(w, plan, pos, 1500, f_conv=1e-3)
    x = np.concatenate(D.unsoa(plan, st["pos"]))
    v = np.concatenate(D.unsoa(plan, st["vel"]))
    state = dict(dt=st["fire_dt"].cpu().numpy().astype(np.float64), alpha=st["fire_alpha"].cpu().numpy().astype(np.float64),
                 npos=st["fire_npos"].cpu().numpy(), status=st["status"].cpu().numpy())
    nat = np.array([w["mols"][t].n for t in rep_type])
    # (ii) certificate at the GPU's final positions
    Fo, Eo, _, _ = O.eval_batch(w["B"], w["geo"], w["mols"], rep_type, x)
    off = np.concatenate([[0], np.cumsum(nat)])
    fo = np.array([np.linalg.norm(Fo[off[r]:off[r + 1]]) for r in range(len(rep_type))])
    conv = (state["status"] & G.REP_CONVERGED) != 0
    announce(f"  converged {conv.sum()}/{len(conv)}; oracle |F| at converged GPU states max "
             f"{fo[conv].max() if conv.any() else 0:.2e}")
    assert conv.any()
    assert (fo[conv] < 1e-3 + 2e-4).all()
    assert (np.abs(out["E"].cpu().numpy() - Eo) < 2e-5 * nat + 1e-6 * np.abs(Eo)).all()
    # (i) five more moves from the GPU's state on both sides (converged replicas stay put)
    st2, out2 = _fire(w, plan, None, 5, f_conv=1e-3, st=st)
    ref = O.fire_batch(w["B"], w["geo"], w["mols"], rep_type, x, 5, vel=v, state=state, f_conv=1e-3)
    x2 = np.concatenate(D.unsoa(plan, st2["pos"]))
    dx = np.abs(x2 - ref["pos"]).max()
    announce(f"  teacher-forced 5 moves: max |dx| = {dx:.2e} A")
    assert dx < 2e-5
    assert np.array_equal(out2["steps"].cpu().numpy(), ref["steps"])
    assert np.array_equal(st2["status"].cpu().numpy(), ref["status"])
    assert np.abs(st2["fire_dt"].cpu().numpy() - ref["dt"]).max() < 1e-6


def test_fire_hand_worked_trajectory_on_the_gpu():
    """The GPU's FIRE moves follow the hand-worked trajectory of the update order (one
    charge in an anisotropic quadratic bowl represented exactly by the B-spline model,
    N_min = 0, a restart on the first move, then two adapting moves).  Tolerances are set by
    the FP32 rounding of the start position (~1.2e-7 A) and of the coefficients."""
    from tests.test_oracle_closed_forms import FIRE_HAND, _bowl_grid, _charge
    D.require_gpu()
    announce("fire hand-worked trajectory")
    B, spec_o, rs = _bowl_grid()
    n, h = spec_o["nx"], spec_o["dx"]
    spec = G.grid_spec(n, n, n, 0.0, 0.0, 0.0, h)
    grid = D.pack_from_coefficients(B, spec, G.STORE_F32, n * h, n * h)
    topo = G.Topology([_charge()])
    x0 = rs + np.array([0.3, 0.2, 0.0])
    for moves in (1, 2, 3):
        plan = G.Plan(topo, np.array([0]), block_threads=64)
        st = D.fire_state(plan, [x0[None]], vel_per_rep=[np.array([[0.206, -0.142, 0.0]])])
        out = D.outputs(plan)
        prm = G.relax_params(G.MODE_FIRE, moves, False, f_conv=1e-9, nmin=0)
        G.relax_batch(grid.desc, topo, plan, prm, st, out["E"], out["fnorm"], out["steps"])
        torch.cuda.synchronize()
        v, d, dt, a, npos = FIRE_HAND[moves - 1]
        xg = D.unsoa(plan, st["pos"])[0][0]
        vg = D.unsoa(plan, st["vel"])[0][0]
        announce(f"  {moves} moves: |dx| {np.abs(xg[:2] - rs[:2] - d).max():.2e} A, |dv| {np.abs(vg[:2] - v).max():.2e}")
        assert np.abs(xg[:2] - rs[:2] - d).max() < 5e-7
        assert np.abs(vg[:2] - v).max() < 2e-7
        assert abs(st["fire_dt"].item() - dt) < 1e-8 and abs(st["fire_alpha"].item() - a) < 1e-8
        assert st["fire_npos"].item() == npos and out["steps"].item() == moves
