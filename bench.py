#!/usr/bin/env python3
"""Benchmark of the GridFF hot path on one MI355X.

Workload (default): 16 384 replicas of the 38-atom planar molecule on the 2x2-cell,
3-plane rock-salt slab, grids 112 x 112 x 150 x 3 built and fitted on the GPU (FP64)
and stored in FP32; velocity-Verlet NVE, dt = 0.5 fs, 300 K start, FP64 drift
accounting every step.  One benchmark step = one gff_relax_batch launch that advances
every replica by 5000 MD steps (grid interpolation + intramolecular field + integrator,
all inside the kernel).  value = replica-steps/s over the K timed launches.

Prints one JSON line.  Roofline: the dominant kernel is the replica kernel.  Its binding
resource is VALU issue, so the record is an ALU roofline: the method's algorithmic work, about
68 kflop per replica-step of the 38-atom molecule (38 interpolations of about 0.75 kflop plus
about 40 kflop of intramolecular field), divided by the kernel's mean launch time from HIP
events on its stream, against the FP32 vector peak.  The memory roofline of the same launch
(64 stencil nodes x 3 channels x 4 B per atom per force evaluation, against the 8 TB/s HBM
peak) is reported beside it under `memory`.  `traffic` (fabric bytes per launch) and `valu`
(VALU wave instructions per launch, and their share of the issue slots in the measured time)
come from rocprofv3 counters stored below with the digests of the kernel sources they were
taken on; both are null once those sources change.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak from the unit counts: 256 CUs x 4 SIMDs x 16 lanes x 2 flop per FMA x 2.4 GHz
# = 78.6 TFLOP/s in scalar FP32 instructions, twice that with packed FP32 (two FMAs per lane);
# the kernels here are built without packed FP32 instructions
FP32_PEAK_TFLOPS = 157.3
FP32_UNPACKED_PEAK_TFLOPS = 78.6
# algorithmic work per replica-step of the 38-atom molecule: 38 atom-interpolations of about
# 0.75 kflop (channel pre-mix and tensor-product contraction) and about 40 kflop of the
# intramolecular field (each non-bonded pair, bond, angle and torsion once)
FLOP_PER_REPLICA_STEP = 68e3

# Fabric-side traffic of the replica kernel (L2 misses to MALL/HBM) from two rocprofv3 --pmc
# passes, FETCH_SIZE then WRITE_SIZE, in KiB for one launch of the workload named by the key
# (storage, replicas, MD steps, block threads).  A plain 1 GiB elementwise kernel reads as 512 MiB by
# FETCH_SIZE and writes as 1 GiB by WRITE_SIZE, so the counters are scaled by 2.0 and 1.0.
# The figures hold only for the kernel sources whose SHA-256 they carry.
COUNTER_SCALE = {"fetch": 2.0, "write": 1.0}
MEASURED_TRAFFIC = {
    ("f32", 16384, 5000, 192): {
        "sources": {"paper_2508_15522_amd/csrc/gff_relax.hip":
                    "9dc9019c3b2ac01344b26dfaa5a1347af45c3a2681ff828ec5b3c877fe659e02",
                    "paper_2508_15522_amd/csrc/gff_internal.hpp":
                    "292688bf231d8aa97cae1d155c53d9cd5057b10c7087da7ad24bc2be08d79351",
                    "paper_2508_15522_amd/csrc/gff_host.hip":
                    "2aa04dd935f3d23fd37d27ccea38d3373c1936d34b561ec069f5a5d707862209"},
        "fetch_kib": 214912281.9375, "write_kib": 100342.1875,
        "valu_insts": 190632080689.0,          # SQ_INSTS_VALU (wave instructions) of the launch
    },
}
# FP32 VALU issue slots per second: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def _counters(storage, n_rep, md_steps, block):
    """The stored counter record for this launch, or None if the kernel has changed since."""
    import hashlib
    rec = MEASURED_TRAFFIC.get((storage, n_rep, md_steps, block))
    if rec is None:
        return None
    for path, digest in rec["sources"].items():
        with open(os.path.join(ROOT, path), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return rec


def measured_traffic(storage, n_rep, md_steps, block):
    """Fabric bytes per launch from the stored counters (None if the kernel has changed)."""
    rec = _counters(storage, n_rep, md_steps, block)
    if rec is None:
        return None
    return rec["fetch_kib"] * 1024 * COUNTER_SCALE["fetch"] + rec["write_kib"] * 1024 * COUNTER_SCALE["write"]


def valu_utilisation(storage, n_rep, md_steps, block, kernel_s):
    """Stored VALU instruction count of the launch over the issue slots of the measured
    launch time (None if the kernel has changed since the counters were taken)."""
    rec = _counters(storage, n_rep, md_steps, block)
    if rec is None or "valu_insts" not in rec:
        return None
    return {"insts": rec["valu_insts"], "issue_frac": rec["valu_insts"] / (VALU_ISSUE_PEAK * kernel_s),
            "peak_insts_per_s": VALU_ISSUE_PEAK}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--md-steps", type=int, default=5000, help="MD steps per relax_batch launch")
    ap.add_argument("--replicas", type=int, default=16384)
    ap.add_argument("--storage", choices=["f32", "f16"], default="f32")
    ap.add_argument("--block", type=int, default=192,
                    help="block threads (192: five 38-atom replicas fill 190 of 192 lanes; the fastest of a "
                         "64..448 sweep)")
    ap.add_argument("--compare-f16", action="store_true", help="(default) also time the FP16-grid variant")
    ap.add_argument("--no-f16", action="store_true", help="skip the FP16-grid arm")
    ap.add_argument("--no-minima", action="store_true", help="skip the learned-vs-uniform minima/s comparison")
    ap.add_argument("--no-c5", action="store_true", help="skip the large-substrate (c5) record")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the chain (c1) and uneven-size (c3) records (autotuned launches)")
    ap.add_argument("--compare-langevin", action="store_true",
                    help="also time the same replicas under Langevin dynamics (BAOAB, 300 K, gamma 0.01/fs)")
    ap.add_argument("--compare-trilinear", action="store_true",
                    help="also time the trilinear energy/force storage (the earlier scheme) and its NVE drift")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--minima", action="store_true",
                    help="(default) learned vs uniform proposals: minima found per second")
    ap.add_argument("--train-steps", type=int, default=1000, help="IMLE steps of the proposer (--minima)")
    ap.add_argument("--imle-batch", type=int, default=1024, help="training minima per IMLE step (--minima)")
    ap.add_argument("--imle-k", type=int, default=64, help="noise candidates per training minimum (--minima)")
    ap.add_argument("--weight-power", type=float, default=1.0,
                    help="training weight of a minimum: (members of its energy class)^-p (--minima)")
    ap.add_argument("--scans", action="store_true",
                    help="batched restrained scans: relaxed detachment and drag of pah38, 4096 paths")
    ap.add_argument("--defect", action="store_true",
                    help="large defect supercell grid (20x20x3, 1128x1128x80): build, and a batched drag over the defect")
    ap.add_argument("--hopping", action="store_true",
                    help="minima hopping (Langevin + FIRE) vs uniform proposals: minima found per second")
    ap.add_argument("--extra", nargs="*", default=[], choices=["c1", "c3", "c5"],
                    help="also time the chain (c1), uneven-size (c3) or large-substrate (c5) workloads")
    ap.add_argument("--direct", nargs="*", default=[], choices=["c2", "c5"],
                    help="also time the all-atom comparison mode (direct substrate sums over 9 cells) against "
                         "GridFF on the C2 (48 substrate atoms) or C5 (3072) replicas")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device copy first (reference for HBM counter scaling)")
    args = ap.parse_args()
    args.compare_f16 = not args.no_f16
    args.minima = not args.no_minima
    if not args.no_c5 and "c5" not in args.extra:
        args.extra = list(args.extra) + ["c5"]
    if not args.no_small:
        args.extra = list(args.extra) + [w for w in ("c1", "c3") if w not in args.extra]
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "replicas are independent, so more GPUs would each run their own share", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2508_15522_amd import configs, device as D, gridff as G, synth as S
    D.require_gpu()
    wl = configs.C2_PAH_NVE
    cfg = wl.grid
    sub = cfg.substrate()
    spec = D.spec_for(cfg)
    mol = S.mol_pah38()
    mols = [mol]
    n_rep = args.replicas
    block = args.block

    def setup(storage):
        grid = D.build_physical_grid(sub, spec, storage)
        return grid

    log("building grid (FP64 build + fit on GPU)")
    t0 = time.time()
    grid = setup(G.STORE_F16 if args.storage == "f16" else G.STORE_F32)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    topo = G.Topology(mols)
    plan = G.Plan(topo, np.zeros(n_rep, np.int32), block_threads=block)
    pos0 = S.place_replicas(mol, n_rep, sub, S.SEED_PLACE * 2)
    vel0 = S.mb_velocities(mol.mass, n_rep, 300.0, S.SEED_NVE)
    st0 = D.fire_state(plan, pos0, vel_per_rep=vel0)
    out = D.outputs(plan)
    prm = G.relax_params(G.MODE_NVE, args.md_steps, True, dt=0.5, drift_every=1)
    stream = torch.cuda.current_stream()

    def run_once(g, st):
        G.relax_batch(g.desc, topo, plan, prm, st, out["E"], out["fnorm"], out["steps"], out["drift"], stream)

    def fresh_state():
        return {k: v.clone() for k, v in st0.items()}

    def timed(g, K, W):
        for _ in range(W):
            run_once(g, fresh_state())
        torch.cuda.synchronize()
        states = [fresh_state() for _ in range(K)]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * K)]
        torch.cuda.synchronize()
        t = time.time()
        for k in range(K):
            ev[2 * k].record(stream)
            run_once(g, states[k])
            ev[2 * k + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.time() - t
        per = [ev[2 * k].elapsed_time(ev[2 * k + 1]) / 1e3 for k in range(K)]
        return wall, per, states[-1]

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")     # 1 GiB read, 1 GiB written
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    log(f"warmup {args.warmup}, timing {args.steps} launches of {args.md_steps} MD steps x {n_rep} replicas")
    wall, per, st_last = timed(grid, args.steps, args.warmup)
    rs = n_rep * args.md_steps
    value = rs * args.steps / wall
    kern_avg = float(np.mean(per))
    kern_med = float(np.median(per))
    drift = out["drift"].cpu().numpy()
    status = st_last["status"].cpu().numpy()
    # algorithmic bytes: 64 stencil nodes x 3 channels per atom per force evaluation
    bpn = 4 if args.storage == "f32" else 2
    evals = args.md_steps + 1
    alg_bytes = n_rep * mol.n * evals * 64 * 3 * bpn
    achieved = alg_bytes / kern_avg / 1e9
    # algorithmic flops: the per-replica-step work of the 38-atom molecule over every replica-step
    alg_flops = FLOP_PER_REPLICA_STEP * rs
    tflops = alg_flops / kern_avg / 1e12
    res = {
        "metric": "replica-steps/s",
        "value": value,
        "unit": "replica-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {
            "workload": f"pah38-nve-{n_rep}",
            "substrate": "rock-salt 2x2 cells x 3 planes (48 atoms), a=5.64 A, +-0.7 e",
            "grid": f"{cfg.nx}x{cfg.ny}x{cfg.nz}x3 {args.storage} (0.1 A)",
            "replicas": n_rep, "atoms_per_replica": mol.n, "md_steps_per_launch": args.md_steps,
            "dt_fs": 0.5, "block_threads": block, "drift_fp64_every": 1,
        },
        "interpolations_per_s": n_rep * mol.n * evals * args.steps / wall,
        "kernel_avg_s": kern_avg,
        "kernel_median_s": kern_med,
        "replica_steps_per_s_median_launch": rs / kern_med,
        "grid_build_fit_s": build_s,
        "nve_max_abs_drift_eV": float(np.nanmax(drift[:, 2])),
        "nonfinite_replicas": int(((status & G.REP_NONFINITE) != 0).sum()),
        # the kernel is bound by VALU issue (valu.issue_frac): the register stencil cache removes
        # three quarters of the gather traffic, so HBM is not what limits it.  On the method's
        # own roofline (about 2.3 flop per gathered byte, below the FP32 ridge) the memory roof
        # would bind; that fraction is `memory.frac`.
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_PEAK_TFLOPS,
                     "traffic": measured_traffic(args.storage, n_rep, args.md_steps, block),
                     "kernel": f"k_replicas<{args.storage},NVE>",
                     "flop_per_replica_step": FLOP_PER_REPLICA_STEP, "flop_per_launch": alg_flops,
                     "peak_unpacked": FP32_UNPACKED_PEAK_TFLOPS,
                     "frac_unpacked": tflops / FP32_UNPACKED_PEAK_TFLOPS,
                     "valu": valu_utilisation(args.storage, n_rep, args.md_steps, block, kern_avg),
                     "memory": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": alg_bytes}},
    }
    tr = res["roofline"]["traffic"]
    res["roofline"]["memory"]["fabric_GBps"] = tr / kern_avg / 1e9 if tr else None
    res["roofline"]["memory"]["fabric_frac"] = tr / kern_avg / 1e9 / HBM_PEAK_GBS if tr else None
    # interpolation alone: one evaluation launch (grid part only, no stencil reuse) over the
    # same atoms, repeated
    F = torch.empty_like(st0["pos"])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    G.eval_forces(grid.desc, topo, plan, False, st0["pos"], F, None, None, None, stream)
    n_eval = 20
    e0.record(stream)
    for _ in range(n_eval):
        G.eval_forces(grid.desc, topo, plan, False, st0["pos"], F, None, None, None, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ev_s = e0.elapsed_time(e1) / 1e3 / n_eval
    res["eval_interpolations_per_s"] = n_rep * mol.n / ev_s
    res["eval_launch_s"] = ev_s
    log(f"eval_forces (grid only): {res['eval_interpolations_per_s']:.3e} interpolations/s, {ev_s * 1e3:.3f} ms per launch")
    res["gather_probe"] = gather_probe(grid, log)
    res["roofline"]["memory"]["serving_probe_GBps"] = res["gather_probe"]["grid_coefficients"]
    # the evaluation launch in the probe's own unit: every atom reads 16 z-column segments of
    # four padded 16-byte nodes (64 B each, the probe's chunk), of which 48 B are coefficients
    chunk_bytes = n_rep * mol.n * 16 * (64 if args.storage == "f32" else 32)
    res["eval_chunk_GBps"] = chunk_bytes / ev_s / 1e9
    res["eval_vs_gather_probe"] = res["eval_chunk_GBps"] / res["gather_probe"]["grid_coefficients"]
    if args.compare_f16 and args.storage == "f32":
        g16 = setup(G.STORE_F16)
        w16, p16, st16 = timed(g16, args.steps, 1)
        drift16 = out["drift"].cpu().numpy()
        # storage error of the FP16 arm: grid forces of both storages at the workload's start
        # positions and at the FP16 run's final positions (one evaluation launch each)
        errs = []
        for pos in (st0["pos"], st16["pos"]):
            F32, F16 = torch.empty_like(pos), torch.empty_like(pos)
            G.eval_forces(grid.desc, topo, plan, False, pos, F32, None, None, None, stream)
            G.eval_forces(g16.desc, topo, plan, False, pos, F16, None, None, None, stream)
            torch.cuda.synchronize()
            errs.append(torch.linalg.vector_norm((F16 - F32).double(), dim=0).cpu().numpy())
        err = np.concatenate(errs)
        err = err[np.isfinite(err)]
        res["f16"] = {"value": rs * args.steps / w16, "kernel_avg_s": float(np.mean(p16)),
                      "kernel_median_s": float(np.median(p16)), "vs_f32": rs * args.steps / w16 / value,
                      "force_err_vs_f32_storage_eV_per_A": {"max": float(err.max()), "rms": float(np.sqrt((err ** 2).mean())),
                                                            "atoms": int(err.size)},
                      "nve_max_abs_drift_eV": float(np.nanmax(drift16[:, 2])),
                      "grid": f"{cfg.nx}x{cfg.ny}x{cfg.nz}x3 f16 (per-channel scale, Pauli residual half)"}
        res["f16_value"] = res["f16"]["value"]
        res["f16_vs_f32"] = res["f16"]["vs_f32"]
        log(f"FP16 grid: {res['f16_value']:.3e} replica-steps/s ({res['f16_vs_f32']:.3f}x FP32), force error vs "
            f"FP32 storage max {err.max():.2e} eV/A")
    if args.compare_langevin:
        lprm = G.relax_params(G.MODE_LANGEVIN, args.md_steps, True, dt=0.5, T=300.0, gamma=0.01, seed=S.SEED_PHILOX)
        lts = []
        for k in range(args.steps + 1):
            stl = fresh_state()
            lprm.round = k
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            G.relax_batch(grid.desc, topo, plan, lprm, stl, out["E"], out["fnorm"], out["steps"], None, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            if k > 0:                                    # the first launch is a warm-up
                lts.append(e0.elapsed_time(e1) / 1e3)
        res["langevin_kernel_avg_s"] = float(np.mean(lts))
        res["langevin_value"] = rs / res["langevin_kernel_avg_s"]
        res["langevin_vs_nve_kernel"] = kern_avg / res["langevin_kernel_avg_s"]
        log(f"Langevin: {res['langevin_value']:.3e} replica-steps/s by kernel time "
            f"({res['langevin_vs_nve_kernel']:.3f}x the NVE kernel time ratio)")
    if args.compare_trilinear and args.storage == "f32":
        gtri = setup(G.STORE_TRILINEAR)
        wt, pt, _ = timed(gtri, args.steps, 1)
        res["trilinear_value"] = rs * args.steps / wt
        res["trilinear_kernel_avg_s"] = float(np.mean(pt))
        res["trilinear_vs_bspline"] = res["trilinear_value"] / value
        drift_t = float(out["drift"].cpu().numpy()[:, 2].max())
        res["trilinear_max_abs_drift_eV"] = drift_t
        log(f"trilinear storage: {res['trilinear_value']:.3e} replica-steps/s "
            f"({res['trilinear_vs_bspline']:.2f}x the B-spline), drift {drift_t}")
    if args.minima:
        from paper_2508_15522_amd import sampling as SM
        log("learned vs uniform proposals (minima found per second)")
        g32 = grid if args.storage == "f32" else setup(G.STORE_F32)
        cmp = SM.compare_learned_vs_uniform(g32, S.mol_chain24(), collect_minima=1_000_000, collect_rep=4096,
                                            train_steps=args.train_steps, eval_rounds=4, eval_rep=8192, log=log,
                                            weight_power=args.weight_power, imle_batch=args.imle_batch,
                                            imle_k=args.imle_k)
        for name in ("uniform", "learned"):
            log(f"{name} discovery curve (proposals, distinct minima, s): {cmp[name]['short_curve']}")
        res["minima_per_s"] = {"learned": cmp["learned"]["minima_per_s"], "uniform": cmp["uniform"]["minima_per_s"],
                               "gain": cmp["gain_minima_per_s"],
                               "flow_learned": cmp["learned"]["flow"]["minima_per_s"],
                               "flow_uniform": cmp["uniform"]["flow"]["minima_per_s"],
                               "flow_gain": cmp["gain_minima_per_s_flow"],
                               "gain_rmsd": cmp["gain_minima_per_s_rmsd"],
                               "flow_gain_rmsd": cmp["gain_minima_per_s_flow_rmsd"], "detail": cmp,
                               "workload": ("chain24 FIRE to 1e-4 eV/A (max 5000 steps), distinct within 0.01 eV; "
                                            "proposer trained on >= 1M converged minima of uniform rounds")}
        uc, lc = cmp["uniform"]["short_curve"], cmp["learned"]["short_curve"]
        rate = lambda c: c[1] / c[2]
        res["minima_per_s"]["short_horizon"] = {
            "proposals": [c[0] for c in uc], "uniform": [c[1] for c in uc], "learned": [c[1] for c in lc],
            "gain_first_round": rate(lc[0]) / rate(uc[0]), "gain_last_round": rate(lc[-1]) / rate(uc[-1])}
        res["minima_per_s"]["gain_with_training"] = _gain_with_training(cmp)
        # a landscape that does not saturate within the horizon: the 70-atom molecule of the
        # size series (seven rotatable torsions), proposer trained on 100k of its minima
        mol70 = [m for m in S.molecule_types("sizes") if m.n == 70][0]
        log("learned vs uniform proposals on the 70-atom molecule")
        c70 = SM.compare_learned_vs_uniform(g32, mol70, collect_minima=100_000, collect_rep=4096,
                                            train_steps=args.train_steps, eval_rounds=4, eval_rep=8192, log=log,
                                            weight_power=args.weight_power, imle_batch=args.imle_batch,
                                            imle_k=args.imle_k)
        res["minima_per_s_size70"] = {
            "learned": c70["learned"]["minima_per_s"], "uniform": c70["uniform"]["minima_per_s"],
            "gain": c70["gain_minima_per_s"], "flow_gain": c70["gain_minima_per_s_flow"],
            "gain_with_training": _gain_with_training(c70),
            "distinct": {"uniform": c70["uniform"]["distinct_minima"], "learned": c70["learned"]["distinct_minima"]},
            "distinct_rmsd": {"uniform": c70["uniform"]["distinct_minima_rmsd"],
                              "learned": c70["learned"]["distinct_minima_rmsd"]},
            "gain_rmsd": c70["gain_minima_per_s_rmsd"], "training": c70["training"],
            "workload": ("size-series 70-atom molecule (7 rotatable torsions), FIRE to 1e-4 eV/A (max 5000 steps), "
                         "4 x 8192 proposals per form, distinct within 0.01 eV; proposer trained on >= 100k "
                         "converged minima of uniform rounds")}
    if args.hopping:
        from paper_2508_15522_amd import sampling as SM
        log("minima hopping vs uniform proposals (minima found per second)")
        g32 = grid if args.storage == "f32" else setup(G.STORE_F32)
        hop = SM.compare_hopping_vs_uniform(g32, S.mol_chain24(), n_rep=4096, n_hops=4, log=log)
        res["minima_hopping"] = {k: {kk: v for kk, v in hop[k].items() if kk != "hops"} for k in hop}
        res["minima_hopping"]["workload"] = ("chain24, 4096 replicas: 1000 Langevin steps at 300 K (dt 0.5 fs, "
                                             "gamma 0.01/fs) then FIRE to 1e-4 eV/A (max 5000 steps), 4 hops "
                                             "after the initial relaxation; distinct within 0.01 eV / 0.1 A RMSD")
    if args.defect:
        res["defect_supercell"] = run_defect(log)
    if args.scans:
        res["restrained_scans"] = run_scans(grid if args.storage == "f32" else setup(G.STORE_F32), log)
    for extra in args.extra:
        res.setdefault("other_workloads", {})[extra] = run_workload(extra, log)
    for name in args.direct:
        res.setdefault("all_atom_comparison", {})[name] = run_direct(name, log)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(mol, cfg, args.cpu_seconds)
    print(json.dumps(res), flush=True)


def _gain_with_training(cmp):
    """Learned over uniform distinct minima per second in rounds, with the proposer's IMLE
    training time added to the learned form's GPU time (the collection of the training minima
    is uniform sampling and is not counted against either form)."""
    L, U = cmp["learned"], cmp["uniform"]
    return (L["distinct_minima"] / (L["seconds"] + cmp["training"]["train_s"])) / max(U["minima_per_s"], 1e-12)


def run_workload(name, log):
    """The other configurations, timed with HIP events around one relaxation launch."""
    import torch
    from paper_2508_15522_amd import autotune as AT, configs, device as D, gridff as G, synth as S
    wl = {"c1": configs.C1_CHAIN_FIRE, "c3": configs.C3_SIZES_FIRE, "c5": configs.C5_PAH_FIRE_LARGE}[name]
    cfg = wl.grid
    sub = cfg.substrate()
    spec = D.spec_for(cfg)
    t0 = time.time()
    grid = D.build_physical_grid(sub, spec, G.STORE_F32)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    mols = S.molecule_types(wl.molecules)
    rep_type = np.arange(wl.n_rep) % len(mols)
    pos = []
    for t, m in enumerate(mols):
        k = int((rep_type == t).sum())
        pos.append(S.place_replicas(m, k, sub, S.SEED_PLACE * (3 if name == "c3" else 1) + t))
    it = [iter(p) for p in pos]
    per_rep = [next(it[t]) for t in rep_type]
    topo = G.Topology(mols)
    prm = G.relax_params(G.MODE_FIRE, wl.n_steps, True, f_conv=1e-4)
    launch = (192, 0, 0)          # 8 x 24 or 5 x 38 atoms fill a 192-thread block
    tuned = None
    if name in ("c1", "c3"):      # small or mixed batches: the launch shape is measured
        plan0 = G.Plan(topo, rep_type)
        st = D.fire_state(plan0, per_rep)
        tune_prm = G.relax_params(G.MODE_FIRE, 50, True, f_conv=1e-4)
        launch, tuned = AT.launch_for(grid, topo, rep_type, tune_prm, st, use_cache=False)
        log(f"{name} autotuned launch {launch} ({tuned:.3e} replica-steps/s on 50 steps)")
    plan = G.Plan(topo, rep_type, *launch)
    st = D.fire_state(plan, per_rep)
    out = D.outputs(plan)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0.record(stream)
    G.relax_batch(grid.desc, topo, plan, prm, st, out["E"], out["fnorm"], out["steps"], None, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    steps = out["steps"].cpu().numpy()
    status = st["status"].cpu().numpy()
    moves = int(steps.sum())
    r = {"workload": wl.name, "replicas": wl.n_rep, "types": [m.n for m in mols], "max_steps": wl.n_steps,
         "seconds": secs, "replica_steps_per_s_moves": moves / secs,
         "replica_steps_per_s_launch": wl.n_rep * wl.n_steps / secs,
         "converged": int(((status & G.REP_CONVERGED) != 0).sum()), "grid_build_fit_s": build_s,
         "grid": f"{cfg.nx}x{cfg.ny}x{cfg.nz}x3 f32", "substrate_atoms": sub.n, "launch": list(launch)}
    if tuned is not None:
        r["autotune_rate"] = tuned
    log(f"{name}: {r}")
    return r


def run_scans(grid, log, n_paths=4096):
    """Restrained scans of pah38 (one rim O atom held) on the small slab, every path a
    replica: a relaxed detachment (held atom lifted from 1.3 to 20 A above the top plane in
    0.1 A steps, FIRE to 1e-3 eV/A, at most 5000 moves per point) and a drag along the cell
    diagonal at 3.3 A (0.1 A steps over one diagonal period, 5000 moves per point with a
    force threshold of 0 so that every point takes all of them, the paper's timing
    protocol).  Each scan is one fused launch (gff_relax_scan); the detachment is also run
    point by point (one launch per point) for comparison.  Wall time of the whole scan.
    The detachment runs two lanes per atom in 256-thread blocks: its paths need very
    different numbers of moves, its wall time is that of the slowest path, and two lanes
    per atom shorten a lone block's move; the drag, where every path takes every move, runs
    one lane per atom in 192-thread blocks, the throughput layout."""
    import torch
    from paper_2508_15522_amd import device as D, gridff as G, scans as SC, synth as S
    mol = S.mol_pah38()
    topo = G.Topology([mol])
    plan = G.Plan(topo, np.zeros(n_paths, np.int32), block_threads=192)
    plan_lat = G.Plan(topo, np.zeros(n_paths, np.int32), block_threads=256, lanes_per_atom=2)
    sub = S.rocksalt_slab(2, 3)
    start = list(S.f32(S.place_replicas(mol, n_paths, sub, S.SEED_PLACE * 7, h_range=(3.0, 3.5))))
    held = np.full(n_paths, mol.elem.index("O"), np.int32)
    out = {}
    z = 1.3 + 0.1 * np.arange(188)
    tg = SC.detachment_targets(start, held, z)
    for name, fn in (("detachment", SC.restrained_scan_fused), ("detachment_point_by_point", SC.restrained_scan)):
        r = fn(grid, topo, plan_lat, start, held, tg, f_conv=1e-3, max_steps=5000)
        moves = int(r["steps"].sum())
        out[name] = {"paths": n_paths, "points": len(z), "launch": [256, 0, 0, 2], "seconds": r["seconds"],
                     "scan_points_per_s": n_paths * len(z) / r["seconds"], "replica_steps_per_s": moves / r["seconds"],
                     "mean_moves_per_point": moves / (n_paths * len(z)),
                     "converged_fraction": float(((r["status"] & G.REP_CONVERGED) != 0).mean())}
        log(f"{name} scan: {out[name]}")
    L = np.hypot(sub.Lx, sub.Ly) / 2                     # one period along the diagonal
    npts = int(round(L / 0.1)) + 1
    tg = SC.drag_targets(start, held, (1.0, 1.0), 0.1, npts, height=3.3)
    r = SC.restrained_scan_fused(grid, topo, plan, start, held, tg, f_conv=0.0, max_steps=5000)
    moves = int(r["steps"].sum())
    out["drag"] = {"paths": n_paths, "points": npts, "launch": [192, 0, 0, 1], "seconds": r["seconds"],
                   "scan_points_per_s": n_paths * npts / r["seconds"], "replica_steps_per_s": moves / r["seconds"],
                   "moves_per_point": moves / (n_paths * npts)}
    log(f"drag scan: {out['drag']}")
    out["workload"] = ("pah38 on the 2x2x3 slab (112x112x150 FP32 grid), 4096 paths, one rim O held: "
                       "detachment 1.3-20 A (188 points, FIRE to 1e-3 eV/A, <= 5000 moves; two lanes per atom); "
                       "drag along the diagonal at 3.3 A, 0.1 A steps, 5000 moves per point (one lane per atom)")
    return out


def run_defect(log, n_paths=512, n_points=200):
    """The dragging-over-a-defect case on a large supercell grid: build (FP64 sums, fit, FP32
    pack) of the 20x20x3 slab with a vacancy pair and of the pristine slab, then the same
    batched drag on both: pah38 (random orientation, lowest atom 3-3.5 A above the top plane)
    with a rim O held at its start height, dragged 20 A along the cell diagonal across the
    defect (paths offset sideways by up to 3 A), FIRE to 1e-3 eV/A with at most 2000 moves
    per point.  Pinning: per path
    the lowest energy along the defect run minus the lowest along the pristine run."""
    import torch
    from paper_2508_15522_amd import configs, device as D, gridff as G, scans as SC, synth as S
    out = {}
    mol = S.mol_pah38()
    topo = G.Topology([mol])
    # 512 paths of 38 atoms leave most of the GPU idle at one lane per atom: four lanes per atom
    plan = G.Plan(topo, np.zeros(n_paths, np.int32), block_threads=256, lanes_per_atom=4)
    held = np.full(n_paths, mol.elem.index("O"), np.int32)
    rng = np.random.default_rng(77)
    cfg = configs.GRID_DEFECT
    c = np.array([cfg.n_cells * S.SLAB_A / 2 + S.SLAB_A / 4, cfg.n_cells * S.SLAB_A / 2])   # between the two vacancies
    d = np.array([1.0, 1.0]) / np.sqrt(2.0)
    perp = np.array([1.0, -1.0]) / np.sqrt(2.0)
    probe = S.rocksalt_slab(2, 3)
    start = []
    for k, base in enumerate(S.place_replicas(mol, n_paths, probe, S.SEED_PLACE * 9, h_range=(3.0, 3.5))):
        x = base.copy()
        p0 = c - 10.0 * d + rng.uniform(-3.0, 3.0) * perp
        x[:, :2] += p0 - x[held[k], :2]
        start.append(S.f32(x))
    tg = SC.drag_targets(start, held, (1.0, 1.0), 0.1, n_points)    # at each held atom's start height
    E = {}
    for name, gcfg in (("defect", cfg), ("pristine", configs.GRID_DEFECT_PRISTINE)):
        sub = gcfg.substrate()
        spec = D.spec_for(gcfg)
        torch.cuda.synchronize()
        t0 = time.time()
        grid = D.build_physical_grid(sub, spec, G.STORE_F32)
        torch.cuda.synchronize()
        bsec = time.time() - t0
        r = SC.restrained_scan_fused(grid, topo, plan, start, held, tg, f_conv=1e-3, max_steps=2000)
        E[name] = r["E"]
        moves = int(r["steps"].sum())
        out[name] = {"substrate_atoms": sub.n, "grid": f"{spec.nx}x{spec.ny}x{spec.nz}x3 f32",
                     "grid_bytes": G.grid_bytes(spec, G.STORE_F32), "build_fit_pack_s": bsec,
                     "scan_seconds": r["seconds"], "replica_steps_per_s": moves / r["seconds"],
                     "converged_fraction": float(((r["status"] & G.REP_CONVERGED) != 0).mean())}
        log(f"defect supercell ({name}): {out[name]}")
        del grid
        torch.cuda.empty_cache()
    pin = E["defect"].min(1) - E["pristine"].min(1)
    out["pinning_eV"] = {"mean": float(pin.mean()), "min": float(pin.min()), "max": float(pin.max())}
    out["profile_mean_eV"] = {"defect": [float(v) for v in E["defect"].mean(0)[::10]],
                              "pristine": [float(v) for v in E["pristine"].mean(0)[::10]]}
    out["workload"] = (f"pah38, {n_paths} paths, one rim O held at its start height, dragged 20 A along "
                       f"the diagonal across the defect in 0.1 A steps ({n_points} points), FIRE to 1e-3 eV/A "
                       "(<= 2000 moves per point)")
    log(f"defect pinning: {out['pinning_eV']}")
    return out


def run_direct(name, log):
    """GridFF against the all-atom comparison mode on the same replicas, molecule and
    integrator (C2: NVE on the 48-atom slab; C5: FIRE on the 3072-atom slab): replica-steps/s
    of each over a short launch (HIP events) and their ratio."""
    import torch
    from paper_2508_15522_amd import configs, device as D, gridff as G, synth as S
    wl = {"c2": configs.C2_PAH_NVE, "c5": configs.C5_PAH_FIRE_LARGE}[name]
    cfg = wl.grid
    sub = cfg.substrate()
    mol = S.mol_pah38()
    grid = D.build_physical_grid(sub, D.spec_for(cfg), G.STORE_F32)
    direct = G.Direct(sub, cfg.alpha, 1)
    topo = G.Topology([mol])
    plan = G.Plan(topo, np.zeros(wl.n_rep, np.int32), block_threads=192)
    pos = S.place_replicas(mol, wl.n_rep, sub, S.SEED_PLACE * (2 if name == "c2" else 1))
    if name == "c2":
        vel = S.mb_velocities(mol.mass, wl.n_rep, 300.0, S.SEED_NVE)
        prm = G.relax_params(G.MODE_NVE, 200, True, dt=0.5, drift_every=1)
        steps = 200
    else:
        vel = None
        prm = G.relax_params(G.MODE_FIRE, 10, True, f_conv=1e-4)
        steps = 10
    out = D.outputs(plan)
    stream = torch.cuda.current_stream()

    def timed(fn):
        st = D.fire_state(plan, pos, vel_per_rep=vel)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn(st)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    drift = out["drift"] if name == "c2" else None
    grid_run = lambda st: G.relax_batch(grid.desc, topo, plan, prm, st, out["E"], out["fnorm"], out["steps"],
                                        drift, stream)
    direct_run = lambda st: G.relax_batch_direct(direct, topo, plan, prm, st, out["E"], out["fnorm"],
                                                 out["steps"], drift, stream)
    timed(grid_run)
    tg = timed(grid_run)
    timed(direct_run)
    td = timed(direct_run)
    r = {"workload": wl.name, "substrate_atoms": sub.n, "substrate_terms_per_atom": 9 * sub.n, "steps": steps,
         "gridff_replica_steps_per_s": wl.n_rep * steps / tg, "all_atom_replica_steps_per_s": wl.n_rep * steps / td,
         "gridff_speedup": td / tg}
    log(f"all-atom comparison {name}: {r}")
    return r


def gather_probe(grid, log, reps=10):
    """Random 64-byte-chunk gather bandwidth (gff_gather_probe) on three working sets: the
    grid's own coefficient buffer (the interpolation's working set), 4 MiB (one XCD's L2) and
    4 GiB (beyond the Infinity Cache: HBM).  GB/s, median of `reps` calls timed with HIP
    events on the launch stream."""
    import torch
    from paper_2508_15522_amd import gridff as G
    n_threads, iters = 256 * 2048, 64
    sink = torch.empty(n_threads, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    moved = n_threads * iters * 16
    out = {"unit": "GB/s", "chunk_bytes": 64, "bytes_per_call": moved}
    bufs = {"grid_coefficients": grid.coef.view(torch.uint8),
            "l2_4MiB": torch.zeros(4 << 20, dtype=torch.uint8, device="cuda"),
            "hbm_4GiB": torch.zeros(4 << 30, dtype=torch.uint8, device="cuda")}
    for name, buf in bufs.items():
        nbytes = buf.numel() // 64 * 64
        b = buf[:nbytes]
        G.gather_probe(b, n_threads, iters, 1, sink, stream)                 # warm-up
        times = []
        for r in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            G.gather_probe(b, n_threads, iters, 2 + r, sink, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        out[name] = moved / float(np.median(times)) / 1e9
        out[name + "_bytes"] = nbytes
        log(f"gather probe {name} ({nbytes / 2**20:.1f} MiB): {out[name]:.0f} GB/s")
    del bufs
    return out


def cpu_baseline(mol, cfg, budget_s):
    """The FP64 oracle on the host cores: NVE of the same molecule on a grid of the same
    size (random coefficients from the seeded generator -- the oracle's cost does not
    depend on the coefficient values), on a bounded sample of replicas and steps."""
    import oracle as O
    from paper_2508_15522_amd import synth as S
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    B = S.random_coefficients(cfg.nx, cfg.ny, cfg.nz, 1, (1e-3, 1e-2, 1e-1))
    geo = dict(nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, x0=0.0, y0=0.0, z0=cfg.z0, dx=2 * S.SLAB_A / cfg.nx,
               dy=2 * S.SLAB_A / cfg.ny, dz=cfg.dz)
    sub = S.rocksalt_slab(2, 3)
    # calibrate on the workload's replica count (large enough that thread start-up and the
    # per-call set-up do not dominate), then fill the budget with MD steps
    # (a call with s steps evaluates forces s + 1 times, so the cost of one step is the
    # difference between a 3-step and a 1-step call)
    n_rep = 16384
    el = {}
    for n_steps in (1, 3):
        pos = S.place_replicas(mol, n_rep, sub, 77).reshape(-1, 3)
        vel = S.mb_velocities(mol.mass, n_rep, 300.0, 7).reshape(-1, 3)
        t = time.time()
        O.nve_batch(B, geo, [mol], np.zeros(n_rep, np.int32), pos, vel, n_steps)
        el[n_steps] = time.time() - t
    per = max((el[3] - el[1]) / 2, el[3] / 8, 1e-4) / n_rep
    n_steps = int(max(2, min(5000, budget_s / (per * n_rep))))
    pos = S.place_replicas(mol, n_rep, sub, 78).reshape(-1, 3)
    vel = S.mb_velocities(mol.mass, n_rep, 300.0, 8).reshape(-1, 3)
    t = time.time()
    O.nve_batch(B, geo, [mol], np.zeros(n_rep, np.int32), pos, vel, n_steps)
    el = time.time() - t
    # one thread, on 1024 replicas for about a third of the budget
    n1 = 1024
    prev = O.set_threads(1)
    try:
        steps1 = int(max(2, min(5000, budget_s / 3 / (per * max(threads, 1) * n1))))
        t = time.time()
        O.nve_batch(B, geo, [mol], np.zeros(n1, np.int32), pos[:n1 * mol.n], vel[:n1 * mol.n], steps1)
        el1 = time.time() - t
    finally:
        O.set_threads(prev)
    # the oracle's molecule-substrate part alone, B-spline model against the all-atom direct
    # sum over the cell and its 8 lateral images, on the same atoms (all threads)
    plq = np.tile(O.mixing(mol.eps, mol.R, mol.q), (n_rep, 1))
    pts = pos.reshape(-1, 3)
    rates = {}
    for name, fn in (("bspline", lambda p, q: O.bspline_eval(B, geo, p, q)),
                     ("all_atom", lambda p, q: O.direct_images(sub, p, q, nimg=1))):
        n_pts = 4096
        while True:
            t = time.time()
            fn(pts[:n_pts], plq[:n_pts])
            dt = time.time() - t
            if dt > budget_s / 20 or n_pts >= len(pts):
                break
            n_pts = min(len(pts), n_pts * 4)
        rates[name] = {"atom_evaluations_per_s": n_pts / dt, "sample": f"{n_pts} atoms, {dt:.2f} s"}
    rates["substrate_terms_per_atom"] = int(sub.n * 9)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": n_rep * n_steps / el, "unit": "replica-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_rep} replicas x {n_steps} NVE steps of the 38-atom molecule, FP64 B-spline model + "
                      f"intramolecular field, {el:.1f} s",
            "one_thread": {"value": n1 * steps1 / el1, "sample": f"{n1} replicas x {steps1} steps, {el1:.1f} s"},
            "grid_vs_all_atom": rates, "cpu_model": model, "nproc": os.cpu_count()}


if __name__ == "__main__":
    main()
