"""Configuration sampling: minima hopping, uniform or learned proposals (host orchestration only).

Minima hopping (Section "Configuration sampling on GPU"): every replica starts from a relaxed
uniform proposal; each hop runs Langevin dynamics at 300 K from the replica's last minimum,
relaxes with FIRE to |F| < f_conv and deduplicates the converged minima; replicas continue
from their new minimum (from the previous one if the relaxation did not converge).
Proposal rounds: proposals (uniform Philox DOF, or the MLP's output from Philox noise,
decoded) -> poses -> FIRE relaxation in one persistent launch -> dedupe.  Every converged
minimum is deduplicated twice, by energy (0.01 eV) and by the lattice-translated RMSD
(0.1 A), against the archive of the run.
Training (IMLE): the distinct minima are encoded; for each training minimum K noise rows
are decoded by the network, the nearest output is kept and a step on it follows.
Every numerical step is a libgridff call; this module only sequences them.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import device as D, gridff as G, synth as S

H_LO, H_HI = 3.0, 5.0            # uniform proposals: height of the lowest atom (A)
DEC_LO, DEC_HI = 1.0, 8.0        # learned proposals: heights outside this range are clamped


RMSD_TOL = 0.1                   # A, the paper's uniqueness threshold
E_TOL = 0.01                     # eV


@dataclass
class Archive:
    """Distinct minima found so far: energies (energy criterion) and coordinates with their
    centroids (RMSD criterion), on the device."""
    capacity: int = 200000
    max_atoms: int = 128
    rmsd_capacity: int = 50000
    E: torch.Tensor = None
    types: torch.Tensor = None
    n: torch.Tensor = None

    def __post_init__(self):
        self.E = torch.zeros(self.capacity, dtype=torch.float64, device="cuda")
        self.types = torch.zeros(self.capacity, dtype=torch.int32, device="cuda")
        self.n = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.pos = torch.zeros(self.rmsd_capacity, self.max_atoms, 3, device="cuda")
        self.cen = torch.zeros(self.rmsd_capacity, 3, dtype=torch.float64, device="cuda")
        self.rtypes = torch.zeros(self.rmsd_capacity, dtype=torch.int32, device="cuda")
        self.rn = torch.zeros(1, dtype=torch.int32, device="cuda")

    def count(self):
        return int(self.n.item())

    def count_rmsd(self):
        return int(self.rn.item())


@dataclass
class RoundStats:
    proposals: int
    converged: int
    new_minima: int
    fire_steps_converged: float
    seconds: float
    rms_move_converged: float = float("nan")   # mean over converged replicas of the RMS atom move (A)
    new_pos: list = field(default_factory=list)
    new_minima_rmsd: int = 0


class Sampler:
    def __init__(self, grid, mol, n_rep, f_conv=1e-4, max_steps=5000, seed=S.SEED_PHILOX, block=256):
        self.grid, self.mol, self.n_rep = grid, mol, n_rep
        self.topo = G.Topology([mol])
        self.plan = G.Plan(self.topo, np.zeros(n_rep, np.int32), block_threads=block)
        self.T = len(mol.rot_quads)
        self.f_conv, self.max_steps, self.seed = f_conv, max_steps, seed
        self.Lx, self.Ly = grid.Lx, grid.Ly
        self.dof = torch.empty(n_rep, 7 + self.T, device="cuda")
        self.types = torch.zeros(n_rep, dtype=torch.int32, device="cuda")
        self.ntors = torch.full((n_rep,), self.T, dtype=torch.int32, device="cuda")
        self.is_new = torch.empty(n_rep, dtype=torch.int32, device="cuda")
        self.is_new_rmsd = torch.empty(n_rep, dtype=torch.int32, device="cuda")
        self.rmsd_work = torch.empty(max(G.dedupe_rmsd_workspace_bytes(n_rep), 1), dtype=torch.uint8, device="cuda")
        self.out = D.outputs(self.plan)

    def _dedupe(self, archive, pos, ok):
        """Energy and RMSD dedupe of the replicas flagged in ok (device int32 [n_rep]);
        returns the two counts of new minima."""
        G.dedupe_energy(self.out["E"], self.types, ok, E_TOL, archive.capacity, archive.E, archive.types, archive.n,
                        self.is_new)
        G.dedupe_rmsd(self.plan, pos, ok, RMSD_TOL, self.Lx, self.Ly, archive.rmsd_capacity, archive.max_atoms,
                      archive.pos, archive.cen, archive.rtypes, archive.rn, self.is_new_rmsd, self.rmsd_work)
        return int(self.is_new.sum().item()), int(self.is_new_rmsd.sum().item())

    def _relax_and_dedupe(self, archive, keep_new):
        st = {"pos": torch.empty(3, self.plan.n_atoms, device="cuda"),
              "vel": torch.zeros(3, self.plan.n_atoms, device="cuda"),
              "fire_dt": torch.full((self.n_rep,), 0.05, device="cuda"),
              "fire_alpha": torch.full((self.n_rep,), 0.1, device="cuda"),
              "fire_npos": torch.zeros(self.n_rep, dtype=torch.int32, device="cuda"),
              "status": torch.zeros(self.n_rep, dtype=torch.int32, device="cuda")}
        G.pose_from_dof(self.topo, self.plan, self.dof, 7 + self.T, self.Lx, self.Ly, 0.0, st["pos"])
        pos0 = st["pos"].clone()
        prm = G.relax_params(G.MODE_FIRE, self.max_steps, True, f_conv=self.f_conv)
        G.relax_batch(self.grid.desc, self.topo, self.plan, prm, st, self.out["E"], self.out["fnorm"],
                      self.out["steps"])
        ok = ((st["status"] & G.REP_CONVERGED) != 0).to(torch.int32)
        _, self._last_new_rmsd = self._dedupe(archive, st["pos"], ok)
        torch.cuda.synchronize()
        okh = ok.cpu().numpy().astype(bool)
        steps = self.out["steps"].cpu().numpy()
        newh = self.is_new.cpu().numpy().astype(bool)
        kept = [st["pos"].clone(), self.out["E"].cpu().numpy()] if keep_new else []
        # how far relaxation moved each replica: RMS over its atoms of |x_min - x_proposed|
        d2 = ((st["pos"] - pos0) ** 2).sum(0).cpu().numpy().astype(np.float64)
        off = self.plan.atom_off
        rms = np.sqrt(np.add.reduceat(d2, off[:-1]) / np.diff(off))
        move = float(rms[okh].mean()) if okh.any() else float("nan")
        return okh, steps, newh, kept, move

    def round_uniform(self, archive, rnd, keep_new=False):
        t0 = time.time()
        G.propose_uniform(self.n_rep, self.T, self.seed, rnd, H_LO, H_HI, self.dof)
        okh, steps, newh, kept, move = self._relax_and_dedupe(archive, keep_new)
        rs = RoundStats(self.n_rep, int(okh.sum()), int(newh.sum()),
                        float(steps[okh].mean()) if okh.any() else float("nan"), time.time() - t0, move)
        rs.new_pos = [(kept[0], newh, okh, kept[1])] if keep_new else []
        rs.new_minima_rmsd = self._last_new_rmsd
        return rs

    def round_learned(self, archive, mlp, rnd):
        t0 = time.time()
        noise = torch.empty(self.n_rep, 64, device="cuda")
        G.normal_philox(self.n_rep * 64, self.seed + 1, rnd, noise)
        enc = torch.empty(self.n_rep, 41, device="cuda")
        mlp.forward(noise, self.types, enc)
        G.decode_dof(enc, self.T, DEC_LO, DEC_HI, self.dof)
        okh, steps, newh, _, move = self._relax_and_dedupe(archive, False)
        return RoundStats(self.n_rep, int(okh.sum()), int(newh.sum()),
                          float(steps[okh].mean()) if okh.any() else float("nan"), time.time() - t0, move,
                          new_minima_rmsd=self._last_new_rmsd)

    # ---------------------------------------------------------------- minima hopping
    def minima_hopping(self, archive, n_hops, md_steps=1000, T=300.0, gamma=0.01, dt=0.5, log=None, keep=False):
        """The paper's sampler on all n_rep replicas at once.  Hop 0 relaxes uniform
        proposals; hop h >= 1 restores every replica to its last minimum, runs md_steps of
        Langevin dynamics at T (friction gamma [1/fs], step dt [fs], Philox round h) in one
        launch, relaxes with FIRE (max_steps moves, |F| < f_conv) in one launch and
        deduplicates the converged minima by energy and by RMSD.  Converged replicas move
        their base to the new minimum.  Returns per-hop dicts of counts and wall times; with
        keep=True also each hop's starting positions, positions after the dynamics, relaxed
        positions and status (host)."""
        n = self.n_rep
        say = log or (lambda m: None)
        st = {"pos": torch.empty(3, self.plan.n_atoms, device="cuda"),
              "vel": torch.zeros(3, self.plan.n_atoms, device="cuda"),
              "fire_dt": torch.full((n,), 0.05, device="cuda"),
              "fire_alpha": torch.full((n,), 0.1, device="cuda"),
              "fire_npos": torch.zeros(n, dtype=torch.int32, device="cuda"),
              "status": torch.zeros(n, dtype=torch.int32, device="cuda")}
        base = {"pos": torch.empty_like(st["pos"]), "vel": torch.empty_like(st["vel"]),
                "status": torch.empty_like(st["status"])}
        all1 = torch.ones(n, dtype=torch.int32, device="cuda")
        p_md = G.relax_params(G.MODE_LANGEVIN, md_steps, True, dt=dt, T=T, gamma=gamma, seed=self.seed)
        p_fire = G.relax_params(G.MODE_FIRE, self.max_steps, True, f_conv=self.f_conv)
        hops = []
        for h in range(n_hops + 1):
            t0 = time.time()
            kept = {"base_in": D.unsoa(self.plan, base["pos"])} if keep and h > 0 else {}
            if h == 0:
                G.propose_uniform(n, self.T, self.seed, 0, H_LO, H_HI, self.dof)
                G.pose_from_dof(self.topo, self.plan, self.dof, 7 + self.T, self.Lx, self.Ly, 0.0, st["pos"])
            else:
                G.refill(self.plan, all1, base["pos"], st)          # back to the last minimum, v = 0
                p_md.round = h
                G.relax_batch(self.grid.desc, self.topo, self.plan, p_md, st, self.out["E"], self.out["fnorm"],
                              self.out["steps"])
                if keep:
                    kept["md_out"] = D.unsoa(self.plan, st["pos"])
                G.refill(self.plan, all1, st["pos"], st)            # keep positions, reset FIRE state
            G.relax_batch(self.grid.desc, self.topo, self.plan, p_fire, st, self.out["E"], self.out["fnorm"],
                          self.out["steps"])
            ok = ((st["status"] & G.REP_CONVERGED) != 0).to(torch.int32)
            new_e, new_r = self._dedupe(archive, st["pos"], ok)
            if keep:
                kept.update(pos_out=D.unsoa(self.plan, st["pos"]), status=st["status"].cpu().numpy())
            # converged replicas continue from the new minimum (hop 0: every replica)
            G.refill(self.plan, all1 if h == 0 else ok, st["pos"], base)
            torch.cuda.synchronize()
            conv = int(ok.sum().item())
            hops.append(dict(hop=h, converged=conv, new_minima=new_e, new_minima_rmsd=new_r,
                             seconds=time.time() - t0, **kept))
            say(f"hop {h}: converged {conv}/{n}, new {new_e} (energy) {new_r} (rmsd), {time.time() - t0:.2f} s")
        return hops

    # ---------------------------------------------------------------- continuous flow
    def propose_uniform_rows(self, rnd):
        G.propose_uniform(self.n_rep, self.T, self.seed, rnd, H_LO, H_HI, self.dof)

    def propose_learned_rows(self, mlp):
        noise = torch.empty(self.n_rep, 64, device="cuda")
        enc = torch.empty(self.n_rep, 41, device="cuda")

        def fill(rnd):
            G.normal_philox(self.n_rep * 64, self.seed + 1, rnd, noise)
            mlp.forward(noise, self.types, enc)
            G.decode_dof(enc, self.T, DEC_LO, DEC_HI, self.dof)
        return fill

    def flow(self, archive, n_proposals, propose, chunk=250, record=False):
        """Continuous-flow relaxation of n_proposals proposals through the n_rep slots:
        FIRE launches of `chunk` steps continue every slot's state; between launches the
        slots whose proposal converged, went non-finite or used its max_steps budget are
        harvested (converged minima deduplicated into `archive`) and refilled with new
        proposals (`propose(rnd)` fills self.dof for every slot; the refilled slots take
        their rows).  Each proposal follows the trajectory one uninterrupted launch of
        max_steps would give it (max_steps must be a multiple of chunk).  Returns a dict of
        counts and the wall time; with record=True also each harvested proposal's DOF row,
        energy, convergence flag and move count."""
        assert self.max_steps % chunk == 0
        n = self.n_rep
        t0 = time.time()
        st = {"pos": torch.empty(3, self.plan.n_atoms, device="cuda"),
              "vel": torch.zeros(3, self.plan.n_atoms, device="cuda"),
              "fire_dt": torch.full((n,), 0.05, device="cuda"),
              "fire_alpha": torch.full((n,), 0.1, device="cuda"),
              "fire_npos": torch.zeros(n, dtype=torch.int32, device="cuda"),
              "status": torch.zeros(n, dtype=torch.int32, device="cuda")}
        pos_new = torch.empty_like(st["pos"])
        rnd = 0
        propose(rnd)
        G.pose_from_dof(self.topo, self.plan, self.dof, 7 + self.T, self.Lx, self.Ly, 0.0, st["pos"])
        dof_slot = self.dof.cpu().numpy().copy() if record else None
        active = np.ones(n, bool)
        if n_proposals < n:
            active[n_proposals:] = False
        issued = int(active.sum())
        moves = np.zeros(n, np.int64)
        mode = torch.zeros(n, dtype=torch.int32, device="cuda")
        if not active.all():
            mode.copy_(torch.from_numpy(np.where(active, 0, 2).astype(np.int32)))
            G.refill(self.plan, mode, st["pos"], st)
        prm = G.relax_params(G.MODE_FIRE, chunk, True, f_conv=self.f_conv)
        conv_total, new_total, new_rmsd_total, done_total, steps_conv, rec = 0, 0, 0, 0, [], []
        launches = 0
        while active.any():
            G.relax_batch(self.grid.desc, self.topo, self.plan, prm, st, self.out["E"], self.out["fnorm"],
                          self.out["steps"])
            launches += 1
            status = st["status"].cpu().numpy()
            moves += np.where(active, self.out["steps"].cpu().numpy(), 0)
            conv = active & ((status & G.REP_CONVERGED) != 0)
            done = active & (conv | ((status & G.REP_NONFINITE) != 0) | (moves >= self.max_steps))
            if not done.any():
                continue
            ok = torch.from_numpy(conv.astype(np.int32)).cuda()
            ne, nr = self._dedupe(archive, st["pos"], ok)
            new_total += ne
            new_rmsd_total += nr
            conv_total += int(conv.sum()); done_total += int(done.sum())
            steps_conv += list(moves[conv])
            if record:
                E = self.out["E"].cpu().numpy()
                for k in np.where(done)[0]:
                    rec.append((dof_slot[k].copy(), float(E[k]), bool(conv[k]), int(moves[k])))
            idx = np.where(done)[0]
            take = idx[:max(0, min(len(idx), n_proposals - issued))]
            m = np.zeros(n, np.int32)
            m[idx] = 2
            if len(take):
                rnd += 1
                propose(rnd)
                G.pose_from_dof(self.topo, self.plan, self.dof, 7 + self.T, self.Lx, self.Ly, 0.0, pos_new)
                m[take] = 1
                if record:
                    rows = self.dof.cpu().numpy()
                    dof_slot[take] = rows[take]
                issued += len(take)
            mode.copy_(torch.from_numpy(m))
            G.refill(self.plan, mode, pos_new, st)
            moves[idx] = 0
            active[idx] = False
            active[take] = True
        torch.cuda.synchronize()
        res = dict(proposals=done_total, converged=conv_total, new_minima=new_total, new_minima_rmsd=new_rmsd_total,
                   seconds=time.time() - t0,
                   launches=launches, mean_steps_converged=float(np.mean(steps_conv)) if steps_conv else float("nan"))
        if record:
            res["records"] = rec
        return res

    def encode_minima(self, pos, mask):
        """Encodings [m][41] of the replicas selected by mask (host bool array)."""
        work = torch.empty_like(pos)
        enc = torch.empty(self.n_rep, 41, device="cuda")
        G.encode_pose(self.topo, self.plan, pos, self.Lx, self.Ly, 0.0, work, enc)
        idx = torch.from_numpy(np.where(mask)[0]).cuda()
        return enc.index_select(0, idx)


def train_imle(mlp, targets, ntors, types, steps, batch=1024, K=64, lr=1e-3, seed=S.SEED_MLP, log=None,
               weights=None):
    """IMLE training on encoded minima (device tensors targets [m][41], ntors [m], types [m]);
    batches draw minima with probabilities proportional to `weights` (host, default uniform)."""
    m = targets.shape[0]
    rng = np.random.default_rng(seed)
    cdf = None if weights is None else np.cumsum(np.asarray(weights, np.float64))
    cand_noise = torch.empty(batch * K, 64, device="cuda")
    cand_out = torch.empty(batch * K, 41, device="cuda")
    best = torch.empty(batch, dtype=torch.int32, device="cuda")
    sel_noise = torch.empty(batch, 64, device="cuda")
    out = torch.empty(batch, 41, device="cuda")
    loss = torch.empty(batch, device="cuda")
    hist = []
    # every step's batch drawn up front and copied once, so that the loop queues work without
    # waiting for the device
    if cdf is None:
        picks = rng.integers(0, m, (steps, batch))
    else:
        picks = np.minimum(np.searchsorted(cdf, rng.random((steps, batch)) * cdf[-1], side="right"), m - 1)
    picks = torch.from_numpy(np.ascontiguousarray(picks, np.int64)).cuda()
    for s in range(steps):
        idx = picks[s]
        tg = targets.index_select(0, idx).contiguous()
        nt = ntors.index_select(0, idx).contiguous()
        ty = types.index_select(0, idx).contiguous()
        G.normal_philox(batch * K * 64, seed, s, cand_noise)
        ty_rep = ty.repeat_interleave(K).contiguous()
        mlp.forward(cand_noise, ty_rep, cand_out)
        G.imle_select(cand_out.view(batch, K, 41), tg, nt, best)
        G.gather_rows(cand_noise.view(batch * K, 64), K, best, sel_noise)
        mlp.train_step(sel_noise, ty, tg, nt, lr, out, loss)
        if s % 50 == 0 or s == steps - 1:
            torch.cuda.synchronize()
            hist.append((s, float(loss.mean().item())))
            if log:
                log(f"imle step {s}: loss {hist[-1][1]:.4f}")
    return hist


def compare_learned_vs_uniform(grid, mol, collect_minima=50_000, collect_rep=4096, train_steps=400, eval_rounds=6,
                               eval_rep=1024, seed=S.SEED_PHILOX, log=None, max_collect_rounds=4000,
                               weight_power=1.0, short_rep=512, short_rounds=8, imle_batch=1024, imle_k=64):
    """Collect at least collect_minima converged minima with rounds of uniform proposals,
    train the proposer on every converged minimum (the relaxed poses the method generated),
    a minimum of an energy class with c members weighted c^-weight_power (1: every distinct
    minimum the same total weight, 0: every minimum the same weight), then run equal numbers
    of proposals with each
    method against fresh archives.  Returns a dict of counts, wall times, minima/s, mean FIRE
    steps and mean RMS relaxation move per converged minimum, and for each form the curve
    (proposals, distinct minima, seconds) over short_rounds rounds of short_rep proposals."""
    say = log or (lambda m: None)
    col = Sampler(grid, mol, collect_rep, seed=seed)
    arch = Archive(max_atoms=mol.n)
    targets, energies = [], []
    t0 = time.time()
    got, r = 0, 0
    while got < collect_minima and r < max_collect_rounds:
        rs = col.round_uniform(arch, r, keep_new=True)
        pos, newh, okh, E = rs.new_pos[0]
        if okh.any():
            targets.append(col.encode_minima(pos, okh))
            energies.append(E[okh])
        got += rs.converged
        if r % 25 == 0:
            say(f"collect round {r}: converged {rs.converged}/{rs.proposals}, new {rs.new_minima}, "
                f"mean steps {rs.fire_steps_converged:.0f}, {rs.seconds:.2f} s; {got} minima so far")
        r += 1
    collect_s, collect_rounds = time.time() - t0, r
    tg = torch.cat(targets, 0).contiguous()
    m = tg.shape[0]
    ntors = torch.full((m,), len(mol.rot_quads), dtype=torch.int32, device="cuda")
    types = torch.zeros(m, dtype=torch.int32, device="cuda")
    # each distinct minimum (energy cluster of the archive) gets the same total weight, spread
    # over its converged members: frequent basins do not crowd out rare ones
    E = np.concatenate(energies)
    aE = arch.E[:arch.count()].cpu().numpy()
    order = np.argsort(aE)
    sE = aE[order]
    if len(sE) == 1:
        cl = np.zeros(len(E), np.int64)
    else:                                                            # nearest archived energy
        hi = np.clip(np.searchsorted(sE, E), 1, len(sE) - 1)
        cl = order[np.where(np.abs(E - sE[hi - 1]) <= np.abs(E - sE[hi]), hi - 1, hi)]
    w = np.bincount(cl, minlength=len(aE))[cl].astype(np.float64) ** -weight_power
    mlp = G.MLP(1, S.mlp_init_params(1))
    t0 = time.time()
    hist = train_imle(mlp, tg, ntors, types, train_steps, batch=min(imle_batch, max(64, m)), K=imle_k, log=say,
                      weights=w)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    ev = Sampler(grid, mol, eval_rep, seed=seed + 17)
    res = {}
    for name in ("uniform", "learned"):
        a = Archive(max_atoms=mol.n)
        secs, conv, props, steps, moves = 0.0, 0, 0, [], []
        for r in range(eval_rounds):
            rs = ev.round_uniform(a, 1000 + r) if name == "uniform" else ev.round_learned(a, mlp, 1000 + r)
            secs += rs.seconds; conv += rs.converged; props += rs.proposals
            steps.append(rs.fire_steps_converged); moves.append(rs.rms_move_converged)
        n_min = a.count()
        res[name] = dict(distinct_minima=n_min, proposals=props, converged=conv, seconds=secs,
                         minima_per_s=n_min / secs, mean_fire_steps=float(np.nanmean(steps)),
                         mean_rms_move=float(np.nanmean(moves)), distinct_minima_rmsd=a.count_rmsd(),
                         minima_per_s_rmsd=a.count_rmsd() / secs)
        say(f"{name}: {n_min} distinct minima ({a.count_rmsd()} by RMSD) from {props} proposals ({conv} converged) "
            f"in {secs:.2f} s, "
            f"mean FIRE steps {res[name]['mean_fire_steps']:.0f}, mean RMS move {res[name]['mean_rms_move']:.2f} A")
    # the same comparison in continuous flow (finished slots refilled between 250-step
    # launches), where a proposal costs the steps it needs rather than its launch's slowest
    for name in ("uniform", "learned"):
        fl = Sampler(grid, mol, eval_rep, seed=seed + 29)
        prop = fl.propose_uniform_rows if name == "uniform" else fl.propose_learned_rows(mlp)
        a = Archive(max_atoms=mol.n)
        r = fl.flow(a, eval_rounds * eval_rep, prop, chunk=250)
        res[name]["flow"] = dict(distinct_minima=r["new_minima"], proposals=r["proposals"], converged=r["converged"],
                                 seconds=r["seconds"], minima_per_s=r["new_minima"] / r["seconds"],
                                 mean_fire_steps=r["mean_steps_converged"], launches=r["launches"],
                                 distinct_minima_rmsd=r["new_minima_rmsd"],
                                 minima_per_s_rmsd=r["new_minima_rmsd"] / r["seconds"])
        say(f"{name} (flow): {r['new_minima']} distinct minima ({r['new_minima_rmsd']} by RMSD) from "
            f"{r['proposals']} proposals ({r['converged']} converged) in {r['seconds']:.2f} s")
    # discovery curve at a short horizon: distinct minima (energy) after each of short_rounds
    # rounds of short_rep proposals, both forms from fresh archives
    for name in ("uniform", "learned"):
        sh = Sampler(grid, mol, short_rep, seed=seed + 41)
        a = Archive(max_atoms=mol.n)
        curve, secs = [], 0.0
        for r in range(short_rounds):
            rs = sh.round_uniform(a, 2000 + r) if name == "uniform" else sh.round_learned(a, mlp, 2000 + r)
            secs += rs.seconds
            curve.append((short_rep * (r + 1), a.count(), round(secs, 4)))
        res[name]["short_curve"] = curve
    res["gain_minima_per_s_flow"] = (res["learned"]["flow"]["minima_per_s"] /
                                     max(res["uniform"]["flow"]["minima_per_s"], 1e-12))
    res["training"] = dict(minima=m, distinct=arch.count(), steps=train_steps, loss_first=hist[0][1],
                           loss_last=hist[-1][1], collect_s=collect_s, train_s=train_s,
                           collect_rounds=collect_rounds)
    res["gain_minima_per_s"] = res["learned"]["minima_per_s"] / max(res["uniform"]["minima_per_s"], 1e-12)
    res["gain_minima_per_s_rmsd"] = (res["learned"]["minima_per_s_rmsd"] /
                                     max(res["uniform"]["minima_per_s_rmsd"], 1e-12))
    res["gain_minima_per_s_flow_rmsd"] = (res["learned"]["flow"]["minima_per_s_rmsd"] /
                                          max(res["uniform"]["flow"]["minima_per_s_rmsd"], 1e-12))
    return res


def compare_hopping_vs_uniform(grid, mol, n_rep=4096, n_hops=4, md_steps=1000, seed=S.SEED_PHILOX, log=None):
    """Minima hopping against uniform proposal rounds with the same number of relaxations
    (n_rep x (n_hops + 1)), each with a fresh archive: distinct minima by energy and by
    RMSD, wall time (Langevin, relaxation and dedupe included) and minima per second."""
    say = log or (lambda m: None)
    res = {}
    hp = Sampler(grid, mol, n_rep, seed=seed)
    hp.round_uniform(Archive(max_atoms=mol.n, capacity=1000, rmsd_capacity=1000), 999)     # warm-up, not counted
    a = Archive(max_atoms=mol.n)
    hops = hp.minima_hopping(a, n_hops, md_steps=md_steps, log=say)
    secs = sum(h["seconds"] for h in hops)
    res["hopping"] = dict(relaxations=n_rep * (n_hops + 1), converged=sum(h["converged"] for h in hops),
                          distinct_minima=a.count(), distinct_minima_rmsd=a.count_rmsd(), seconds=secs,
                          minima_per_s=a.count() / secs, minima_per_s_rmsd=a.count_rmsd() / secs, hops=hops)
    un = Sampler(grid, mol, n_rep, seed=seed + 41)
    un.round_uniform(Archive(max_atoms=mol.n, capacity=1000, rmsd_capacity=1000), 1999)   # warm-up, not counted
    a = Archive(max_atoms=mol.n)
    secs, conv = 0.0, 0
    for r in range(n_hops + 1):
        rs = un.round_uniform(a, 2000 + r)
        secs += rs.seconds; conv += rs.converged
        say(f"uniform round {r}: converged {rs.converged}/{n_rep}, new {rs.new_minima} (energy) "
            f"{rs.new_minima_rmsd} (rmsd), {rs.seconds:.2f} s")
    res["uniform"] = dict(relaxations=n_rep * (n_hops + 1), converged=conv, distinct_minima=a.count(),
                          distinct_minima_rmsd=a.count_rmsd(), seconds=secs, minima_per_s=a.count() / secs,
                          minima_per_s_rmsd=a.count_rmsd() / secs)
    for k in ("hopping", "uniform"):
        r = res[k]
        say(f"{k}: {r['distinct_minima']} (energy) / {r['distinct_minima_rmsd']} (rmsd) distinct minima from "
            f"{r['relaxations']} relaxations ({r['converged']} converged) in {r['seconds']:.2f} s")
    return res
