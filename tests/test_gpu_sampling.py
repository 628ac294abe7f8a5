"""GPU parity of the sampling rows: uniform proposals (Philox), pose construction, pose
encoding/decoding, energy and RMSD dedupe (a11, a13) and the proposer MLP (a11, a12).

Tolerances: Philox words are compared bit for bit; FP32 DOF/poses against the FP64 oracle
within 1e-5 (angles, fractions) and 1e-4 A (poses); the MLP runs BF16 GEMMs with FP32
accumulation against an FP64 oracle that rounds only the weights to BF16, so outputs and
gradients agree to the BF16 bound (2e-2 relative to the largest magnitude).
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import sampling as OS
from paper_2508_15522_amd import device as D, gridff as G, synth as S
from tests.gpu_common import announce

pytestmark = pytest.mark.gpu

L_CELL = 2 * S.SLAB_A


@pytest.fixture(scope="module")
def mols():
    D.require_gpu()
    return [S.mol_chain24(), S.mol_pah38(), S.mol_size(52, 6), S.mol_size(18, 3)]


def test_propose_uniform_bitexact_stream(mols):
    announce("propose uniform")
    T = 16
    n = 5003
    dof = torch.empty(n, 7 + T, device="cuda")
    nb = 2 + (T - 2 + 3) // 4
    raw = torch.empty(n, nb, 4, dtype=torch.int32, device="cuda")
    G.propose_uniform(n, T, S.SEED_PHILOX, 7, 3.0, 5.0, dof, raw)
    torch.cuda.synchronize()
    rg = raw.cpu().numpy().view(np.uint32)
    key = [S.SEED_PHILOX & 0xFFFFFFFF, S.SEED_PHILOX >> 32]
    for r in (0, 1, 17, 4096, n - 1):
        for b in range(nb):
            assert list(rg[r, b]) == O.philox4x32_10([r, b, 7, 0], key)
    ref = O.propose_uniform(n, T, S.SEED_PHILOX, 7)
    assert np.abs(dof.cpu().numpy() - ref).max() < 2e-5


def _plan_and_pos(mols, rep_type, dof):
    topo = G.Topology(mols)
    plan = G.Plan(topo, rep_type)
    Tmax = max(len(mols[t].rot_quads) for t in rep_type)
    d = torch.from_numpy(np.ascontiguousarray(dof, np.float32)).cuda()
    pos = torch.empty(3, plan.n_atoms, device="cuda")
    G.pose_from_dof(topo, plan, d, dof.shape[1], L_CELL, L_CELL, 0.0, pos)
    return topo, plan, pos


def test_pose_and_encoding_parity(mols):
    announce("pose + encode")
    rng = np.random.default_rng(2)
    rep_type = rng.integers(0, len(mols), 301)
    Tm = 16
    dof = S.f32(O.propose_uniform(len(rep_type), Tm, 99, 1))
    topo, plan, pos = _plan_and_pos(mols, rep_type, dof)
    work = torch.empty_like(pos)
    enc = torch.empty(len(rep_type), 41, device="cuda")
    G.encode_pose(topo, plan, pos, L_CELL, L_CELL, 0.0, work, enc)
    torch.cuda.synchronize()
    xs = D.unsoa(plan, pos)
    eg = enc.cpu().numpy()
    for r, t in enumerate(rep_type):
        ref = O.pose(mols[t], dof[r, :7 + len(mols[t].rot_quads)], L_CELL, L_CELL, 0.0)[0]
        assert np.abs(xs[r] - ref).max() < 1e-4, r
        eo = OS.encode_pose(mols[t], ref, L_CELL, L_CELL, 0.0)
        assert np.abs(eg[r] - eo).max() < 2e-4, (r, np.abs(eg[r] - eo).max())
    # decode inverts encode (up to FP32)
    dd = torch.empty(len(rep_type), 7 + Tm, device="cuda")
    G.decode_dof(enc, Tm, 0.0, 10.0, dd)
    torch.cuda.synchronize()
    dg = dd.cpu().numpy()
    q = dof[:, 3:7] * np.where(dof[:, 3:4] < 0, -1, 1)
    assert np.abs(dg[:, :3] - dof[:, :3]).max() < 1e-4
    assert np.abs(dg[:, 3:7] - q).max() < 1e-4
    for r, t in enumerate(rep_type):
        T = len(mols[t].rot_quads)
        if T:
            ang = (dg[r, 7:7 + T] - dof[r, 7:7 + T] + np.pi) % (2 * np.pi) - np.pi
            assert np.abs(ang).max() < 1e-4


def test_dedupe_matches_oracle():
    announce("dedupe")
    rng = np.random.default_rng(5)
    n = 3000
    E = np.round(rng.normal(-1.0, 0.3, n), 3) + rng.uniform(-0.004, 0.004, n)
    E[17] = np.nan
    types = rng.integers(0, 3, n)
    ok = (rng.random(n) < 0.9).astype(np.int32)
    cap = 100000
    dE = torch.from_numpy(E).cuda()
    dt = torch.from_numpy(types.astype(np.int32)).cuda()
    dok = torch.from_numpy(ok).cuda()
    aE = torch.zeros(cap, dtype=torch.float64, device="cuda")
    at = torch.zeros(cap, dtype=torch.int32, device="cuda")
    an = torch.zeros(1, dtype=torch.int32, device="cuda")
    isn = torch.empty(n, dtype=torch.int32, device="cuda")
    half = n // 2
    G.dedupe_energy(dE[:half], dt[:half], dok[:half], 0.01, cap, aE, at, an, isn[:half])
    G.dedupe_energy(dE[half:], dt[half:], dok[half:], 0.01, cap, aE, at, an, isn[half:])
    torch.cuda.synchronize()
    ref_new, arch = OS.dedupe_energy(E, types, ok, 0.01)
    assert np.array_equal(isn.cpu().numpy(), ref_new)
    assert an.item() == len(arch)
    assert np.array_equal(aE[:len(arch)].cpu().numpy(), np.array([a[0] for a in arch]))


def _rmsd_candidates(mols, n, seed, Lx, Ly, n_base=25):
    """Candidates around a few base poses per type: small per-atom noise (RMSD ~0.02 A to
    their base), rigid shifts of 0.06 A and 0.12 A along x (a chain: neighbours 0.06 apart,
    ends 0.12 apart) or 0.4 A, and random lattice translations."""
    rng = np.random.default_rng(seed)
    sub = S.rocksalt_slab(2, 3)
    bases = [S.place_replicas(m, n_base, sub, 9100 + t) for t, m in enumerate(mols)]
    types = rng.integers(0, len(mols), n)
    pos = []
    for t in types:
        x = bases[t][rng.integers(0, n_base)].copy()
        kind = rng.integers(0, 5)
        if kind == 0:
            x += rng.normal(0, 0.008, x.shape)
        elif kind in (1, 2):
            x[:, 0] += 0.06 * kind
        elif kind == 3:
            x[:, 1] += 0.4
        x[:, :2] += [rng.integers(-2, 3) * Lx, rng.integers(-2, 3) * Ly]
        pos.append(S.f32(x))
    return types.astype(np.int32), pos


def test_dedupe_rmsd_matches_oracle():
    announce("dedupe rmsd")
    mols = [S.mol_chain24(), S.mol_pah38(), S.mol_size(10, 1)]
    Lx, Ly = 11.28, 11.28
    topo = G.Topology(mols)
    cap, max_atoms = 4000, 38
    arch_pos = torch.zeros(cap, max_atoms, 3, device="cuda")
    arch_cen = torch.zeros(cap, 3, dtype=torch.float64, device="cuda")
    arch_type = torch.zeros(cap, dtype=torch.int32, device="cuda")
    arch_n = torch.zeros(1, dtype=torch.int32, device="cuda")
    ref_arch = None
    for call, seed in enumerate((31, 32)):
        types, pos = _rmsd_candidates(mols, 400, seed, Lx, Ly)
        ok = (np.random.default_rng(seed).random(len(types)) < 0.9).astype(np.int32)
        if call == 0:
            pos[7][3, 2] = np.nan
        plan = G.Plan(topo, types)
        dpos = D.soa(plan, pos)
        isn = torch.empty(plan.n_rep, dtype=torch.int32, device="cuda")
        G.dedupe_rmsd(plan, dpos, torch.from_numpy(ok).cuda(), 0.1, Lx, Ly, cap, max_atoms, arch_pos, arch_cen,
                      arch_type, arch_n, isn)
        torch.cuda.synchronize()
        ref_new, ref_arch = OS.dedupe_rmsd(pos, types, ok, 0.1, Lx, Ly, ref_arch)
        got = isn.cpu().numpy()
        announce(f"  call {call}: {int(got.sum())} new of {len(types)} (oracle {int(ref_new.sum())}), "
                 f"archive {arch_n.item()}")
        assert np.array_equal(got, ref_new)
    na = arch_n.item()
    assert na == len(ref_arch)
    ap, at, ac = arch_pos.cpu().numpy(), arch_type.cpu().numpy(), arch_cen.cpu().numpy()
    for k, (x, t) in enumerate(ref_arch):
        assert at[k] == t
        assert np.array_equal(ap[k, :len(x)].astype(np.float64), x)
        assert np.abs(ac[k] - x.mean(0)).max() < 1e-12
    # every decision is robust: no accepted pair of one type lies within 1e-4 A of the threshold
    d = [OS.rmsd_lattice(x, y, Lx, Ly) for i, (x, t) in enumerate(ref_arch) for (y, u) in ref_arch[:i] if t == u]
    assert min(abs(np.array(d) - 0.1)) > 1e-4


def test_dedupe_rmsd_capacity_and_arguments():
    announce("dedupe rmsd capacity")
    mols = [S.mol_chain24()]
    topo = G.Topology(mols)
    types, pos = _rmsd_candidates(mols, 50, 33, 11.28, 11.28)
    plan = G.Plan(topo, types)
    dpos = D.soa(plan, pos)
    cap = 3
    arch_pos = torch.zeros(cap, 24, 3, device="cuda")
    arch_cen = torch.zeros(cap, 3, dtype=torch.float64, device="cuda")
    arch_type = torch.zeros(cap, dtype=torch.int32, device="cuda")
    arch_n = torch.zeros(1, dtype=torch.int32, device="cuda")
    isn = torch.empty(plan.n_rep, dtype=torch.int32, device="cuda")
    G.dedupe_rmsd(plan, dpos, None, 0.1, 11.28, 11.28, cap, 24, arch_pos, arch_cen, arch_type, arch_n, isn)
    torch.cuda.synchronize()
    ref_new, _ = OS.dedupe_rmsd(pos, types, None, 0.1, 11.28, 11.28)
    got = isn.cpu().numpy()
    first = np.where(ref_new)[0][:cap]
    assert arch_n.item() == cap and np.array_equal(np.where(got)[0], first)
    with pytest.raises(G.GffError):       # archive entries too small for the plan's molecules
        G.dedupe_rmsd(plan, dpos, None, 0.1, 11.28, 11.28, cap, 23, arch_pos, arch_cen, arch_type, arch_n, isn)
    with pytest.raises(G.GffError):
        G.dedupe_rmsd(plan, dpos, None, -0.1, 11.28, 11.28, cap, 24, arch_pos, arch_cen, arch_type, arch_n, isn)
    small = torch.empty(G.dedupe_rmsd_workspace_bytes(plan.n_rep) - 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(G.GffError):       # workspace below the query
        G.dedupe_rmsd(plan, dpos, None, 0.1, 11.28, 11.28, cap, 24, arch_pos, arch_cen, arch_type, arch_n, isn, small)


def _bf16_bits(a):
    a = np.asarray(a, np.float32)
    return (OS.bf16(a).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


@pytest.mark.parametrize("shape", [(64, 64, 32), (130, 41, 256), (37, 256, 96), (256, 96, 1000)])
def test_gemm_bf16_mfma_layout(shape):
    """The MFMA tile against an exact FP64 product of the same BF16 inputs."""
    M, N, K = shape
    announce(f"gemm {shape}")
    rng = np.random.default_rng(M + N + K)
    A = rng.normal(size=(M, K)); B = rng.normal(size=(K, N))
    Ab, Bb = _bf16_bits(A), _bf16_bits(B)
    dA = torch.from_numpy(Ab.view(np.int16)).cuda()
    dB = torch.from_numpy(Bb.view(np.int16)).cuda()
    dC = torch.empty(M, N, device="cuda")
    G.gemm_bf16(dA, dB, dC)
    torch.cuda.synchronize()
    ref = OS.bf16(A) @ OS.bf16(B)
    err = np.abs(dC.cpu().numpy() - ref).max()
    assert err < 1e-5 * np.sqrt(K) * np.abs(ref).max() + 1e-5, err


def _strided_case(rng, M, N, K, sam, sak, sbk, sbn, offA=0, offB=0):
    """Flat BF16 buffers holding A(m,k) at offA + m*sam + k*sak and B(k,n) at offB + k*sbk + n*sbn
    (other words random too), and the exact FP64 product of the two logical matrices."""
    na = offA + (M - 1) * sam + (K - 1) * sak + 1 if M and K else offA + 1
    nb = offB + (K - 1) * sbk + (N - 1) * sbn + 1 if N and K else offB + 1
    fa, fb = _bf16_bits(rng.normal(size=na)), _bf16_bits(rng.normal(size=nb))
    m, k, n = np.arange(M)[:, None], np.arange(K)[None, :], np.arange(N)[None, :]
    A = fa[offA + m * sam + k * sak] if K else np.zeros((M, 0), np.uint16)
    B = fb[offB + np.arange(K)[:, None] * sbk + n * sbn] if K else np.zeros((0, N), np.uint16)
    to64 = lambda w: (w.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return fa, fb, to64(A) @ to64(B)


@pytest.mark.parametrize("case", [
    # (M, N, K, sam, sak, sbk, sbn, offA, offB, split): the staging layouts and the split-K path
    (200, 200, 1000, 1, 200, 200, 1, 0, 0, True),      # A and B contiguous along rows, K split, ragged tail
    (200, 200, 1000, 1, 200, 200, 1, 0, 0, False),     # the same in one pass over K
    (41, 256, 1024, 1, 41, 256, 1, 0, 0, True),        # A rows of 41: element loads, K split in 16
    (130, 72, 256, 256, 1, 1, 259, 0, 0, True),        # A along k; B along k with an odd stride
    (96, 64, 320, 320, 1, 64, 1, 1, 3, True),          # both operands misaligned by whole words
    (64, 40, 0, 8, 1, 40, 1, 0, 0, True),              # K = 0: zeros
])
def test_gemm_bf16_strided_layouts_and_split(case):
    """Every staging layout (16-byte loads along k or along rows, element loads for odd
    strides or misaligned bases) and the split-K reduction against the exact product."""
    M, N, K, sam, sak, sbk, sbn, offA, offB, split = case
    announce(f"gemm strided {case}")
    rng = np.random.default_rng(M * 7 + N + K)
    fa, fb, ref = _strided_case(rng, M, N, K, sam, sak, sbk, sbn, offA, offB)
    dA = torch.from_numpy(fa.view(np.int16)).cuda()[offA:]
    dB = torch.from_numpy(fb.view(np.int16)).cuda()[offB:]
    ldc = N + 5
    dC = torch.full((M, ldc), 7.0, device="cuda")
    work = torch.empty(G.gemm_bf16_workspace_bytes(), dtype=torch.uint8, device="cuda") if split else None
    G.gemm_bf16_strided(M, N, K, dA, sam, sak, dB, sbk, sbn, dC, ldc, work)
    torch.cuda.synchronize()
    C = dC.cpu().numpy()
    err = np.abs(C[:, :N] - ref).max() if K else np.abs(C[:, :N]).max()
    assert err <= 1e-5 * np.sqrt(max(K, 1)) * (np.abs(ref).max() if K else 0.0) + 1e-5, err
    assert (C[:, N:] == 7.0).all()                       # the row padding is left alone
    if split:                                            # deterministic: a second call agrees bit for bit
        dC2 = torch.zeros_like(dC)
        G.gemm_bf16_strided(M, N, K, dA, sam, sak, dB, sbk, sbn, dC2, ldc, work)
        torch.cuda.synchronize()
        assert torch.equal(dC[:, :N], dC2[:, :N])


def test_gemm_bf16_strided_rejects_invalid_arguments():
    dA = torch.zeros(64 * 64, dtype=torch.int16, device="cuda")
    dC = torch.empty(64, 64, device="cuda")
    small = torch.empty(G.gemm_bf16_workspace_bytes() - 4, dtype=torch.uint8, device="cuda")
    for bad in (dict(sam=0), dict(sak=-1), dict(ldc=63)):
        a = dict(sam=64, sak=1, ldc=64); a.update(bad)
        with pytest.raises(G.GffError):
            G.gemm_bf16_strided(64, 64, 64, dA, a["sam"], a["sak"], dA, 64, 1, dC, a["ldc"])
    with pytest.raises(G.GffError):
        G.gemm_bf16_strided(64, 64, 64, dA, 64, 1, dA, 64, 1, dC, 64, small)


def test_normal_philox_parity():
    n = 10001
    z = torch.empty(n, device="cuda")
    G.normal_philox(n, 1234567, 3, z)
    torch.cuda.synchronize()
    ref = OS.normal_philox(n, 1234567, 3)
    assert np.abs(z.cpu().numpy() - ref).max() < 2e-5 * (1 + np.abs(ref).max())


def test_mlp_forward_backward_adam_imle():
    announce("mlp")
    n_types = 4
    p0 = S.mlp_init_params(n_types)
    mlp = G.MLP(n_types, p0)
    rng = np.random.default_rng(3)
    B = 300
    noise = S.mlp_noise(B, 11)
    types = rng.integers(0, n_types, B).astype(np.int32)
    target = S.f32(rng.normal(size=(B, 41)) * 0.5)
    ntors = rng.integers(0, 17, B).astype(np.int32)
    dn = torch.from_numpy(noise.astype(np.float32)).cuda()
    dt = torch.from_numpy(types).cuda()
    dtg = torch.from_numpy(target.astype(np.float32)).cuda()
    dnt = torch.from_numpy(ntors).cuda()
    out = torch.empty(B, 41, device="cuda")
    mlp.forward(dn, dt, out)
    torch.cuda.synchronize()
    Y, _ = OS.forward(p0, n_types, noise, types)
    yg = out.cpu().numpy()
    assert np.abs(yg - Y).max() < 2e-2 * np.abs(Y).max()
    # gradient (lr = 0: no update)
    loss = torch.empty(B, device="cuda")
    mlp.train_step(dn, dt, dtg, dnt, 0.0, out, loss)
    torch.cuda.synchronize()
    L, gref, _ = OS.loss_and_grad(p0, n_types, noise, types, target, ntors)
    pg, gg = mlp.params()
    assert np.array_equal(pg, p0)
    o = 0
    blocks = []
    for l in range(4):
        nW = OS.DIMS[l + 1] * OS.DIMS[l]
        blocks += [(f"W{l}", o, o + nW), (f"b{l}", o + nW, o + nW + OS.DIMS[l + 1])]
        o += nW + OS.DIMS[l + 1]
    blocks.append(("emb", o, len(gref)))
    rel = {name: np.abs(gg[a:b] - gref[a:b]).max() / np.abs(gref[a:b]).max() for name, a, b in blocks}
    announce("  gradient error / largest magnitude: " + ", ".join(f"{k} {v:.2e}" for k, v in rel.items()))
    for name, v in rel.items():
        assert v < 2e-2, (name, v)
    assert abs(loss.cpu().numpy().mean() - L) < 2e-2 * L
    # first Adam step against the oracle's step from its own gradient: the step is
    # -lr g/(|g| + eps) ~ -lr sign(g), fixed wherever the gradient is not near zero
    mlp.train_step(dn, dt, dtg, dnt, 1e-3, out, loss)
    torch.cuda.synchronize()
    p1, _ = mlp.params()
    pe, _, _ = OS.adam(p0.astype(np.float64), gref, 0.0, 0.0, 1, 1e-3)
    big = np.abs(gref) > 0.1 * np.abs(gref).max()
    assert np.abs(p1 - pe)[big].max() < 1e-6
    assert np.abs(p1 - p0).max() <= 1e-3 + 2e-7       # plus the FP32 rounding of p - step
    # loss decreases over a few steps on a fixed batch
    losses = []
    for _ in range(30):
        mlp.train_step(dn, dt, dtg, dnt, 1e-3, out, loss)
        torch.cuda.synchronize()
        losses.append(loss.cpu().numpy().mean())
    announce(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.95 * losses[0] and losses[-1] < losses[len(losses) // 2]
    # IMLE selection against the oracle on the GPU's candidate outputs
    K = 8
    cand = torch.from_numpy(S.f32(rng.normal(size=(B, K, 41))).astype(np.float32)).cuda()
    best = torch.empty(B, dtype=torch.int32, device="cuda")
    bd = torch.empty(B, device="cuda")
    G.imle_select(cand, dtg, dnt, best, bd)
    torch.cuda.synchronize()
    cn = cand.cpu().numpy().astype(np.float64)
    bo, do = OS.imle_select(cn, target, ntors)
    bg = best.cpu().numpy()
    # indices agree exactly, except where the candidate the GPU chose is, in the oracle's
    # FP64 distance, as near as the oracle's best within FP32 rounding of the 41-term sum
    # (a near-tie the two precisions may break differently)
    for i in np.where(bg != bo)[0]:
        dg = OS.enc_dist(cn[i, bg[i]], target[i], ntors[i])[0]
        assert dg - do[i] <= 41 * 2.0 ** -23 * do[i], (i, dg, do[i])
    announce(f"  IMLE: {int((bg != bo).sum())} near-tie index differences of {B}")
    assert np.allclose(bd.cpu().numpy(), do, rtol=1e-5)


def test_continuous_flow_matches_single_launch():
    """Relaxing in 250-step launches with finished replicas replaced by new proposals gives
    every proposal exactly the result of one uninterrupted launch (same energy, convergence
    flag and move count, bit for bit)."""
    announce("continuous flow")
    from paper_2508_15522_amd import configs, sampling as SM
    D.require_gpu()
    cfg = configs.GRID_SMALL
    grid = D.build_physical_grid(cfg.substrate(), D.spec_for(cfg))
    mol = S.mol_chain24()
    smp = SM.Sampler(grid, mol, 128, max_steps=1000)
    arch = SM.Archive()
    res = smp.flow(arch, 400, smp.propose_uniform_rows, chunk=250, record=True)
    recs = res["records"]
    assert res["proposals"] == 400 and len(recs) == 400
    assert res["new_minima"] == arch.count() > 0
    dof = torch.from_numpy(np.stack([r[0] for r in recs]).astype(np.float32)).cuda()
    topo = G.Topology([mol])
    plan = G.Plan(topo, np.zeros(len(recs), np.int32))
    st = {"pos": torch.empty(3, plan.n_atoms, device="cuda"),
          "vel": torch.zeros(3, plan.n_atoms, device="cuda"),
          "fire_dt": torch.full((len(recs),), 0.05, device="cuda"),
          "fire_alpha": torch.full((len(recs),), 0.1, device="cuda"),
          "fire_npos": torch.zeros(len(recs), dtype=torch.int32, device="cuda"),
          "status": torch.zeros(len(recs), dtype=torch.int32, device="cuda")}
    G.pose_from_dof(topo, plan, dof, dof.shape[1], grid.Lx, grid.Ly, 0.0, st["pos"])
    out = D.outputs(plan)
    G.relax_batch(grid.desc, topo, plan, G.relax_params(G.MODE_FIRE, 1000, True), st, out["E"], out["fnorm"],
                  out["steps"])
    torch.cuda.synchronize()
    conv = (st["status"].cpu().numpy() & G.REP_CONVERGED) != 0
    E = out["E"].cpu().numpy()
    steps = out["steps"].cpu().numpy()
    assert np.array_equal(conv, np.array([r[2] for r in recs]))
    assert np.array_equal(E, np.array([r[1] for r in recs]))
    assert np.array_equal(steps, np.array([r[3] for r in recs]))
