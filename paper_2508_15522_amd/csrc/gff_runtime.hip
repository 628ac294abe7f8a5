// Runtime helpers around the replica kernel: a captured HIP graph of one relaxation launch
// (re-launchable on the same buffers without host-side argument work), and a measured
// autotuner over launch shapes (block size, replicas per block, persistent grid size).
#include "gff_internal.hpp"
#include <algorithm>
#include <cstring>
#include <vector>

struct gff_graph_s {
    hipStream_t stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" gff_status gff_relax_graph_create(const gff_grid *grid, const gff_topology *topo, const gff_plan *plan,
                                             const gff_relax_params *params, const gff_state *state,
                                             double *d_E_rep, float *d_fnorm_rep, int *d_steps_rep,
                                             double *d_drift_rep, gff_graph **out) {
    if (!out) return GFF_EINVAL;
    auto *g = new gff_graph_s();
    if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) { delete g; return GFF_EHIP; }
    if (hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(g->stream);
        delete g;
        return GFF_EHIP;
    }
    const gff_status rc = gff_relax_batch(grid, topo, plan, params, state, d_E_rep, d_fnorm_rep, d_steps_rep,
                                          d_drift_rep, g->stream);
    const hipError_t e = hipStreamEndCapture(g->stream, &g->graph);
    if (rc != GFF_OK || e != hipSuccess) {
        if (e == hipSuccess) (void)hipGraphDestroy(g->graph);
        (void)hipStreamDestroy(g->stream);
        delete g;
        return rc != GFF_OK ? rc : GFF_EHIP;
    }
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        (void)hipStreamDestroy(g->stream);
        delete g;
        return GFF_EHIP;
    }
    *out = g;
    return GFF_OK;
}

extern "C" gff_status gff_graph_launch(gff_graph *g, void *stream) {
    if (!g) return GFF_EINVAL;
    return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? GFF_OK : GFF_EHIP;
}

extern "C" void gff_graph_destroy(gff_graph *g) {
    if (!g) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    (void)hipStreamDestroy(g->stream);
    delete g;
}

// Measured choice of the launch shape for a batch: every candidate block size (and, per
// block size, the packings below, persistent grids of 1-4 blocks per CU and, on B-spline
// grids, 2 lanes per atom, and 4 for small batches) runs `params` on a copy of the caller's
// state; the fastest (replica-steps per second) wins.
// Candidates that the device cannot launch are skipped.  The caller's state is untouched.
extern "C" gff_status gff_autotune(const gff_grid *grid, const gff_topology *topo, int n_rep, const int *rep_type_h,
                                   const gff_relax_params *params, const gff_state *state, gff_launch *best,
                                   float *best_rate, void *stream) {
    if (!grid || !topo || n_rep < 1 || !rep_type_h || !params || !state || !best) return GFF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int max_n = 0;
    for (int r = 0; r < n_rep; ++r) {
        if (rep_type_h[r] < 0 || rep_type_h[r] >= topo->n_types) return GFF_EINVAL;
        max_n = std::max(max_n, topo->natoms[rep_type_h[r]]);
    }
    int n_atoms = 0;
    for (int r = 0; r < n_rep; ++r) n_atoms += topo->natoms[rep_type_h[r]];
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    // scratch copies of the state (autotuning is a setup step and may allocate)
    const size_t a3 = (size_t)3 * n_atoms * sizeof(float), rb = (size_t)n_rep * sizeof(float);
    void *buf = nullptr;
    const size_t total = 2 * a3 + 4 * rb + (size_t)n_rep * (sizeof(double) * 7 + sizeof(float) + sizeof(int));
    if (hipMalloc(&buf, total) != hipSuccess) return GFF_ENOMEM;
    char *p = (char *)buf;
    gff_state t{};
    t.d_pos = (float *)p; p += a3;
    t.d_vel = (float *)p; p += a3;
    t.d_fire_dt = (float *)p; p += rb;
    t.d_fire_alpha = (float *)p; p += rb;
    t.d_fire_npos = (int *)p; p += rb;
    t.d_status = (unsigned *)p; p += rb;
    t.d_fixed_atom = state->d_fixed_atom;       // read only: shared with the caller
    t.d_fixed_pos = state->d_fixed_pos;
    double *E = (double *)p; p += (size_t)n_rep * sizeof(double);
    double *drift = (double *)p; p += (size_t)n_rep * 6 * sizeof(double);
    float *fn = (float *)p; p += (size_t)n_rep * sizeof(float);
    int *steps = (int *)p;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best_t = -1.f;
    gff_launch chosen{256, 0, 0, 1};
    gff_status rc = GFF_OK;
    // replicas per block: the densest packing, and when that leaves fewer than two packs per
    // compute unit, sparser packings (at most 1, 2, 4, 8 replicas per block) that spread a
    // small batch over more of the GPU.  Lanes per atom on B-spline grids: 2 for every batch
    // (two lanes share a large molecule's non-bonded partners: faster on the uneven-size batch
    // even when it fills the GPU), 4 when the batch has fewer atoms than one wave per SIMD
    const int rpb_cand[5] = {0, 1, 2, 4, 8};
    const bool bspline = grid->storage == GFF_STORE_F32 || grid->storage == GFF_STORE_F16;
    const bool small = (long)n_atoms < 4L * 64 * n_cu;
    for (int lpa = 1; lpa <= 4 && rc == GFF_OK; lpa *= 2) {
    if (lpa > 1 && !bspline) break;
    if (lpa == 4 && !small) break;
    for (int bt = 64; bt <= 1024 && rc == GFF_OK; bt += 64) {
        if (bt < max_n * lpa) continue;
        int dense_packs = -1, last_packs = -1;
        for (int ri = 0; ri < 5 && rc == GFF_OK; ++ri) {
            if (ri > 0 && (dense_packs < 0 || dense_packs >= 2 * n_cu)) break;
            for (int gm = 0; gm <= 4; ++gm) {
                gff_launch L{bt, rpb_cand[ri], gm == 0 ? 0 : gm * n_cu, lpa};
                gff_plan *plan = nullptr;
                if (gff_plan_create(topo, n_rep, rep_type_h, &L, &plan) != GFF_OK) break;
                if (gm == 0) {
                    if (ri == 0) dense_packs = plan->n_packs;
                    else if (plan->n_packs == last_packs || plan->n_packs == dense_packs) {   // same packing
                        gff_plan_destroy(plan);
                        break;
                    }
                    last_packs = plan->n_packs;
                }
                if (gm > 0 && L.grid_blocks >= plan->n_packs) { gff_plan_destroy(plan); break; }
                auto cp = [&](void *d, const void *src, size_t b) {
                    return src ? hipMemcpyAsync(d, src, b, hipMemcpyDeviceToDevice, s) : hipSuccess;
                };
                hipError_t e = cp(t.d_pos, state->d_pos, a3);
                if (e == hipSuccess) e = cp(t.d_vel, state->d_vel, a3);
                if (e == hipSuccess) e = cp(t.d_fire_dt, state->d_fire_dt, rb);
                if (e == hipSuccess) e = cp(t.d_fire_alpha, state->d_fire_alpha, rb);
                if (e == hipSuccess) e = cp(t.d_fire_npos, state->d_fire_npos, rb);
                if (e == hipSuccess) e = cp(t.d_status, state->d_status, rb);
                if (e != hipSuccess) { gff_plan_destroy(plan); rc = GFF_EHIP; break; }
                (void)hipEventRecord(e0, s);
                const gff_status r = gff_relax_batch(grid, topo, plan, params, &t, E, fn, steps,
                                                     params->mode == GFF_MODE_NVE ? drift : nullptr, s);
                (void)hipEventRecord(e1, s);
                gff_plan_destroy(plan);
                if (r != GFF_OK) { (void)hipGetLastError(); continue; }
                if (hipEventSynchronize(e1) != hipSuccess) { rc = GFF_EHIP; break; }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (best_t < 0.f || ms < best_t) { best_t = ms; chosen = L; }
            }
        }
    }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (rc != GFF_OK) return rc;
    if (best_t < 0.f) return GFF_EUNSUPPORTED;
    *best = chosen;
    if (best_rate) *best_rate = (float)((double)n_rep * std::max(1, params->n_steps) / (best_t * 1e-3));
    return GFF_OK;
}
