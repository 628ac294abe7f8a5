// Pose proposals for the sampling loop: uniform random degrees of freedom from a
// counter-based Philox4x32-10 stream (Salmon et al., SC'11), decoding of the learned
// proposer's output encoding, pose construction (torsions, then rigid rotation and
// placement), minimum deduplication and the inverse map from relaxed poses to the
// encoding used to train the proposer.
//
// DOF layout per replica (float): [u, v, h, qw, qx, qy, qz, phi_0 .. phi_{T-1}]
//   u, v   lateral position of the centroid as fractions of the cell
//   h      height of the lowest atom above the top substrate plane
//   q      unit quaternion of the rigid rotation about the centroid
//   phi_k  target dihedral of rotatable torsion k (IUPAC convention)
#include "gff_internal.hpp"
#include <algorithm>
#include <cmath>
#include <mutex>

namespace gff {

constexpr float kTwoPiF = 6.28318530717958647692f;

__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * (1.f / 16777216.f); }

__global__ void __launch_bounds__(256) k_propose_uniform(int n_rep, int T, uint32_t key0, uint32_t key1, uint32_t round,
                                                         float hlo, float hhi, float *dof, uint32_t *raw) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rep) return;
    const int nb = 2 + (T > 2 ? (T - 2 + 3) / 4 : 0);
    float u[24];
#pragma unroll 1
    for (int b = 0; b < nb; ++b) {
        uint32_t c[4] = {(uint32_t)r, (uint32_t)b, round, 0u};
        philox4x32_10(c, key0, key1);
        for (int k = 0; k < 4; ++k) {
            u[4 * b + k] = u01(c[k]);
            if (raw) raw[((size_t)r * nb + b) * 4 + k] = c[k];
        }
    }
    float *d = dof + (size_t)r * (7 + T);
    d[0] = u[0]; d[1] = u[1]; d[2] = hlo + (hhi - hlo) * u[2];
    const float a = sqrtf(1.f - u[3]), bq = sqrtf(u[3]);
    float s2, c2, s3, c3;
    sincosf(kTwoPiF * u[4], &s2, &c2);
    sincosf(kTwoPiF * u[5], &s3, &c3);
    d[3] = bq * c3; d[4] = a * s2; d[5] = a * c2; d[6] = bq * s3;       // Shoemake
    for (int k = 0; k < T; ++k) d[7 + k] = kTwoPiF * u[6 + k];
}

__device__ __forceinline__ float3 ld3(const float *p, int i, int N) { return make_float3(p[i], p[i + N], p[i + 2 * N]); }
__device__ __forceinline__ void st3(float *p, int i, int N, float3 v) { p[i] = v.x; p[i + N] = v.y; p[i + 2 * N] = v.z; }
__device__ __forceinline__ float3 sub3(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float dihedral(float3 p0, float3 p1, float3 p2, float3 p3) {
    const float3 b1 = sub3(p1, p0), b2 = sub3(p2, p1), b3 = sub3(p3, p2);
    const float3 m = cross3(b1, b2), n = cross3(b2, b3);
    return atan2f(sqrtf(dot3(b2, b2)) * dot3(b1, n), dot3(m, n));
}

// One thread per replica, working in the caller's position array (SoA [3][N]).
__global__ void __launch_bounds__(128) k_pose(DevTopo t, const int *rep_type, const int *atom_off, int n_rep, int N,
                                              const float *dof, int stride, float Lx, float Ly, float ztop, float *pos) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rep) return;
    const int ty = rep_type[r];
    const TypeInfo ti = t.types[ty];
    const int n = ti.n, a0 = atom_off[r];
    const float *d = dof + (size_t)r * stride;
    for (int a = 0; a < n; ++a) {
        const float4 p = t.refpos[ti.abase + a];
        st3(pos, a0 + a, N, make_float3(p.x, p.y, p.z));
    }
    const int2 ri = t.rotinfo[ty];
    for (int k = 0; k < ri.y; ++k) {
        const int4 q = t.rotq[ri.x + k];
        const uint4 mk = t.rotm[ri.x + k];
        const float3 pi = ld3(pos, a0 + q.x, N), pj = ld3(pos, a0 + q.y, N), pk = ld3(pos, a0 + q.z, N),
                     pl = ld3(pos, a0 + q.w, N);
        const float ang = d[7 + k] - dihedral(pi, pj, pk, pl);
        float3 ax = sub3(pk, pj);
        const float il = rsqrtf(dot3(ax, ax));
        ax = make_float3(ax.x * il, ax.y * il, ax.z * il);
        float sn, cs;
        sincosf(ang, &sn, &cs);
        for (int a = 0; a < n; ++a) {
            const unsigned w = a < 32 ? mk.x : (a < 64 ? mk.y : (a < 96 ? mk.z : mk.w));
            if (!((w >> (a & 31)) & 1u)) continue;
            const float3 v = sub3(ld3(pos, a0 + a, N), pj);
            const float3 kv = cross3(ax, v);
            const float kd = dot3(ax, v) * (1.f - cs);
            st3(pos, a0 + a, N, make_float3(pj.x + v.x * cs + kv.x * sn + ax.x * kd,
                                            pj.y + v.y * cs + kv.y * sn + ax.y * kd,
                                            pj.z + v.z * cs + kv.z * sn + ax.z * kd));
        }
    }
    float3 c = make_float3(0.f, 0.f, 0.f);
    for (int a = 0; a < n; ++a) { const float3 p = ld3(pos, a0 + a, N); c.x += p.x; c.y += p.y; c.z += p.z; }
    c = make_float3(c.x / n, c.y / n, c.z / n);
    const float w = d[3], x = d[4], y = d[5], z = d[6];
    const float R00 = 1.f - 2.f * (y * y + z * z), R01 = 2.f * (x * y - z * w), R02 = 2.f * (x * z + y * w);
    const float R10 = 2.f * (x * y + z * w), R11 = 1.f - 2.f * (x * x + z * z), R12 = 2.f * (y * z - x * w);
    const float R20 = 2.f * (x * z - y * w), R21 = 2.f * (y * z + x * w), R22 = 1.f - 2.f * (x * x + y * y);
    float zmin = 3.4e38f;
    for (int a = 0; a < n; ++a) {
        const float3 p = sub3(ld3(pos, a0 + a, N), c);
        const float3 q = make_float3(R00 * p.x + R01 * p.y + R02 * p.z, R10 * p.x + R11 * p.y + R12 * p.z,
                                     R20 * p.x + R21 * p.y + R22 * p.z);
        st3(pos, a0 + a, N, q);
        zmin = fminf(zmin, q.z);
    }
    const float3 sh = make_float3(d[0] * Lx, d[1] * Ly, ztop + d[2] - zmin);
    for (int a = 0; a < n; ++a) {
        const float3 p = ld3(pos, a0 + a, N);
        st3(pos, a0 + a, N, make_float3(p.x + sh.x, p.y + sh.y, p.z + sh.z));
    }
}

// ---------------------------------------------------------------- deduplication
// Distinct minima in discovery order (energy criterion): candidate c of type t (with
// ok[c] != 0 and a finite energy) is new if |E_c - E_k| > tol for every archived minimum k
// of type t, including those accepted earlier in the same batch.  Three passes: every
// candidate against the archive as it was (is_new 1 for the survivors), every survivor
// against the earlier survivors (is_new 3 when one of its type lies within tol), then one
// workgroup in order: a survivor without such an earlier survivor is new outright, the
// others are compared with the minima accepted so far in the call.  Appends to the archive.
__global__ void __launch_bounds__(256) k_dedupe_archive(int n_new, const double *E, const int *type, const int *ok,
                                                        double tol, int capacity, const double *arch_E,
                                                        const int *arch_type, const int *arch_n, int *is_new) {
    __shared__ int s_state;              // 0 candidate, no match yet; 1 match or not a candidate
    const int c = blockIdx.x;
    const double e = E[c];
    const int t = type[c];
    if (threadIdx.x == 0) s_state = ((ok == nullptr || ok[c] != 0) && fabs(e) < 1e300) ? 0 : 1;
    __syncthreads();
    if (s_state == 0) {
        const int na = min(*arch_n, capacity);
        volatile int *vs = &s_state;
        for (int k = threadIdx.x; k < na && *vs == 0; k += blockDim.x)
            if (arch_type[k] == t && fabs(arch_E[k] - e) <= tol) *vs = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) is_new[c] = s_state == 0;
}

__global__ void __launch_bounds__(256) k_dedupe_pairs(const double *E, const int *type, double tol, int *is_new) {
    __shared__ int s_hit;
    const int c = blockIdx.x;
    if ((is_new[c] & 1) == 0) return;                  // uniform; bit 0 is never cleared here
    const double e = E[c];
    const int t = type[c];
    if (threadIdx.x == 0) s_hit = 0;
    __syncthreads();
    volatile int *vh = &s_hit;
    for (int j = threadIdx.x; j < c && *vh == 0; j += blockDim.x)
        if ((is_new[j] & 1) && type[j] == t && fabs(E[j] - e) <= tol) *vh = 1;
    __syncthreads();
    if (threadIdx.x == 0 && s_hit) is_new[c] = 3;
}

constexpr int kDedupeChunk = 2048;

__global__ void __launch_bounds__(1024) k_dedupe_batch(int n_new, const double *E, const int *type, double tol,
                                                       int capacity, double *arch_E, int *arch_type, int *arch_n,
                                                       int *is_new) {
    __shared__ int s_state[kDedupeChunk];
    __shared__ double s_e[kDedupeChunk];
    __shared__ int s_t[kDedupeChunk];
    __shared__ int s_fresh[kDedupeChunk];
    __shared__ int s_hit;
    const int na0 = min(*arch_n, capacity);
    int na = na0;                                      // identical in every thread
    for (int c0 = 0; c0 < n_new; c0 += kDedupeChunk) {
        const int m = min(kDedupeChunk, n_new - c0);
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            s_state[i] = is_new[c0 + i]; s_e[i] = E[c0 + i]; s_t[i] = type[c0 + i];
        }
        __syncthreads();
        for (int i = 0; i < m; ++i) {
            const int state = s_state[i];
            if (state == 0) { if (threadIdx.x == 0) s_fresh[i] = 0; continue; }
            const double e = s_e[i];
            const int t = s_t[i];
            bool fresh = na < capacity;
            if (state == 3 && fresh && na > na0) {
                __syncthreads();                       // the appends so far are visible
                if (threadIdx.x == 0) s_hit = 0;
                __syncthreads();
                for (int k = na0 + threadIdx.x; k < na; k += blockDim.x)
                    if (arch_type[k] == t && fabs(arch_E[k] - e) <= tol) s_hit = 1;
                __syncthreads();
                fresh = s_hit == 0;
            }
            if (threadIdx.x == 0) {
                s_fresh[i] = fresh;
                if (fresh) { arch_E[na] = e; arch_type[na] = t; }
            }
            if (fresh) ++na;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < m; i += blockDim.x) is_new[c0 + i] = s_fresh[i];
        __syncthreads();
    }
    if (threadIdx.x == 0) *arch_n = na;
}

// ---------------------------------------------------------------- RMSD deduplication
// Two minima of one molecule type (same atom order) are the same when the RMSD of their
// atoms, minimised over the lateral lattice translations t = (a Lx, b Ly), is at most tol
// (Section "Configuration sampling on GPU": site and orientation count; no rotation fit, no
// permutation).  The mean square is |t - m|^2 + const with m the mean coordinate
// difference, so the best t is the lattice vector nearest m.  The sum of squares runs in
// FP64 over the atoms in order and stops once it exceeds n tol^2: its terms are
// non-negative, so stopping never changes the decision.
//
// Three passes keep the order-dependent part small.  (1) one block per candidate: its
// centroid, and whether it matches a minimum archived before the call; (2) one block per
// surviving candidate: whether any earlier survivor of its type matches it; (3) one
// workgroup walks the survivors in order: one with no earlier matching survivor is new
// without further comparison, the others are compared with the minima accepted so far in
// the call.
struct RmsdArgs {
    const int *rep_type, *atom_off, *ok;
    const float *pos;                    // [3][N]
    int N, n_rep, capacity, max_atoms;
    double Lx, Ly, tol2;
    float *arch_pos;                     // [capacity][max_atoms][3]
    double *arch_cen;                    // [capacity][3]
    int *arch_type, *arch_n, *is_new;    // is_new: 1 survivor of pass 1, 3 with an earlier matching survivor
    double4 *cen;                        // [n_rep] candidate centroids (w: pass 3's decision)
    int *acc;                            // [n_rep] candidates accepted in the call, in order
};

// Candidate c's atoms into LDS (x, y, z per atom).
__device__ void stage_candidate(const RmsdArgs &A, int c, float *s_x) {
    const int g0 = A.atom_off[c], n = A.atom_off[c + 1] - g0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        s_x[3 * i] = A.pos[g0 + i]; s_x[3 * i + 1] = A.pos[g0 + i + A.N]; s_x[3 * i + 2] = A.pos[g0 + i + 2 * A.N];
    }
}

// Lattice-translated RMSD test of the staged candidate (atoms s_x, centroid c) against an
// entry given by its atoms (x, y, z at stride sx within an atom, sa between atoms) and
// centroid e.
__device__ __forceinline__ bool same_minimum(const RmsdArgs &A, const float *s_x, double cx, double cy, int n,
                                             const float *ex, const float *ey, const float *ez, long sa, double ecx,
                                             double ecy) {
    const double tx = rint((cx - ecx) / A.Lx) * A.Lx, ty = rint((cy - ecy) / A.Ly) * A.Ly;
    const double lim = n * A.tol2;
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        const double dx = (double)s_x[3 * i] - (double)ex[i * sa] - tx;
        const double dy = (double)s_x[3 * i + 1] - (double)ey[i * sa] - ty;
        const double dz = (double)s_x[3 * i + 2] - (double)ez[i * sa];
        s += dx * dx + dy * dy + dz * dz;
        if (s > lim) return false;
    }
    return true;
}

__device__ __forceinline__ bool same_as_archived(const RmsdArgs &A, const float *s_x, double4 c, int n, int k) {
    const float *ap = A.arch_pos + (size_t)k * 3 * A.max_atoms;
    const double *ac = A.arch_cen + 3 * (size_t)k;
    return same_minimum(A, s_x, c.x, c.y, n, ap, ap + 1, ap + 2, 3, ac[0], ac[1]);
}

// Pass 1, one block per candidate: centroid (FP64, atoms in order) and the match against
// the minima archived before the call.  is_new[c] = 1 for a candidate (ok, finite) that
// matches none of them, 0 otherwise.
__global__ void __launch_bounds__(256) k_rmsd_archive(RmsdArgs A) {
    __shared__ float s_x[3 * kMaxAtoms];
    __shared__ double4 s_c;
    __shared__ int s_state;              // 0 candidate, no match yet; 1 match; 2 not a candidate
    const int c = blockIdx.x;
    const int n = A.atom_off[c + 1] - A.atom_off[c], t = A.rep_type[c];
    stage_candidate(A, c, s_x);
    __syncthreads();
    if (threadIdx.x == 0) {
        bool fin = true;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int i = 0; i < n; ++i) {
            const float x = s_x[3 * i], y = s_x[3 * i + 1], z = s_x[3 * i + 2];
            fin = fin && __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z);
            sx += x; sy += y; sz += z;
        }
        s_c = make_double4(sx / n, sy / n, sz / n, fin ? 1.0 : 0.0);
        A.cen[c] = s_c;
        s_state = (fin && (A.ok == nullptr || A.ok[c] != 0)) ? 0 : 2;
    }
    __syncthreads();
    if (s_state == 0) {
        const double4 cc = s_c;
        const int na = min(*A.arch_n, A.capacity);
        volatile int *vs = &s_state;
        for (int k = threadIdx.x; k < na && *vs == 0; k += blockDim.x)
            if (A.arch_type[k] == t && same_as_archived(A, s_x, cc, n, k)) *vs = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) A.is_new[c] = s_state == 0;
}

// Pass 2, one block per survivor c: does an earlier survivor of the same type match it?
// Then is_new[c] = 3.  Only bit 1 is written here, and only by the block of c, so the
// survivor bit read by the other blocks does not change.
__global__ void __launch_bounds__(256) k_rmsd_pairs(RmsdArgs A) {
    __shared__ float s_x[3 * kMaxAtoms];
    __shared__ int s_hit;
    const int c = blockIdx.x;
    if ((A.is_new[c] & 1) == 0) return;                 // uniform across the block
    const int n = A.atom_off[c + 1] - A.atom_off[c], t = A.rep_type[c];
    stage_candidate(A, c, s_x);
    if (threadIdx.x == 0) s_hit = 0;
    __syncthreads();
    const double4 cc = A.cen[c];
    volatile int *vh = &s_hit;
    for (int j = threadIdx.x; j < c && *vh == 0; j += blockDim.x) {
        if ((A.is_new[j] & 1) == 0 || A.rep_type[j] != t) continue;
        const double4 cj = A.cen[j];
        const int g0 = A.atom_off[j];
        if (same_minimum(A, s_x, cc.x, cc.y, n, A.pos + g0, A.pos + g0 + A.N, A.pos + g0 + 2 * A.N, 1, cj.x, cj.y))
            *vh = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_hit) A.is_new[c] = 3;
}

// Pass 3, one workgroup: the survivors in order, their data staged in LDS a chunk at a
// time.  A survivor without an earlier matching survivor (is_new 1) is new; one with (3) is
// compared with the candidates accepted so far in the call (their own coordinates; the
// archive copies are written afterwards).  The decision goes to cen[c].w as the archive
// slot + 1, or 0 (is_new stays as the passes left it while the workgroup reads it).
constexpr int kRmsdChunk = 1024;

__global__ void __launch_bounds__(1024) k_rmsd_batch(RmsdArgs A) {
    __shared__ float s_x[3 * kMaxAtoms];
    __shared__ int s_state[kRmsdChunk], s_type[kRmsdChunk], s_n[kRmsdChunk];
    __shared__ double s_cx[kRmsdChunk], s_cy[kRmsdChunk];
    __shared__ int s_hit;
    const int na0 = min(*A.arch_n, A.capacity);
    int na = na0;                                      // identical in every thread
    for (int c0 = 0; c0 < A.n_rep; c0 += kRmsdChunk) {
        const int m = min(kRmsdChunk, A.n_rep - c0);
        __syncthreads();                               // the previous chunk's LDS reads are done
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            const int c = c0 + i;
            s_state[i] = A.is_new[c]; s_type[i] = A.rep_type[c];
            s_n[i] = A.atom_off[c + 1] - A.atom_off[c];
            const double4 cc = A.cen[c];
            s_cx[i] = cc.x; s_cy[i] = cc.y;
        }
        __syncthreads();
        for (int i = 0; i < m; ++i) {
            const int state = s_state[i];
            if (state == 0) continue;
            const int c = c0 + i, n = s_n[i], t = s_type[i];
            bool fresh = na < A.capacity;
            if (state == 3 && fresh && na > na0) {
                __syncthreads();                       // accepted list and s_x reads are done
                stage_candidate(A, c, s_x);
                if (threadIdx.x == 0) s_hit = 0;
                __syncthreads();
                const double cx = s_cx[i], cy = s_cy[i];
                for (int k = threadIdx.x; k < na - na0; k += blockDim.x) {
                    const int j = A.acc[k];
                    if (A.rep_type[j] != t) continue;
                    const double4 cj = A.cen[j];
                    const int g0 = A.atom_off[j];
                    if (same_minimum(A, s_x, cx, cy, n, A.pos + g0, A.pos + g0 + A.N, A.pos + g0 + 2 * A.N, 1,
                                     cj.x, cj.y))
                        s_hit = 1;
                }
                __syncthreads();
                fresh = s_hit == 0;
            }
            if (threadIdx.x == 0) {
                A.cen[c].w = fresh ? (double)(na + 1) : 0.0;
                if (fresh) A.acc[na - na0] = c;
            }
            if (fresh) ++na;
        }
    }
    if (threadIdx.x == 0) *A.arch_n = na;
}

// Appends the accepted candidates to their archive slots and writes is_new.
__global__ void __launch_bounds__(128) k_rmsd_final(RmsdArgs A) {
    const int c = blockIdx.x;
    const double4 cc = A.cen[c];
    const bool acc = A.is_new[c] != 0 && cc.w > 0.0;
    if (threadIdx.x == 0) A.is_new[c] = acc ? 1 : 0;
    if (!acc) return;
    const int slot = (int)cc.w - 1;
    const int g0 = A.atom_off[c], n = A.atom_off[c + 1] - g0;
    float *ap = A.arch_pos + (size_t)slot * 3 * A.max_atoms;
    for (int i = threadIdx.x; i < 3 * n; i += blockDim.x) {
        const int a = i / 3, d = i - 3 * a;
        ap[i] = A.pos[g0 + a + d * A.N];
    }
    if (threadIdx.x == 0) {
        A.arch_cen[3 * (size_t)slot] = cc.x; A.arch_cen[3 * (size_t)slot + 1] = cc.y;
        A.arch_cen[3 * (size_t)slot + 2] = cc.z;
        A.arch_type[slot] = A.rep_type[c];
    }
}

// ---------------------------------------------------------------- pose -> encoding
// Symmetric 4x4 eigenvector of the largest eigenvalue by cyclic Jacobi rotations.
__device__ void top_eigvec4(float A[4][4], float v[4]) {
    float V[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    for (int sweep = 0; sweep < 12; ++sweep) {
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 4; ++q) {
                const float apq = A[p][q];
                if (fabsf(apq) < 1e-30f) continue;
                const float th = 0.5f * (A[q][q] - A[p][p]) / apq;
                const float tt = (th >= 0.f ? 1.f : -1.f) / (fabsf(th) + sqrtf(th * th + 1.f));
                const float c = rsqrtf(tt * tt + 1.f), sn = tt * c;
                for (int k = 0; k < 4; ++k) {          // A <- J^T A J
                    const float akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - sn * akq; A[k][q] = sn * akp + c * akq;
                }
                for (int k = 0; k < 4; ++k) {
                    const float apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - sn * aqk; A[q][k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < 4; ++k) {
                    const float vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - sn * vkq; V[k][q] = sn * vkp + c * vkq;
                }
            }
    }
    int b = 0;
    for (int k = 1; k < 4; ++k) if (A[k][k] > A[b][b]) b = k;
    for (int k = 0; k < 4; ++k) v[k] = V[k][b];
}

// Encoding of a pose (inverse of k_pose): torsions measured on the pose, the reference
// geometry re-posed with those torsions, and the rigid rotation that best maps it onto the
// pose (Horn's quaternion method).  enc[41] = [cos 2pi u, sin 2pi u, cos 2pi v, sin 2pi v,
// h, qw, qx, qy, qz (qw >= 0), (cos phi_k, sin phi_k) for k < 16 (zero past the type's T)].
__global__ void __launch_bounds__(128) k_encode(DevTopo t, const int *rep_type, const int *atom_off, int n_rep, int N,
                                                const float *pos, float Lx, float Ly, float ztop, float *work,
                                                float *enc) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rep) return;
    const int ty = rep_type[r];
    const TypeInfo ti = t.types[ty];
    const int n = ti.n, a0 = atom_off[r];
    const int2 ri = t.rotinfo[ty];
    float *e = enc + (size_t)r * 41;
    float dof[7 + 16];
    // measured torsions
    for (int k = 0; k < ri.y; ++k) {
        const int4 q = t.rotq[ri.x + k];
        dof[7 + k] = dihedral(ld3(pos, a0 + q.x, N), ld3(pos, a0 + q.y, N), ld3(pos, a0 + q.z, N), ld3(pos, a0 + q.w, N));
    }
    // reference with those torsions, in the work array (same layout as pos)
    for (int a = 0; a < n; ++a) {
        const float4 p = t.refpos[ti.abase + a];
        st3(work, a0 + a, N, make_float3(p.x, p.y, p.z));
    }
    for (int k = 0; k < ri.y; ++k) {
        const int4 q = t.rotq[ri.x + k];
        const uint4 mk = t.rotm[ri.x + k];
        const float3 pj = ld3(work, a0 + q.y, N), pk = ld3(work, a0 + q.z, N);
        const float ang = dof[7 + k] - dihedral(ld3(work, a0 + q.x, N), pj, pk, ld3(work, a0 + q.w, N));
        float3 ax = sub3(pk, pj);
        const float il = rsqrtf(dot3(ax, ax));
        ax = make_float3(ax.x * il, ax.y * il, ax.z * il);
        float sn, cs;
        sincosf(ang, &sn, &cs);
        for (int a = 0; a < n; ++a) {
            const unsigned w = a < 32 ? mk.x : (a < 64 ? mk.y : (a < 96 ? mk.z : mk.w));
            if (!((w >> (a & 31)) & 1u)) continue;
            const float3 v = sub3(ld3(work, a0 + a, N), pj);
            const float3 kv = cross3(ax, v);
            const float kd = dot3(ax, v) * (1.f - cs);
            st3(work, a0 + a, N, make_float3(pj.x + v.x * cs + kv.x * sn + ax.x * kd,
                                             pj.y + v.y * cs + kv.y * sn + ax.y * kd,
                                             pj.z + v.z * cs + kv.z * sn + ax.z * kd));
        }
    }
    float3 cr = make_float3(0.f, 0.f, 0.f), cp = cr;
    float zmin = 3.4e38f;
    for (int a = 0; a < n; ++a) {
        const float3 p = ld3(pos, a0 + a, N), q = ld3(work, a0 + a, N);
        cp.x += p.x; cp.y += p.y; cp.z += p.z; cr.x += q.x; cr.y += q.y; cr.z += q.z;
        zmin = fminf(zmin, p.z);
    }
    cp = make_float3(cp.x / n, cp.y / n, cp.z / n);
    cr = make_float3(cr.x / n, cr.y / n, cr.z / n);
    float S[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int a = 0; a < n; ++a) {
        const float3 x = sub3(ld3(work, a0 + a, N), cr), y = sub3(ld3(pos, a0 + a, N), cp);
        const float xs[3] = {x.x, x.y, x.z}, ys[3] = {y.x, y.y, y.z};
        for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) S[i][j] += xs[i] * ys[j];
    }
    float M[4][4] = {
        {S[0][0] + S[1][1] + S[2][2], S[1][2] - S[2][1], S[2][0] - S[0][2], S[0][1] - S[1][0]},
        {S[1][2] - S[2][1], S[0][0] - S[1][1] - S[2][2], S[0][1] + S[1][0], S[2][0] + S[0][2]},
        {S[2][0] - S[0][2], S[0][1] + S[1][0], -S[0][0] + S[1][1] - S[2][2], S[1][2] + S[2][1]},
        {S[0][1] - S[1][0], S[2][0] + S[0][2], S[1][2] + S[2][1], -S[0][0] - S[1][1] + S[2][2]}};
    float q[4];
    top_eigvec4(M, q);
    const float qn = rsqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float sg = q[0] < 0.f ? -qn : qn;
    float u = cp.x / Lx, v = cp.y / Ly;
    u -= floorf(u); v -= floorf(v);
    float su, cu, sv, cv;
    sincosf(kTwoPiF * u, &su, &cu);
    sincosf(kTwoPiF * v, &sv, &cv);
    e[0] = cu; e[1] = su; e[2] = cv; e[3] = sv; e[4] = zmin - ztop;
    for (int k = 0; k < 4; ++k) e[5 + k] = q[k] * sg;
    for (int k = 0; k < 16; ++k) {
        float sn = 0.f, cs = 0.f;
        if (k < ri.y) sincosf(dof[7 + k], &sn, &cs);
        e[9 + 2 * k] = cs; e[10 + 2 * k] = sn;
    }
}

// Encoding (e.g. the proposer's output) -> DOF: angles from (cos, sin) pairs, the
// quaternion normalised, the height clamped to [h_lo, h_hi].
__global__ void __launch_bounds__(256) k_decode(int n, const float *enc, int T, float hlo, float hhi, float *dof) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const float *e = enc + (size_t)r * 41;
    float *d = dof + (size_t)r * (7 + T);
    float u = atan2f(e[1], e[0]) / kTwoPiF, v = atan2f(e[3], e[2]) / kTwoPiF;
    d[0] = u - floorf(u); d[1] = v - floorf(v);
    d[2] = fminf(fmaxf(e[4], hlo), hhi);
    float qw = e[5], qx = e[6], qy = e[7], qz = e[8];
    float nq = qw * qw + qx * qx + qy * qy + qz * qz;
    if (!(nq > 1e-12f)) { qw = 1.f; qx = qy = qz = 0.f; nq = 1.f; }
    const float inq = rsqrtf(nq);
    d[3] = qw * inq; d[4] = qx * inq; d[5] = qy * inq; d[6] = qz * inq;
    for (int k = 0; k < T; ++k) d[7 + k] = atan2f(e[10 + 2 * k], e[9 + 2 * k]);
}

}  // namespace gff

using namespace gff;

extern "C" gff_status gff_dedupe_energy(int n_new, const double *d_E, const int *d_type, const int *d_ok, double tol,
                                        int capacity, double *d_arch_E, int *d_arch_type, int *d_arch_n,
                                        int *d_is_new, void *stream) {
    if (n_new < 0 || capacity < 0 || !(tol >= 0.0)) return GFF_EINVAL;
    if (n_new > 0 && (!d_E || !d_type || !d_is_new)) return GFF_EINVAL;
    if (!d_arch_E || !d_arch_type || !d_arch_n) return GFF_EINVAL;
    if (n_new == 0) return GFF_OK;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_dedupe_archive, dim3(n_new), dim3(256), 0, s, n_new, d_E, d_type, d_ok, tol, capacity,
                       (const double *)d_arch_E, (const int *)d_arch_type, (const int *)d_arch_n, d_is_new);
    hipLaunchKernelGGL(k_dedupe_pairs, dim3(n_new), dim3(256), 0, s, d_E, d_type, tol, d_is_new);
    hipLaunchKernelGGL(k_dedupe_batch, dim3(1), dim3(1024), 0, s, n_new, d_E, d_type, tol, capacity, d_arch_E,
                       d_arch_type, d_arch_n, d_is_new);
    return hip_status(hipGetLastError());
}

extern "C" size_t gff_dedupe_rmsd_workspace_bytes(int n_rep) {
    return n_rep > 0 ? (size_t)n_rep * (sizeof(double4) + sizeof(int)) : 0;
}

extern "C" gff_status gff_dedupe_rmsd(const gff_plan *plan, const float *d_pos, const int *d_ok, float tol, float Lx,
                                      float Ly, int capacity, int max_atoms, float *d_arch_pos, double *d_arch_cen,
                                      int *d_arch_type, int *d_arch_n, int *d_is_new, void *d_work, size_t work_bytes,
                                      void *stream) {
    if (!plan || !(tol >= 0.f) || !std::isfinite(tol) || !(Lx > 0.f) || !(Ly > 0.f) || capacity < 0) return GFF_EINVAL;
    if (max_atoms < plan->max_n || max_atoms > kMaxAtoms) return GFF_EINVAL;
    if (!d_arch_pos || !d_arch_cen || !d_arch_type || !d_arch_n) return GFF_EINVAL;
    if (plan->n_rep == 0) return GFF_OK;
    if (!d_pos || !d_is_new) return GFF_EINVAL;
    if (!d_work || work_bytes < gff_dedupe_rmsd_workspace_bytes(plan->n_rep)) return GFF_EWORKSPACE;
    RmsdArgs A{plan->d_rep_type, plan->d_atom_off, d_ok, d_pos, plan->n_atoms, plan->n_rep, capacity, max_atoms,
               (double)Lx, (double)Ly, (double)tol * (double)tol, d_arch_pos, d_arch_cen, d_arch_type, d_arch_n,
               d_is_new, static_cast<double4 *>(d_work),
               reinterpret_cast<int *>(static_cast<char *>(d_work) + (size_t)plan->n_rep * sizeof(double4))};
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_rmsd_archive, dim3(plan->n_rep), dim3(256), 0, s, A);
    hipLaunchKernelGGL(k_rmsd_pairs, dim3(plan->n_rep), dim3(256), 0, s, A);
    hipLaunchKernelGGL(k_rmsd_batch, dim3(1), dim3(1024), 0, s, A);
    hipLaunchKernelGGL(k_rmsd_final, dim3(plan->n_rep), dim3(128), 0, s, A);
    return hip_status(hipGetLastError());
}

// ---------------------------------------------------------------- allocation-free dedupe
// The RMSD dedupe's per-candidate scratch (centroids and decisions, accepted list) in a
// file-scope device array, for callers that cannot allocate.  Every GPU holds its own copy
// until the process ends; host code uses only the address hipGetSymbolAddress returns for
// the current device, looked up once per device on the first call there.
namespace gff {
static __device__ __align__(256) unsigned char scratch[(size_t)GFF_DEDUPE_NOALLOC_MAX_REP * (sizeof(double4) + sizeof(int))];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static gff_status scratch_for_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GFF_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GFF_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return GFF_OK;
}
}  // namespace gff

extern "C" gff_status gff_dedupe_rmsd_noalloc(const gff_plan *plan, const float *d_pos, const int *d_ok, float tol,
                                              float Lx, float Ly, int capacity, int max_atoms, float *d_arch_pos,
                                              double *d_arch_cen, int *d_arch_type, int *d_arch_n, int *d_is_new,
                                              void *stream) {
    if (!plan) return GFF_EINVAL;
    if (plan->n_rep > GFF_DEDUPE_NOALLOC_MAX_REP) return GFF_EWORKSPACE;
    void *work = nullptr;
    if (plan->n_rep > 0) {
        const gff_status rc = scratch_for_current_device(&work);
        if (rc != GFF_OK) return rc;
    }
    // the kernels write every scratch entry they read within the call, so nothing is cleared
    return gff_dedupe_rmsd(plan, d_pos, d_ok, tol, Lx, Ly, capacity, max_atoms, d_arch_pos, d_arch_cen, d_arch_type,
                           d_arch_n, d_is_new, work, gff_dedupe_rmsd_workspace_bytes(GFF_DEDUPE_NOALLOC_MAX_REP),
                           stream);
}

extern "C" gff_status gff_encode_pose(const gff_topology *topo, const gff_plan *plan, const float *d_pos, float Lx,
                                      float Ly, float z_top, float *d_work, float *d_enc, void *stream) {
    if (!topo || !plan || (plan->n_rep > 0 && (!d_pos || !d_work || !d_enc))) return GFF_EINVAL;
    for (int t : plan->rep_type_h) if (topo->nrot[t] > 16) return GFF_EUNSUPPORTED;
    if (plan->n_rep == 0) return GFF_OK;
    hipLaunchKernelGGL(k_encode, dim3((plan->n_rep + 127) / 128), dim3(128), 0, (hipStream_t)stream, topo->dev,
                       plan->d_rep_type, plan->d_atom_off, plan->n_rep, plan->n_atoms, d_pos, Lx, Ly, z_top, d_work,
                       d_enc);
    return hip_status(hipGetLastError());
}

extern "C" gff_status gff_decode_dof(int n, const float *d_enc, int n_tors, float h_lo, float h_hi, float *d_dof,
                                     void *stream) {
    if (n < 0 || n_tors < 0 || n_tors > 16 || (n > 0 && (!d_enc || !d_dof))) return GFF_EINVAL;
    if (n == 0) return GFF_OK;
    hipLaunchKernelGGL(k_decode, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, n, d_enc, n_tors, h_lo, h_hi,
                       d_dof);
    return hip_status(hipGetLastError());
}

extern "C" gff_status gff_propose_uniform(int n_rep, int n_tors, uint64_t seed, uint32_t round, float h_lo, float h_hi,
                                          float *d_dof, uint32_t *d_raw, void *stream) {
    if (n_rep < 0 || n_tors < 0 || n_tors > 16 || (n_rep > 0 && !d_dof) || !(h_hi >= h_lo)) return GFF_EINVAL;
    if (n_rep == 0) return GFF_OK;
    hipLaunchKernelGGL(k_propose_uniform, dim3((n_rep + 255) / 256), dim3(256), 0, (hipStream_t)stream, n_rep, n_tors,
                       (uint32_t)seed, (uint32_t)(seed >> 32), round, h_lo, h_hi, d_dof, d_raw);
    return hip_status(hipGetLastError());
}

extern "C" gff_status gff_pose_from_dof(const gff_topology *topo, const gff_plan *plan, const float *d_dof,
                                        int dof_stride, float Lx, float Ly, float z_top, float *d_pos, void *stream) {
    if (!topo || !plan || !d_pos || (plan->n_rep > 0 && !d_dof)) return GFF_EINVAL;
    int tmax = 0;
    for (int t : plan->rep_type_h) tmax = std::max(tmax, topo->nrot[t]);
    if (dof_stride < 7 + tmax) return GFF_EINVAL;
    if (plan->n_rep == 0) return GFF_OK;
    hipLaunchKernelGGL(k_pose, dim3((plan->n_rep + 127) / 128), dim3(128), 0, (hipStream_t)stream, topo->dev,
                       plan->d_rep_type, plan->d_atom_off, plan->n_rep, plan->n_atoms, d_dof, dof_stride, Lx, Ly, z_top,
                       d_pos);
    return hip_status(hipGetLastError());
}

// Continuous-flow relaxation: per replica, mode[r] = 1 replaces its state by a new proposal
// (positions from src, zero velocities, FIRE scalars reset, status cleared), 2 freezes it
// (zero velocities, status CONVERGED, so later launches only evaluate it), 0 leaves it.
__global__ void k_refill(int n_rep, int N, const int *atom_off, const int *mode, const float *src, float *pos,
                         float *vel, float *fdt, float *falpha, int *fnpos, unsigned *status, float dt0, float a0) {
    const int r = blockIdx.x;
    if (r >= n_rep) return;
    const int m = mode[r];
    if (m != 1 && m != 2) return;
    const int b = atom_off[r], n = atom_off[r + 1] - b;
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        const int g = b + a;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (m == 1) pos[g + (size_t)c * N] = src[g + (size_t)c * N];
            vel[g + (size_t)c * N] = 0.f;
        }
    }
    if (threadIdx.x == 0) {
        if (m == 1) {
            if (fdt) fdt[r] = dt0;
            if (falpha) falpha[r] = a0;
            if (fnpos) fnpos[r] = 0;
            status[r] = 0u;
        } else {
            status[r] = GFF_REP_CONVERGED;
        }
    }
}

extern "C" gff_status gff_refill(const gff_plan *plan, const int *d_mode, const float *d_pos_src, float dt0,
                                 float alpha0, const gff_state *state, void *stream) {
    if (!plan || !state || !state->d_pos || !state->d_vel || !state->d_status) return GFF_EINVAL;
    if (plan->n_rep > 0 && (!d_mode || !d_pos_src)) return GFF_EINVAL;
    if (plan->n_rep == 0) return GFF_OK;
    hipLaunchKernelGGL(k_refill, dim3(plan->n_rep), dim3(64), 0, (hipStream_t)stream, plan->n_rep, plan->n_atoms,
                       plan->d_atom_off, d_mode, d_pos_src, state->d_pos, state->d_vel, state->d_fire_dt,
                       state->d_fire_alpha, state->d_fire_npos, state->d_status, dt0, alpha0);
    return hip_status(hipGetLastError());
}

