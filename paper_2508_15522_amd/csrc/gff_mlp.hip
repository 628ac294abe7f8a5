// Learned pose proposer: a 4-layer MLP (width 256, SiLU) from [64-d noise | 32-d type
// embedding] to the 41-wide pose encoding, with hand-written BF16 MFMA GEMMs (FP32
// accumulation), backward pass, Adam with FP32 master weights, IMLE candidate selection
// (Li & Malik 2018) and Philox-based Gaussian noise.
//
// GEMM: C[M x N] = A[M x K] B[K x N], A and B in BF16 read through arbitrary element strides
// (so transposed operands need no copies), tiles of 64 x 64 per 256-thread block staged
// through LDS, each wave owning a 32 x 32 sub-tile of 2 x 2 v_mfma_f32_16x16x32_bf16.
// Operands contiguous along k or along their row index are staged with 16-byte loads, the
// next k-slice's loads in flight during the current slice's MFMAs.  Products with few
// output tiles and a long K (the weight gradients) split K over blocks into FP32 partials
// that a second kernel sums in split order.  Every output element is reduced in one fixed
// order: results are deterministic.
#include "gff_internal.hpp"
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace gff {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kNoise = 64, kEmb = 32, kIn = kNoise + kEmb, kWidth = 256, kOut = 41;

// Round-to-nearest-even FP32 -> BF16 bits (NaN kept quiet).
__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

struct GemmArgs {
    int M, N, K;
    const unsigned short *A; long sam, sak;      // A(m,k) = A[m*sam + k*sak]
    const unsigned short *B; long sbk, sbn;      // B(k,n) = B[k*sbk + n*sbn]
    const float *bias;                           // [N] or null
    int act;                                     // 0 none, 1 SiLU
    float *C; long ldc;                          // FP32 output (pre-activation if Cpre is null), or null
    float *Cpre; long ldp;                       // FP32 pre-activation copy, or null
    unsigned short *Cb; long ldb;                // BF16 output (after activation), or null
    int accumulate;                              // C += result (FP32 output only)
    int modeA, modeB;                            // staging layout of each operand (StageMode)
    int kchunk;                                  // K range of one blockIdx.z (a multiple of 32)
    float *part;                                 // split K: partial sums [gridDim.z][M][N]; null: none
};

// How a thread stages its 8 elements of a 64-row x 32-k operand slice.  K_*: 8 consecutive k
// of one row (thread t: row t/4, k 8(t%4)..+7); R_*: 8 consecutive rows at one k (thread t:
// k t/8, rows 8(t%8)..+7).  *_VEC: one 16-byte load where the 8 elements are in range.
enum StageMode { K_ELEM = 0, K_VEC = 1, R_VEC = 2, R_ELEM = 3 };

// Load this thread's 8 elements of X(row, k) = X[row*srow + k*sk], rows [r0, r0+64) of R,
// k [k0, k0+32) of those below kend; zero outside.
__device__ __forceinline__ uint4 stage_load(const unsigned short *X, long srow, long sk, int mode, int R, int r0,
                                            int k0, int kend, int tid) {
    const bool kmaj = mode == K_ELEM || mode == K_VEC;
    const int r = r0 + (kmaj ? tid >> 2 : 8 * (tid & 7));
    const int k = k0 + (kmaj ? 8 * (tid & 3) : tid >> 3);
    const long base = (long)r * srow + (long)k * sk;
    if (mode == K_VEC && r < R && k + 8 <= kend) return *reinterpret_cast<const uint4 *>(X + base);
    if (mode == R_VEC && r + 8 <= R && k < kend) return *reinterpret_cast<const uint4 *>(X + base);
    unsigned short e[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int ri = kmaj ? r : r + i, ki = kmaj ? k + i : k;
        e[i] = (ri < R && ki < kend) ? X[(long)ri * srow + (long)ki * sk] : (unsigned short)0;
    }
    uint4 v;
    v.x = e[0] | ((unsigned)e[1] << 16); v.y = e[2] | ((unsigned)e[3] << 16);
    v.z = e[4] | ((unsigned)e[5] << 16); v.w = e[6] | ((unsigned)e[7] << 16);
    return v;
}

// Store the thread's 8 elements into the [row][k] LDS slice.
__device__ __forceinline__ void stage_store(unsigned short (*S)[40], int mode, int tid, uint4 v) {
    if (mode == K_ELEM || mode == K_VEC) {
        *reinterpret_cast<uint4 *>(&S[tid >> 2][8 * (tid & 3)]) = v;
    } else {
        const int k = tid >> 3, r = 8 * (tid & 7);
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            S[r + 2 * i][k] = (unsigned short)(w[i] & 0xffffu);
            S[r + 2 * i + 1][k] = (unsigned short)(w[i] >> 16);
        }
    }
}

// Bias, activation and the stores of one output element.
__device__ __forceinline__ void gemm_epilogue(const GemmArgs &g, int m, int n, float z) {
    if (g.bias) z += g.bias[n];
    if (g.Cpre) g.Cpre[m * g.ldp + n] = z;
    const float y = g.act == 1 ? z / (1.f + __expf(-z)) : z;
    if (g.C) {
        if (g.accumulate) g.C[m * g.ldc + n] += y;
        else g.C[m * g.ldc + n] = y;
    }
    if (g.Cb) g.Cb[m * g.ldb + n] = f2bf(y);
}

__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
    __shared__ __align__(16) unsigned short sA[64][40];   // [m][k], row padded against bank conflicts
    __shared__ __align__(16) unsigned short sB[64][40];   // [n][k]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // tiles that share rows of A go to one XCD (workgroups are dealt to the 8 XCDs in turn)
    const int nt = gridDim.x * gridDim.y, lin = blockIdx.y * gridDim.x + blockIdx.x, per = nt >> 3;
    const int tix = lin < 8 * per ? (lin & 7) * per + (lin >> 3) : lin;
    const int m0 = (tix / gridDim.x) * 64, n0 = (tix % gridDim.x) * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int kb = blockIdx.z * g.kchunk, ke = min(g.K, kb + g.kchunk);
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    uint4 va = stage_load(g.A, g.sam, g.sak, g.modeA, g.M, m0, kb, ke, tid);
    uint4 vb = stage_load(g.B, g.sbn, g.sbk, g.modeB, g.N, n0, kb, ke, tid);
    for (int k0 = kb; k0 < ke; k0 += 32) {
        stage_store(sA, g.modeA, tid, va);
        stage_store(sB, g.modeB, tid, vb);
        __syncthreads();
        if (k0 + 32 < ke) {                         // next slice in flight during the MFMAs
            va = stage_load(g.A, g.sam, g.sak, g.modeA, g.M, m0, k0 + 32, ke, tid);
            vb = stage_load(g.B, g.sbn, g.sbk, g.modeB, g.N, n0, k0 + 32, ke, tid);
        }
        const int row = lane & 15, kq = (lane >> 4) * 8;
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(&sA[wm + 16 * i + row][kq]);
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&sB[wn + 16 * j + row][kq]);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // D layout: lane holds rows 4*(lane/16) + r, column lane % 16 of each 16 x 16 tile
    float *part = g.part ? g.part + (size_t)blockIdx.z * g.M * g.N : nullptr;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                if (part) part[(size_t)m * g.N + n] = acc[i][j][r];
                else gemm_epilogue(g, m, n, acc[i][j][r]);
            }
}

// Split K: the partial sums of the gridDim.z slices added in slice order, then the epilogue.
__global__ void k_splitk_sum(GemmArgs g, int splits) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long mn = (long)g.M * g.N;
    if (i >= mn) return;
    float z = 0.f;
    for (int s = 0; s < splits; ++s) z += g.part[s * mn + i];
    gemm_epilogue(g, (int)(i / g.N), (int)(i % g.N), z);
}

__global__ void k_to_bf16(const float *x, unsigned short *y, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// X0 = [noise | embedding(type)] in BF16, [B][96]
__global__ void k_input(int B, const float *noise, const int *type, const float *emb, unsigned short *X0) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)B * kIn) return;
    const int b = (int)(i / kIn), c = (int)(i % kIn);
    const float v = c < kNoise ? noise[(long)b * kNoise + c] : emb[type[b] * kEmb + (c - kNoise)];
    X0[i] = f2bf(v);
}

// Masked squared distance between outputs and targets in the encoding: entries past the
// type's torsions are masked; the quaternion term takes min(|q - t|^2, |q + t|^2).
__device__ __forceinline__ float enc_dist(const float *y, const float *t, int T, float *sign) {
    float d = 0.f;
    for (int c = 0; c < 5; ++c) { const float e = y[c] - t[c]; d += e * e; }
    float dp = 0.f, dm = 0.f;
    for (int c = 5; c < 9; ++c) {
        const float ep = y[c] - t[c], em = y[c] + t[c];
        dp += ep * ep; dm += em * em;
    }
    if (sign) *sign = dm < dp ? -1.f : 1.f;
    d += fminf(dp, dm);
    for (int c = 9; c < 9 + 2 * T; ++c) { const float e = y[c] - t[c]; d += e * e; }
    return d;
}

// IMLE: for each target the nearest of its K candidate outputs (ties: lowest k).  One
// wavefront per target: lane l scores candidates l, l + 64, ..., then a butterfly keeps the
// smaller distance, the lower index on ties (non-finite distances never win).
__global__ void __launch_bounds__(256) k_imle_select(int n, int K, const float *cand, const float *target,
                                                     const int *ntors, int *best, float *bestd) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= n) return;                                 // uniform across the wavefront
    int bk = 0x7fffffff;
    float bd = 3.4e38f;
    for (int k = lane; k < K; k += 64) {
        const float d = enc_dist(cand + ((long)i * K + k) * kOut, target + (long)i * kOut, ntors[i], nullptr);
        if (d < bd) { bd = d; bk = k; }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const float od = __shfl_xor(bd, o, 64);
        const int ok = __shfl_xor(bk, o, 64);
        if (od < bd || (od == bd && ok < bk)) { bd = od; bk = ok; }
    }
    if (lane == 0) {
        best[i] = bk == 0x7fffffff ? 0 : bk;
        if (bestd) bestd[i] = bd;
    }
}

// dY = (2 / B) (Y - s t) on unmasked entries (s = quaternion sign of the nearer target);
// per-sample loss for the batch mean.
__global__ void k_mse_grad(int B, const float *Y, const float *target, const int *ntors, float *dY, float *loss) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float *y = Y + (long)b * kOut, *t = target + (long)b * kOut;
    float s = 1.f;
    const int T = ntors[b];
    const float d = enc_dist(y, t, T, &s);
    float *g = dY + (long)b * kOut;
    const float sc = 2.f / B;
    for (int c = 0; c < kOut; ++c) {
        float tc = t[c];
        if (c >= 5 && c < 9) tc *= s;
        const bool on = c < 9 + 2 * T;
        g[c] = on ? sc * (y[c] - tc) : 0.f;
    }
    loss[b] = d;
}

// dZ = dH * SiLU'(Z), SiLU'(z) = s (1 + z (1 - s)), s = sigmoid(z); BF16 copy for the next GEMM
__global__ void k_silu_back(long n, const float *dH, const float *Z, float *dZ, unsigned short *dZb) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float z = Z[i], s = 1.f / (1.f + __expf(-z));
    const float v = dH[i] * s * (1.f + z * (1.f - s));
    dZ[i] = v;
    dZb[i] = f2bf(v);
}

// column sums (bias gradients) in a fixed order: one thread per column
// Column sums of a [B][N] matrix: one block per 64 columns, 16 row groups of 64 lanes each
// (rows g, g + 16, ...), then the 16 partial sums of a column in a fixed order.
__global__ void __launch_bounds__(1024) k_colsum(int B, int N, const float *X, long ld, float *out) {
    __shared__ float s_p[16][64];
    const int cx = threadIdx.x & 63, ry = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cx;
    float s = 0.f;
    if (c < N)
        for (int b = ry; b < B; b += 16) s += X[(long)b * ld + c];
    s_p[ry][cx] = s;
    __syncthreads();
    if (ry == 0 && c < N) {
        float t = 0.f;
        for (int g = 0; g < 16; ++g) t += s_p[g][cx];
        out[c] = t;
    }
}

// embedding gradient: per type, sum over samples of dX0[:, 64:96]; one block per type,
// 32 row groups of 32 lanes (rows g, g + 32, ...), partial sums combined in a fixed order
__global__ void __launch_bounds__(1024) k_emb_grad(int B, int n_types, const int *type, const float *dX0,
                                                   float *gemb) {
    __shared__ float s_p[32][kEmb];
    const int t = blockIdx.x, c = threadIdx.x % kEmb, ry = threadIdx.x / kEmb;
    float s = 0.f;
    for (int b = ry; b < B; b += 32)
        if (type[b] == t) s += dX0[(long)b * kIn + kNoise + c];
    s_p[ry][c] = s;
    __syncthreads();
    if (ry == 0) {
        float u = 0.f;
        for (int g = 0; g < 32; ++g) u += s_p[g][c];
        gemb[t * kEmb + c] = u;
    }
}

__global__ void k_adam(long n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi, vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi; v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Standard normals by Box-Muller from Philox counter (i/4, round, 1, 0): each counter gives
// two pairs; uniforms (x >> 8 + 0.5) 2^-24 lie in (0, 1).
__global__ void k_normal(long n, uint32_t k0, uint32_t k1, uint32_t round, float *out) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q * 4 >= n) return;
    uint32_t c[4] = {(uint32_t)q, round, 1u, (uint32_t)(q >> 32)};
    philox4x32_10(c, k0, k1);
    float u[4];
    for (int k = 0; k < 4; ++k) u[k] = ((float)(c[k] >> 8) + 0.5f) * (1.f / 16777216.f);
    float z[4];
    for (int p = 0; p < 2; ++p) {
        const float r = sqrtf(-2.f * __logf(u[2 * p]));
        float s, co;
        sincosf(6.28318530717958647692f * u[2 * p + 1], &s, &co);
        z[2 * p] = r * co; z[2 * p + 1] = r * s;
    }
    for (int k = 0; k < 4; ++k) if (q * 4 + k < n) out[q * 4 + k] = z[k];
}

static unsigned blocks(long n, int t) { return (unsigned)((n + t - 1) / t); }

constexpr int kSplitMax = 16;                 // split-K slices at most
constexpr size_t kPartFloats = (size_t)kSplitMax * kWidth * kWidth;   // partials of the largest weight gradient

static int stage_mode(const unsigned short *X, long srow, long sk) {
    const bool al = ((uintptr_t)X & 15) == 0;
    if (sk == 1) return al && srow % 8 == 0 ? K_VEC : K_ELEM;
    if (srow == 1) return al && sk % 8 == 0 ? R_VEC : R_ELEM;
    return K_ELEM;
}

// part: FP32 scratch for split-K partial sums (kPartFloats), or null for no split.
static void gemm(hipStream_t s, int M, int N, int K, const unsigned short *A, long sam, long sak,
                 const unsigned short *B, long sbk, long sbn, const float *bias, int act, float *C, long ldc,
                 float *Cpre, long ldp, unsigned short *Cb, long ldb, int accumulate = 0, float *part = nullptr) {
    const int gx = (N + 63) / 64, gy = (M + 63) / 64;
    int splits = 1;
    if (part && gx * gy < 64 && K >= 128) {
        splits = std::min(kSplitMax, std::min(K / 64, (512 + gx * gy - 1) / (gx * gy)));
        if ((size_t)splits * M * N > kPartFloats) splits = 1;
    }
    const int kchunk = splits > 1 ? ((K + splits - 1) / splits + 31) / 32 * 32 : std::max(K, 32);
    splits = (K + kchunk - 1) / kchunk;
    if (splits < 1) splits = 1;
    GemmArgs g{M, N, K, A, sam, sak, B, sbk, sbn, bias, act, C, ldc, Cpre, ldp, Cb, ldb, accumulate,
               stage_mode(A, sam, sak), stage_mode(B, sbn, sbk), kchunk, splits > 1 ? part : nullptr};
    hipLaunchKernelGGL(k_gemm_bf16, dim3(gx, gy, splits), dim3(256), 0, s, g);
    if (splits > 1)
        hipLaunchKernelGGL(k_splitk_sum, dim3(blocks((long)M * N, 256)), dim3(256), 0, s, g, splits);
}

}  // namespace gff

using namespace gff;

// parameter layout (FP32 masters): W1 [256][96], b1, W2 [256][256], b2, W3 [256][256], b3,
// W4 [41][256], b4 [41], embedding [n_types][32]
struct gff_mlp_s {
    int n_types;
    size_t n_params;
    size_t off_W[4], off_b[4], off_emb;
    float *d_p, *d_g, *d_m, *d_v;
    unsigned short *d_pb;       // BF16 copy of the parameters
    long step;
};

static const int kDims[5] = {kIn, kWidth, kWidth, kWidth, kOut};

extern "C" size_t gff_mlp_n_params(int n_types) {
    size_t n = 0;
    for (int l = 0; l < 4; ++l) n += (size_t)kDims[l + 1] * kDims[l] + kDims[l + 1];
    return n + (size_t)n_types * kEmb;
}

extern "C" gff_status gff_mlp_create(int n_types, const float *params_h, gff_mlp **out) {
    if (n_types < 1 || !params_h || !out) return GFF_EINVAL;
    auto *m = new gff_mlp_s();
    m->n_types = n_types;
    m->n_params = gff_mlp_n_params(n_types);
    size_t o = 0;
    for (int l = 0; l < 4; ++l) {
        m->off_W[l] = o; o += (size_t)kDims[l + 1] * kDims[l];
        m->off_b[l] = o; o += kDims[l + 1];
    }
    m->off_emb = o;
    const size_t bytes = m->n_params * sizeof(float);
    void *p[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool ok = true;
    for (int i = 0; i < 4; ++i) ok = ok && hipMalloc(&p[i], bytes) == hipSuccess;
    ok = ok && hipMalloc(&p[4], m->n_params * sizeof(unsigned short)) == hipSuccess;
    if (!ok) {
        for (void *q : p) if (q) (void)hipFree(q);
        delete m;
        return GFF_ENOMEM;
    }
    m->d_p = (float *)p[0]; m->d_g = (float *)p[1]; m->d_m = (float *)p[2]; m->d_v = (float *)p[3];
    m->d_pb = (unsigned short *)p[4];
    std::vector<float> z(m->n_params, 0.f);
    if (hipMemcpy(m->d_p, params_h, bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_m, z.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_v, z.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(m->d_g, z.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        for (void *q : p) (void)hipFree(q);
        delete m;
        return GFF_EHIP;
    }
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks((long)m->n_params, 256)), dim3(256), 0, 0, m->d_p, m->d_pb,
                       (long)m->n_params);
    if (hipDeviceSynchronize() != hipSuccess) { gff_mlp_destroy(m); return GFF_EHIP; }
    m->step = 0;
    *out = m;
    return GFF_OK;
}

extern "C" void gff_mlp_destroy(gff_mlp *m) {
    if (!m) return;
    (void)hipFree(m->d_p); (void)hipFree(m->d_g); (void)hipFree(m->d_m); (void)hipFree(m->d_v);
    (void)hipFree(m->d_pb);
    delete m;
}

extern "C" gff_status gff_mlp_get_params(const gff_mlp *m, float *params_h, float *grads_h) {
    if (!m || (!params_h && !grads_h)) return GFF_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return GFF_EHIP;
    if (params_h && hipMemcpy(params_h, m->d_p, m->n_params * 4, hipMemcpyDeviceToHost) != hipSuccess) return GFF_EHIP;
    if (grads_h && hipMemcpy(grads_h, m->d_g, m->n_params * 4, hipMemcpyDeviceToHost) != hipSuccess) return GFF_EHIP;
    return GFF_OK;
}

// workspace: X0 (bf16 B x 96), H1..H3 (bf16 B x 256 each), Z1..Z3 (f32 B x 256 each),
// then for the backward pass dY (f32 B x 41), dYb (bf16), dH / dZ (f32 B x 256), dZb (bf16),
// dX0 (f32 B x 96), loss (f32 B), split-K partial sums of the weight gradients
static size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

extern "C" size_t gff_mlp_workspace_bytes(int batch) {
    const size_t B = (size_t)(batch > 0 ? batch : 0);
    return a256(B * kIn * 2) + 3 * a256(B * kWidth * 2) + 3 * a256(B * kWidth * 4) + a256(B * kOut * 4) +
           a256(B * kOut * 2) + 2 * a256(B * kWidth * 4) + a256(B * kWidth * 2) + a256(B * kIn * 4) + a256(B * 4) +
           a256(kPartFloats * 4);
}

struct MlpWork {
    unsigned short *X0, *H[3];
    float *Z[3], *dY; unsigned short *dYb; float *dH, *dZ; unsigned short *dZb; float *dX0, *loss, *part;
};

static MlpWork carve(void *w, int batch) {
    const size_t B = (size_t)batch;
    char *p = (char *)w;
    MlpWork k;
    k.X0 = (unsigned short *)p; p += a256(B * kIn * 2);
    for (int i = 0; i < 3; ++i) { k.H[i] = (unsigned short *)p; p += a256(B * kWidth * 2); }
    for (int i = 0; i < 3; ++i) { k.Z[i] = (float *)p; p += a256(B * kWidth * 4); }
    k.dY = (float *)p; p += a256(B * kOut * 4);
    k.dYb = (unsigned short *)p; p += a256(B * kOut * 2);
    k.dH = (float *)p; p += a256(B * kWidth * 4);
    k.dZ = (float *)p; p += a256(B * kWidth * 4);
    k.dZb = (unsigned short *)p; p += a256(B * kWidth * 2);
    k.dX0 = (float *)p; p += a256(B * kIn * 4);
    k.loss = (float *)p; p += a256(B * 4);
    k.part = (float *)p;
    return k;
}

// keep_pre: store the pre-activations Z (the backward pass needs them; inference does not)
static void forward(gff_mlp *m, hipStream_t s, int B, const float *noise, const int *type, float *out, MlpWork &k,
                    bool keep_pre) {
    hipLaunchKernelGGL(k_input, dim3(blocks((long)B * kIn, 256)), dim3(256), 0, s, B, noise, type,
                       m->d_p + m->off_emb, k.X0);
    const unsigned short *X = k.X0;
    for (int l = 0; l < 3; ++l) {
        const int din = kDims[l], dout = kDims[l + 1];
        gemm(s, B, dout, din, X, din, 1, m->d_pb + m->off_W[l], 1, din, m->d_p + m->off_b[l], 1, nullptr, 0,
             keep_pre ? k.Z[l] : nullptr, dout, k.H[l], dout);
        X = k.H[l];
    }
    gemm(s, B, kOut, kWidth, X, kWidth, 1, m->d_pb + m->off_W[3], 1, kWidth, m->d_p + m->off_b[3], 0, out, kOut,
         nullptr, 0, nullptr, 0);
}

extern "C" gff_status gff_mlp_forward(gff_mlp *m, int batch, const float *d_noise, const int *d_type, float *d_out,
                                      void *d_work, size_t work_bytes, void *stream) {
    if (!m || batch < 0 || (batch > 0 && (!d_noise || !d_type || !d_out))) return GFF_EINVAL;
    if (batch == 0) return GFF_OK;
    if (!d_work || work_bytes < gff_mlp_workspace_bytes(batch)) return GFF_EWORKSPACE;
    MlpWork k = carve(d_work, batch);
    forward(m, (hipStream_t)stream, batch, d_noise, d_type, d_out, k, false);
    return hip_status(hipGetLastError());
}

// Gradient of the batch-mean masked squared error (quaternion sign chosen per sample) with
// respect to every parameter, into the model's gradient buffer; d_out receives the outputs,
// d_loss[batch] the per-sample distances.  With lr > 0 an Adam step (beta 0.9, 0.999,
// eps 1e-8) follows on the FP32 masters and the BF16 copy is refreshed.
extern "C" gff_status gff_mlp_train_step(gff_mlp *m, int batch, const float *d_noise, const int *d_type,
                                         const float *d_target, const int *d_ntors, float lr, float *d_out,
                                         float *d_loss, void *d_work, size_t work_bytes, void *stream) {
    if (!m || batch < 1 || !d_noise || !d_type || !d_target || !d_ntors || !d_out) return GFF_EINVAL;
    if (!d_work || work_bytes < gff_mlp_workspace_bytes(batch)) return GFF_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const int B = batch;
    MlpWork k = carve(d_work, batch);
    forward(m, s, B, d_noise, d_type, d_out, k, true);
    hipLaunchKernelGGL(k_mse_grad, dim3(blocks(B, 256)), dim3(256), 0, s, B, d_out, d_target, d_ntors, k.dY,
                       d_loss ? d_loss : k.loss);
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks((long)B * kOut, 256)), dim3(256), 0, s, k.dY, k.dYb, (long)B * kOut);
    // layer 4: dW4 = dY^T H3, db4 = colsum dY, dH3 = dY W4
    float *g = m->d_g;
    gemm(s, kOut, kWidth, B, k.dYb, 1, kOut, k.H[2], kWidth, 1, nullptr, 0, g + m->off_W[3], kWidth, nullptr, 0,
         nullptr, 0, 0, k.part);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(1024), 0, s, B, kOut, k.dY, (long)kOut, g + m->off_b[3]);
    gemm(s, B, kWidth, kOut, k.dYb, kOut, 1, m->d_pb + m->off_W[3], kWidth, 1, nullptr, 0, k.dH, kWidth, nullptr, 0,
         nullptr, 0);
    for (int l = 2; l >= 0; --l) {
        const int din = kDims[l], dout = kDims[l + 1];
        hipLaunchKernelGGL(k_silu_back, dim3(blocks((long)B * dout, 256)), dim3(256), 0, s, (long)B * dout, k.dH,
                           k.Z[l], k.dZ, k.dZb);
        const unsigned short *Xin = l == 0 ? k.X0 : k.H[l - 1];
        // dW_l = dZ^T X_in  [dout x din]
        gemm(s, dout, din, B, k.dZb, 1, dout, Xin, din, 1, nullptr, 0, g + m->off_W[l], din, nullptr, 0, nullptr, 0, 0,
             k.part);
        hipLaunchKernelGGL(k_colsum, dim3(blocks(dout, 64)), dim3(1024), 0, s, B, dout, k.dZ, (long)dout,
                           g + m->off_b[l]);
        // dX_in = dZ W_l [B x din]
        float *dX = l == 0 ? k.dX0 : k.dH;
        gemm(s, B, din, dout, k.dZb, dout, 1, m->d_pb + m->off_W[l], din, 1, nullptr, 0, dX, din, nullptr, 0, nullptr,
             0);
    }
    hipLaunchKernelGGL(k_emb_grad, dim3(m->n_types), dim3(1024), 0, s, B, m->n_types, d_type, k.dX0,
                       g + m->off_emb);
    if (lr > 0.f) {
        m->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - powf(b1, (float)m->step), c2 = 1.f - powf(b2, (float)m->step);
        hipLaunchKernelGGL(k_adam, dim3(blocks((long)m->n_params, 256)), dim3(256), 0, s, (long)m->n_params, m->d_p,
                           m->d_g, m->d_m, m->d_v, lr, b1, b2, 1e-8f, c1, c2);
        hipLaunchKernelGGL(k_to_bf16, dim3(blocks((long)m->n_params, 256)), dim3(256), 0, s, m->d_p, m->d_pb,
                           (long)m->n_params);
    }
    return hip_status(hipGetLastError());
}

extern "C" gff_status gff_imle_select(int n, int K, const float *d_cand_out, const float *d_target, const int *d_ntors,
                                      int *d_best, float *d_best_dist, void *stream) {
    if (n < 0 || K < 1 || (n > 0 && (!d_cand_out || !d_target || !d_ntors || !d_best))) return GFF_EINVAL;
    if (n == 0) return GFF_OK;
    hipLaunchKernelGGL(k_imle_select, dim3(blocks(n, 4)), dim3(256), 0, (hipStream_t)stream, n, K, d_cand_out,
                       d_target, d_ntors, d_best, d_best_dist);
    return hip_status(hipGetLastError());
}

extern "C" gff_status gff_normal_philox(long n, uint64_t seed, uint32_t round, float *d_out, void *stream) {
    if (n < 0 || (n > 0 && !d_out)) return GFF_EINVAL;
    if (n == 0) return GFF_OK;
    hipLaunchKernelGGL(k_normal, dim3(blocks((n + 3) / 4, 256)), dim3(256), 0, (hipStream_t)stream, n,
                       (uint32_t)seed, (uint32_t)(seed >> 32), round, d_out);
    return hip_status(hipGetLastError());
}

__global__ void k_gather_rows(int n, int len, const float *src, int K, const int *idx, float *dst) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)n * len) return;
    const int r = (int)(i / len), c = (int)(i % len);
    int k = idx[r];
    k = k < 0 ? 0 : (k >= K ? K - 1 : k);          // never read outside the row group
    dst[i] = src[((long)r * K + k) * len + c];
}

// dst[r][:] = src[r * K + idx[r]][:] (rows of `len` floats; idx[r] in [0, K))
extern "C" gff_status gff_gather_rows(int n, int len, const float *d_src, int K, const int *d_idx, float *d_dst,
                                      void *stream) {
    if (n < 0 || len < 1 || K < 1 || (n > 0 && (!d_src || !d_idx || !d_dst))) return GFF_EINVAL;
    if (n == 0) return GFF_OK;
    hipLaunchKernelGGL(k_gather_rows, dim3(blocks((long)n * len, 256)), dim3(256), 0, (hipStream_t)stream, n, len,
                       d_src, K, d_idx, d_dst);
    return hip_status(hipGetLastError());
}

extern "C" size_t gff_gemm_bf16_workspace_bytes(void) { return kPartFloats * sizeof(float); }

// strided GEMM on the MLP's tile, split K when a workspace is given
extern "C" gff_status gff_gemm_bf16_strided(int M, int N, int K, const void *d_A, long sam, long sak, const void *d_B,
                                            long sbk, long sbn, float *d_C, long ldc, void *d_work, size_t work_bytes,
                                            void *stream) {
    if (M < 0 || N < 0 || K < 0 || !d_A || !d_B || !d_C) return GFF_EINVAL;
    if (sam < 1 || sak < 1 || sbk < 1 || sbn < 1 || ldc < N) return GFF_EINVAL;
    if (d_work && work_bytes < gff_gemm_bf16_workspace_bytes()) return GFF_EWORKSPACE;
    if (M == 0 || N == 0) return GFF_OK;
    gemm((hipStream_t)stream, M, N, K, (const unsigned short *)d_A, sam, sak, (const unsigned short *)d_B, sbk, sbn,
         nullptr, 0, d_C, ldc, nullptr, 0, nullptr, 0, 0, (float *)d_work);
    return hip_status(hipGetLastError());
}

// plain GEMM entry for tests of the MFMA tile: C = A B, A [M][K], B [K][N] BF16 row-major, C FP32
extern "C" gff_status gff_gemm_bf16(int M, int N, int K, const void *d_A, const void *d_B, float *d_C, void *stream) {
    if (M < 0 || N < 0 || K < 0 || !d_A || !d_B || !d_C) return GFF_EINVAL;
    if (M == 0 || N == 0) return GFF_OK;
    gemm((hipStream_t)stream, M, N, K, (const unsigned short *)d_A, K, 1, (const unsigned short *)d_B, N, 1, nullptr, 0,
         d_C, N, nullptr, 0, nullptr, 0);
    return hip_status(hipGetLastError());
}
