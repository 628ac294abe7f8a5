// GridFF replica kernels for gfx950: per-atom tricubic B-spline interpolation of the
// Pauli/London/Coulomb grids mixed with the atom's (P, L, Q) (Section "Interpolation",
// Eqs. Bspline1D/Bspline; Section "Principles", Eqs. E, E_Coulomb, E_Morse, V_Morse),
// fused with the intramolecular field and a FIRE, velocity-Verlet or Langevin (BAOAB) step,
// with the whole step loop inside one launch (Section "Configuration sampling on GPU").
//
// Mapping: a block holds a pack of same-type replicas, one lane per atom, replicas
// packed densely (no lane rounding to powers of two).  Positions are exchanged through
// LDS (double-buffered by step parity); per-replica sums (|F|^2, F.v, |v|^2, energies)
// are formed by a quad of reducer lanes per replica from LDS partials in a fixed order,
// so results are deterministic and do not depend on how replicas are packed.  In
// relaxation and MD launches each atom's pre-mixed stencil stays in registers and is
// reloaded only when the atom changes grid cell.
#include "gff_internal.hpp"
#include <cmath>
#include <cstring>
#include <algorithm>

namespace gff {

// MODE_FIRE and MODE_FIRE_CHECKED (replica-wide decisions every k-th move only) form no
// energies in the step loop: the final energies come from an evaluation launch after the
// relaxation, at the same final positions.  MODE_FIRE_SCAN (restrained scans) records each
// point's energy inside the loop.
enum { MODE_EVAL = 0, MODE_FIRE = 1, MODE_NVE = 2, MODE_LANGEVIN = 3, MODE_FIRE_CHECKED = 4, MODE_FIRE_SCAN = 5 };
// storage slot of the all-atom comparison mode (no grid: direct substrate sums)
constexpr int STORE_DIRECT = 3;
constexpr int STORE_TRI = GFF_STORE_TRILINEAR;

struct DirectView {
    const float4 *xyza;        // substrate x, y, z, eps e^{2 alpha R}
    const float2 *bq;          // eps e^{alpha R}, q
    int n, nimg;
    float Lx, Ly;
};

struct GridView {
    const void *coef;
    float x0, y0, z0, idx, idy, idz;
    float dx, dy, dz, zmax;              // zmax = nz - 1
    int nx, ny, nzp;                     // nodes per stored column: col_nodes(nz) (B-spline
                                         // storages, z blocks), nz (trilinear)
    float s0, s1, s2;                    // per-channel decode scales (filled on the device)
    const float *scale;                  // F16: device scales [4]; NULL for F32
    unsigned bytes;                      // size of the coefficient array
    __amdgpu_buffer_rsrc_t rsrc;         // buffer resource over the coefficients (device side)
};

// Decode scales of an F16 grid are read on the device (no host round trip).
__device__ __forceinline__ void fetch_scales(GridView &g) {
    if (g.scale) { g.s0 = g.scale[0]; g.s1 = g.scale[1]; g.s2 = g.scale[2]; }
    g.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(g.coef), (short)0, (int)g.bytes, 0x00020000);
}

struct KArgs {
    GridView g;
    DevTopo t;
    float alpha_l2e, alpha, ke;
    const int4 *packs; const int *pack_reps; const int *atom_off;
    int n_packs, N, tres_max, max_pack_reps, topo_words;
    float *pos, *vel;
    float *fdt, *falpha; int *fnpos; unsigned *status;
    float *F; float *E_atom; double *E_rep; float *fnorm; int *steps; double *drift;
    int n_steps, include_intra, drift_every, nmin;
    int check_every;                    // FIRE: replica-wide decisions every k-th move (>= 1)
    float dt, f_conv, max_disp, finc, fdec, a0, falpha_f, dtmax;
    float lg_c1, lg_c2, kT;             // Langevin: exp(-gamma dt), sqrt(1 - c1^2), k_B T
    unsigned seed_lo, seed_hi, round;   // Langevin: Philox key and fourth counter word
    const unsigned *status_in;          // EVAL after a relaxation: its flags (NONFINITE -> NaN energy)
    const int *fixed_atom;              // FIRE restraint: held atom per replica (nullable)
    const float *fixed_pos;             // its position [n_rep][3]
    // FIRE scan (nullable path): the held atom visits path[rep][p] for p = 0 .. n_points-1,
    // each point relaxed to f_conv or mpp moves, then FIRE restarts (dt0, alpha0) at the next
    const float *path;
    int n_points, mpp;
    float dt0;
    double *E_pts; int *steps_pts; unsigned *st_pts; float *pos_pts;
    DirectView d;                       // all-atom comparison mode only
    float half_inv_alpha;               // 1 / (2 alpha): pair energies summed times alpha (FIRE)
};

__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Cubic B-spline weights of the four nodes i-1..i+2 for t in [0,1] and their t-derivatives
// (B(t+1), B(t), B(1-t), B(2-t) of Eq. Bspline).
__device__ __forceinline__ void bspline_weights(float t, float w[4], float d[4]) {
    const float s = 1.f - t, t2 = t * t, s2 = s * s;
    w[0] = s2 * s * (1.f / 6.f);
    w[1] = 2.f / 3.f - t2 + 0.5f * t2 * t;
    w[2] = 2.f / 3.f - s2 + 0.5f * s2 * s;
    w[3] = t2 * t * (1.f / 6.f);
    d[0] = -0.5f * s2;
    d[1] = t * (1.5f * t - 2.f);
    d[2] = s * (2.f - 1.5f * s);
    d[3] = 0.5f * t2;
}

// Cell index q and in-cell offset t in [0,1] of a coordinate r (relative to the grid origin)
// on an axis with spacing h.  The remainder r - q h is formed with a single rounding (fma),
// so t carries no error proportional to |r| / h (far lateral images stay accurate).
__device__ __forceinline__ float cell_split(float r, float h, float ih, float &t) {
    float q = floorf(r * ih);
    float rem = fmaf(-q, h, r);
    if (rem < 0.f) { q -= 1.f; rem += h; }
    else if (rem >= h) { q += 1.f; rem -= h; }
    t = rem * ih;
    return q;
}

// Exact periodic wrap of an integer-valued cell index into [0, n).
__device__ __forceinline__ int wrap_index(float q, int n) {
    int i = (int)fminf(fmaxf(q, -1073741824.f), 1073741824.f);
    if (i < 0 || i >= n) { i %= n; if (i < 0) i += n; }
    return i;
}

template <int STORE>
__device__ __forceinline__ float4 load_node_buf(__amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (STORE == GFF_STORE_F32) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, 0);
        return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), 0.f);
    } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        const unsigned lo = v[0], hi = v[1];
        __half2 a = *reinterpret_cast<const __half2 *>(&lo), b = *reinterpret_cast<const __half2 *>(&hi);
        const float2 fa = __half22float2(a), fb = __half22float2(b);
        return make_float4(fa.x + fb.y, fa.y, fb.x, 0.f);
    }
}

// ---- trilinear scheme (stored nodal value and index-space gradient per channel)
struct TriKey {
    int i, j, k;
    float tx, ty, tz;
    int state;                            // 0 in the grid, 1 above it (zero), 2 non-finite
};

// Cell and in-cell offsets with the domain rules of grid_key (B-spline); a point exactly on
// the last plane uses the cell below it at offset 1.
__device__ __forceinline__ TriKey tri_key(const GridView &g, float x, float y, float z, unsigned &fl) {
    TriKey K{0, 0, 0, 0.f, 0.f, 0.f, 0};
    if (!(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z))) {
        fl |= GFF_REP_NONFINITE;
        K.state = 2;
        return K;
    }
    const float qx = cell_split(x - g.x0, g.dx, g.idx, K.tx);
    const float qy = cell_split(y - g.y0, g.dy, g.idy, K.ty);
    float qz = cell_split(z - g.z0, g.dz, g.idz, K.tz);
    if (qz < 0.f) { qz = 0.f; K.tz = 0.f; fl |= GFF_REP_OUT_OF_DOMAIN; }
    if (qz > g.zmax || (qz == g.zmax && K.tz > 0.f)) { K.state = 1; return K; }
    if (qz == g.zmax) { qz = g.zmax - 1.f; K.tz = 1.f; }
    K.i = wrap_index(qx, g.nx); K.j = wrap_index(qy, g.ny); K.k = (int)qz;
    return K;
}

__device__ __forceinline__ int tri_cell(const GridView &g, const TriKey &K) { return (K.i * g.ny + K.j) * g.nzp + K.k; }

// The cell's 8 corners, each channel's (E, dE/du, dE/dv, dE/dw) mixed with (P, L, Q);
// corner a*4 + b*2 + c is node (i+a, j+b, k+c).
__device__ __forceinline__ void tri_load(const GridView &g, const TriKey &K, float P, float L, float Q, float4 q[8]) {
    const float4 *T = reinterpret_cast<const float4 *>(g.coef);
    const int i1 = K.i + 1 == g.nx ? 0 : K.i + 1, j1 = K.j + 1 == g.ny ? 0 : K.j + 1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const size_t node = ((size_t)(a ? i1 : K.i) * g.ny + (b ? j1 : K.j)) * g.nzp + K.k + c;
                const float4 c0 = T[3 * node], c1 = T[3 * node + 1], c2 = T[3 * node + 2];
                q[4 * a + 2 * b + c] = make_float4(P * c0.x + L * c1.x + Q * c2.x, P * c0.y + L * c1.y + Q * c2.y,
                                                   P * c0.z + L * c1.z + Q * c2.z, P * c0.w + L * c1.w + Q * c2.w);
            }
}

// Trilinear weights on the 8 corners: energy and force (the stored gradient interpolated on
// its own and scaled to a force).
__device__ __forceinline__ float tri_interp(const GridView &g, const float4 q[8], const TriKey &K, float3 &F) {
    float e = 0.f, gu = 0.f, gv = 0.f, gw = 0.f;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const float w = ((m & 4) ? K.tx : 1.f - K.tx) * ((m & 2) ? K.ty : 1.f - K.ty) * ((m & 1) ? K.tz : 1.f - K.tz);
        e += w * q[m].x; gu += w * q[m].y; gv += w * q[m].z; gw += w * q[m].w;
    }
    F = make_float3(-gu * g.idx, -gv * g.idy, -gw * g.idz);
    return e;
}

__device__ __forceinline__ float3 f3(const float4 &p) { return make_float3(p.x, p.y, p.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator*(float s, float3 a) { return make_float3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Sum over the four lanes of a quad (lanes 4q..4q+3) with DPP quad permutations; every
// lane of the quad receives the same value ((v0+v1)+(v2+v3) in either order).
__device__ __forceinline__ float quad_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));  // [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
    return v;
}

__device__ __forceinline__ double quad_sum(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
    v += __longlong_as_double((long long)(((unsigned long long)(unsigned)__builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false) << 32) |
                                          (unsigned)__builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false)));
    const unsigned long long c = (unsigned long long)__double_as_longlong(v);
    lo = (int)(unsigned)c; hi = (int)(unsigned)(c >> 32);
    v += __longlong_as_double((long long)(((unsigned long long)(unsigned)__builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false) << 32) |
                                          (unsigned)__builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false)));
    return v;
}

// Sum over the LPA lanes of one atom (consecutive lanes within a quad); every one of them
// receives the same value.
template <int LPA>
__device__ __forceinline__ float sub_sum(float v) {
    if constexpr (LPA >= 2)
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));  // [1,0,3,2]
    if constexpr (LPA >= 4)
        v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
    return v;
}

// Hand-off of one atom's grid lookup: owner lane -> the quad that gathers for it; k is the
// slot in the stored column of the first plane of the cell's z window (window_node).
struct GridKey { int i, j, k, valid; };

// Owner side: cell indices and in-cell offsets.  Index arithmetic never leaves the grid:
// x, y wrap, z below the first plane is clamped to it (flag OUT_OF_DOMAIN), points above
// the last plane get no stencil (zero), non-finite coordinates none either (flag NONFINITE).
__device__ __forceinline__ GridKey grid_key(const GridView &g, float x, float y, float z, float4 &t, unsigned &fl) {
    GridKey key{0, 0, 0, 0};
    t = make_float4(0.f, 0.f, 0.f, 0.f);
    if (!(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z))) {
        fl |= GFF_REP_NONFINITE;
        return key;
    }
    float tx, ty, tz;
    const float qx = cell_split(x - g.x0, g.dx, g.idx, tx);
    const float qy = cell_split(y - g.y0, g.dy, g.idy, ty);
    float qz = cell_split(z - g.z0, g.dz, g.idz, tz);
    if (qz < 0.f) { qz = 0.f; tz = 0.f; fl |= GFF_REP_OUT_OF_DOMAIN; }
    if (qz > g.zmax || (qz == g.zmax && tz > 0.f)) return key;         // above the grid: zero
    key.i = wrap_index(qx, g.nx); key.j = wrap_index(qy, g.ny); key.k = window_node((int)qz); key.valid = 1;
    t = make_float4(tx, ty, tz, 0.f);
    return key;
}

// Quad side, fetch: lane s of the quad loads slot key.k + s, z node k-1+s of cell k, of
// each of the 16 columns (so the quad reads each column as one contiguous 64-byte (F32) /
// 32-byte (F16) segment inside one z block, hence inside one 128-byte line) and
// mixes the channels with the atom's (P, L, Q): m[4a+b] is the mixed coefficient of
// column (i-1+a, j-1+b) on the lane's plane.
template <int STORE>
__device__ __forceinline__ void quad_fetch(const GridView &g, GridKey key, float P, float L, float Q, int s,
                                           float m[16]) {
    const int i = key.i, j = key.j;
    int ix[4], jy[4];
    ix[0] = (i == 0 ? g.nx : i) - 1; ix[1] = i;
    ix[2] = (i + 1 == g.nx) ? 0 : i + 1; ix[3] = (i + 2 >= g.nx) ? i + 2 - g.nx : i + 2;
    jy[0] = (j == 0 ? g.ny : j) - 1; jy[1] = j;
    jy[2] = (j + 1 == g.ny) ? 0 : j + 1; jy[3] = (j + 2 >= g.ny) ? j + 2 - g.ny : j + 2;
    const float Ps = P * g.s0, Ls = L * g.s1, Qs = Q * g.s2;
    // 32-bit unsigned byte offsets into a buffer resource (out-of-range offsets would read 0)
    constexpr unsigned NB = STORE == GFF_STORE_F32 ? 16 : 8;
    const unsigned col_stride = (unsigned)g.nzp * NB;
    unsigned yoff[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) yoff[b] = (unsigned)jy[b] * col_stride + (unsigned)(key.k + s) * NB;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const unsigned xoff = (unsigned)ix[a] * (unsigned)g.ny * col_stride;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float4 c = load_node_buf<STORE>(g.rsrc, xoff + yoff[b]);
            m[4 * a + b] = Ps * c.x + Ls * c.y + Qs * c.z;
        }
    }
}

// Quad side, split fetch for overlapping the loads with other work: quad_issue loads the
// nodes of x-planes a0, a0+1 (8 columns) of the lane's plane; quad_mix decodes and mixes
// them into m[4 a0 .. 4 a0 + 7] with the same arithmetic as quad_fetch.
struct QuadAddr { unsigned xoff[4], yoff[4]; };
template <int STORE>
__device__ __forceinline__ QuadAddr quad_addr(const GridView &g, int4 ki, int s) {
    const int i = ki.x, j = ki.y;
    int ix[4], jy[4];
    ix[0] = (i == 0 ? g.nx : i) - 1; ix[1] = i;
    ix[2] = (i + 1 == g.nx) ? 0 : i + 1; ix[3] = (i + 2 >= g.nx) ? i + 2 - g.nx : i + 2;
    jy[0] = (j == 0 ? g.ny : j) - 1; jy[1] = j;
    jy[2] = (j + 1 == g.ny) ? 0 : j + 1; jy[3] = (j + 2 >= g.ny) ? j + 2 - g.ny : j + 2;
    constexpr unsigned NB = STORE == GFF_STORE_F32 ? 16 : 8;
    const unsigned col_stride = (unsigned)g.nzp * NB;
    QuadAddr q;
#pragma unroll
    for (int b = 0; b < 4; ++b) q.yoff[b] = (unsigned)jy[b] * col_stride + (unsigned)(ki.z + s) * NB;
#pragma unroll
    for (int a = 0; a < 4; ++a) q.xoff[a] = (unsigned)ix[a] * (unsigned)g.ny * col_stride;
    return q;
}
// Raw node words as loaded (F32: three channel floats; F16: two words of packed halves);
// decoding is left to the mixing step so that nothing waits on the load before then.
template <int STORE> struct RawNode;
template <> struct RawNode<GFF_STORE_F32> { unsigned w[3]; };
template <> struct RawNode<GFF_STORE_F16> { unsigned w[2]; };

template <int STORE>
__device__ __forceinline__ RawNode<STORE> load_raw(__amdgpu_buffer_rsrc_t r, unsigned off) {
    RawNode<STORE> n;
    if constexpr (STORE == GFF_STORE_F32) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, off, 0, 0);
        n.w[0] = v[0]; n.w[1] = v[1]; n.w[2] = v[2];
    } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        n.w[0] = v[0]; n.w[1] = v[1];
    }
    return n;
}

template <int STORE>
__device__ __forceinline__ float mix_raw(const RawNode<STORE> &n, float Ps, float Ls, float Qs) {
    if constexpr (STORE == GFF_STORE_F32) {
        return Ps * __uint_as_float(n.w[0]) + Ls * __uint_as_float(n.w[1]) + Qs * __uint_as_float(n.w[2]);
    } else {
        const unsigned lo = n.w[0], hi = n.w[1];
        const float2 fa = __half22float2(*reinterpret_cast<const __half2 *>(&lo));
        const float2 fb = __half22float2(*reinterpret_cast<const __half2 *>(&hi));
        return Ps * (fa.x + fb.y) + Ls * fa.y + Qs * fb.x;
    }
}

template <int STORE>
__device__ __forceinline__ void quad_issue(const GridView &g, const QuadAddr &q, int a0, RawNode<STORE> c[8]) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) c[4 * a + b] = load_raw<STORE>(g.rsrc, q.xoff[a0 + a] + q.yoff[b]);
}
template <int STORE>
__device__ __forceinline__ void quad_mix(const RawNode<STORE> c[8], float Ps, float Ls, float Qs, int a0, float m[16]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) m[4 * a0 + k] = mix_raw<STORE>(c[k], Ps, Ls, Qs);
}

// Quad side, contraction: the lane's share of the tensor-product sum over its plane; the
// quad sum is the atom's energy and gradient (in grid units).  The z weights enter once
// per lane: E = sum_s wz[s] (...), dE/dz = sum_s dz[s] (...).
__device__ __forceinline__ float4 quad_contract(const float m[16], float4 t, int s, bool valid) {
    float E = 0.f, Ex = 0.f, Ey = 0.f, Ez = 0.f;
    if (valid) {
        float wx[4], dx[4], wy[4], dy[4], wz[4], dz[4];
        bspline_weights(t.x, wx, dx);
        bspline_weights(t.y, wy, dy);
        bspline_weights(t.z, wz, dz);
        const float wzs = s == 0 ? wz[0] : (s == 1 ? wz[1] : (s == 2 ? wz[2] : wz[3]));
        const float dzs = s == 0 ? dz[0] : (s == 1 ? dz[1] : (s == 2 ? dz[2] : dz[3]));
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            float yv = 0.f, yy = 0.f;
#pragma unroll
            for (int b = 0; b < 4; ++b) { yv += wy[b] * m[4 * a + b]; yy += dy[b] * m[4 * a + b]; }
            E += wx[a] * yv; Ex += dx[a] * yv; Ey += wx[a] * yy;
        }
        Ez = E * dzs;
        E *= wzs; Ex *= wzs; Ey *= wzs;
    }
    return make_float4(quad_sum(E), quad_sum(Ex), quad_sum(Ey), quad_sum(Ez));
}

// Linear index of the stencil's first stored slot, the key of a cached stencil (-1: none).
// It fits in an int: the coefficient array is addressed with 32-bit byte offsets.
__device__ __forceinline__ int stencil_id(const GridView &g, int4 ki) {
    return ki.w ? (ki.x * g.ny + ki.y) * g.nzp + ki.z : -1;
}

// Non-bonded pairs (i, j) of this lane's atom i with j in [j0, j1) that are more than two
// bonds apart: Morse with depth eps_i eps_j at R_i + R_j factorised as
// P_i P_j e^{-2 alpha r} - L_i L_j e^{-alpha r}/2, plus k_e Q_i Q_j / r.  Adds the force on i
// to (fx, fy, fz) and the full pair energies to e (the caller halves the sum).  FOLD (the
// FIRE kernels): the Morse factor alpha of -dE/dr is folded into the atom's factors, one
// multiply per pair fewer, and e receives alpha times the pair energies (the caller scales
// the sum by 1 / (2 alpha)); every FIRE kernel forms the same forces.  Ranges are
// block-uniform; consecutive ranges accumulate in the order of one pass over [0, n).
template <int LPA, bool WITH_E, bool FOLD>
__device__ __forceinline__ void pair_range(const KArgs &A, const float4 *sp, const float4 *splq, int rbase, int j0,
                                           int j1, float3 xi, float4 me, uint4 ex, int sub, float &fx, float &fy,
                                           float &fz, float &e) {
    const float keQ = A.ke * me.z;
    const float Pi = FOLD ? A.alpha * me.x : me.x, Li = FOLD ? (0.5f * A.alpha) * me.y : 0.5f * me.y;
    for (int jb = j0 & ~31; jb < j1; jb += 32) {
        const int w = jb >> 5;
        const unsigned m = w == 0 ? ex.x : (w == 1 ? ex.y : (w == 2 ? ex.z : ex.w));
        const int js0 = max(j0, jb), je = min(j1, jb + 32);
        // with several lanes per atom, sub-lane u takes the partners j = u (mod LPA)
        const int js = LPA == 1 ? js0 : js0 + ((sub - js0) & (LPA - 1));
        if constexpr (LPA == 4) {
            // two partners per pass, both read before either is computed: a small batch leaves
            // a wave alone on its SIMD, which would otherwise wait out every LDS read.  (The
            // other lane layouts keep the loop below as written: routed through this helper
            // they compile to more register copies.)
            auto pair = [&](int j, const float4 pj, const float4 qj) {
                const float ddx = xi.x - pj.x, ddy = xi.y - pj.y, ddz = xi.z - pj.z;
                const float r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                const bool skip = (m >> (j - jb)) & 1u;
                const float rinv = skip ? 0.f : __builtin_amdgcn_rsqf(r2);   // as below
                const float r = r2 * rinv;
                const float u = __builtin_amdgcn_exp2f(-A.alpha_l2e * r);
                const float eu = Pi * qj.x * u * u, el = Li * qj.y * u, ec = keQ * qj.z * rinv;
                float g;
                if constexpr (FOLD) g = (2.f * eu - el) + ec * rinv;
                else g = A.alpha * (2.f * eu - el) + ec * rinv;
                const float sc = g * rinv;
                fx += sc * ddx; fy += sc * ddy; fz += sc * ddz;
                if constexpr (WITH_E) {
                    if constexpr (FOLD) e += skip ? 0.f : (eu - el) + A.alpha * ec;
                    else e += skip ? 0.f : (eu - el + ec);
                }
            };
            int j = js;
            for (; j + LPA < je; j += 2 * LPA) {
                const float4 pa = sp[rbase + j], qa = splq[rbase + j];
                const float4 pb = sp[rbase + j + LPA], qb = splq[rbase + j + LPA];
                pair(j, pa, qa);
                pair(j + LPA, pb, qb);
            }
            if (j < je) pair(j, sp[rbase + j], splq[rbase + j]);
        } else {
            // unrolled by two at two lanes per atom only: at one lane per atom the unrolled
            // loop moves spills into the step loop
            constexpr int UNROLL = LPA == 2 ? 2 : 1;
#pragma unroll UNROLL
            for (int j = js; j < je; j += LPA) {
                const float4 pj = sp[rbase + j];
                const float4 qj = splq[rbase + j];
                const float ddx = xi.x - pj.x, ddy = xi.y - pj.y, ddz = xi.z - pj.z;
                const float r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                const bool skip = (m >> (j - jb)) & 1u;
                // an excluded pair (the atom itself included, r2 = 0) gets 1/r = 0: then r = 0,
                // e^{-alpha r} = 1 and the force factor g / r is 0 with no further select
                const float rinv = skip ? 0.f : __builtin_amdgcn_rsqf(r2);
                const float r = r2 * rinv;
                const float u = __builtin_amdgcn_exp2f(-A.alpha_l2e * r);
                const float eu = Pi * qj.x * u * u, el = Li * qj.y * u, ec = keQ * qj.z * rinv;
                float g;                                                    // -dE/dr
                if constexpr (FOLD) g = (2.f * eu - el) + ec * rinv;
                else g = A.alpha * (2.f * eu - el) + ec * rinv;
                const float sc = g * rinv;
                fx += sc * ddx; fy += sc * ddy; fz += sc * ddz;
                if constexpr (WITH_E) {
                    if constexpr (FOLD) e += skip ? 0.f : (eu - el) + A.alpha * ec;
                    else e += skip ? 0.f : (eu - el + ec);
                }
            }
        }
    }
}

// Bonds and angles incident to this lane's atom (each term evaluated by every
// participant for its own slot; the slot-0 participant carries the energy).
template <int LPA, bool WITH_E>
__device__ __forceinline__ float bond_angle_terms(const KArgs &A, const float4 *sp, int rbase, int abase, int at,
                                                  int sub, float3 xi, float &fx, float &fy, float &fz) {
    float e = 0.f;
    const int4 ia = A.t.incA[abase + at];
    for (int b = ia.x + sub; b < ia.x + ia.y; b += LPA) {
        const BondInc bi = A.t.bnd[b];
        const float3 d = xi - f3(sp[rbase + bi.other]);
        const float d2 = dot(d, d), rinv = __builtin_amdgcn_rsqf(d2);
        const float dr = d2 * rinv - bi.r0;
        const float g = bi.k * dr * rinv;
        fx -= g * d.x; fy -= g * d.y; fz -= g * d.z;
        if (WITH_E && bi.slot == 0) e += 0.5f * bi.k * dr * dr;
    }
    for (int q = ia.z + sub; q < ia.z + ia.w; q += LPA) {
        const AngInc ai = A.t.ang[q];
        const int ia0 = ai.abcs & 0xff, ib = (ai.abcs >> 8) & 0xff, ic = (ai.abcs >> 16) & 0xff, slot = ai.abcs >> 24;
        const float3 pa = f3(sp[rbase + ia0]), pb = f3(sp[rbase + ib]), pc = f3(sp[rbase + ic]);
        const float3 u = pa - pb, v = pc - pb;
        const float uu = dot(u, u), vv = dot(v, v);
        const float inv = __builtin_amdgcn_rsqf(uu * vv);
        const float cs = dot(u, v) * inv;
        const float de = ai.k * (cs - ai.cos0);
        const float3 ga = inv * v - (cs * __builtin_amdgcn_rcpf(uu)) * u;
        const float3 gc = inv * u - (cs * __builtin_amdgcn_rcpf(vv)) * v;
        float3 gs = slot == 0 ? ga : (slot == 2 ? gc : make_float3(-ga.x - gc.x, -ga.y - gc.y, -ga.z - gc.z));
        fx -= de * gs.x; fy -= de * gs.y; fz -= de * gs.z;
        if (WITH_E && slot == 0) e += 0.5f * ai.k * (cs - ai.cos0) * (cs - ai.cos0);
    }
    return e;
}

// One torsion term 1/2 V (1 - cos(n phi - phi0)) evaluated once: its energy, and the
// per-term data from which each participant's force follows,
//   F_i = A, F_l = B, F_j = -(1+p) A + q B, F_k = p A - (1+q) B,
// with A = -dE/dphi dphi/dr_i, B = -dE/dphi dphi/dr_l, p = b1.b2/|b2|^2, q = b3.b2/|b2|^2.
__device__ __forceinline__ float torsion_term(const TorDef td, const float4 *sp, int rbase, float4 &oA, float4 &oB) {
    const int i0 = td.ijkln & 0x7f, i1 = (td.ijkln >> 7) & 0x7f, i2 = (td.ijkln >> 14) & 0x7f;
    const int i3 = (td.ijkln >> 21) & 0x7f, nmul = (td.ijkln >> 28) & 0xf;
    const float3 p0 = f3(sp[rbase + i0]), p1 = f3(sp[rbase + i1]), p2 = f3(sp[rbase + i2]), p3 = f3(sp[rbase + i3]);
    const float3 b1 = p1 - p0, b2 = p2 - p1, b3 = p3 - p2;
    const float3 mm = cross(b1, b2), nn = cross(b2, b3);
    const float m2 = dot(mm, mm), n2 = dot(nn, nn), bb = dot(b2, b2);
    if (m2 < 1e-12f || n2 < 1e-12f) {             // collinear: dihedral undefined, term dropped
        oA = make_float4(0.f, 0.f, 0.f, 0.f); oB = oA;
        return 0.f;
    }
    const float ibb = __builtin_amdgcn_rcpf(bb), lb = bb * __builtin_amdgcn_rsqf(bb);
    const float inv = __builtin_amdgcn_rsqf(m2 * n2);
    const float c1 = dot(mm, nn) * inv, s1 = lb * dot(b1, nn) * inv;    // cos phi, sin phi
    float cn = c1, sn = s1;
    for (int r = 1; r < nmul; ++r) {                                    // (cos n phi, sin n phi)
        const float c2 = cn * c1 - sn * s1;
        sn = sn * c1 + cn * s1; cn = c2;
    }
    const float carg = cn * td.c0 + sn * td.s0, sarg = sn * td.c0 - cn * td.s0;
    const float dEdphi = 0.5f * td.V * (float)nmul * sarg;
    const float fa = dEdphi * lb * __builtin_amdgcn_rcpf(m2), fb = -dEdphi * lb * __builtin_amdgcn_rcpf(n2);
    oA = make_float4(fa * mm.x, fa * mm.y, fa * mm.z, dot(b1, b2) * ibb);   // A = fa mm, B = fb nn
    oB = make_float4(fb * nn.x, fb * nn.y, fb * nn.z, dot(b3, b2) * ibb);
    return 0.5f * td.V * (1.f - carg);
}

// All-atom comparison (Section "Configuration sampling on GPU"): the molecule-substrate
// energy of this lane's atom summed directly over every substrate atom of the cell and of
// its lateral images |a|, |b| <= nimg, with the grids' Pauli/London factorisation and bare
// Coulomb, no cutoff.  The substrate index is wave-uniform, so its data arrive through
// scalar loads.
__device__ __forceinline__ float direct_terms(const KArgs &A, float3 xi, float4 me, float3 &F) {
    const DirectView &d = A.d;
    float e = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
    const float keQ = A.ke * me.z;
    for (int j = 0; j < d.n; ++j) {
        const float4 s = d.xyza[j];
        const float2 t = d.bq[j];
        const float ap = me.x * s.w, al = me.y * t.x, ac = keQ * t.y;
        const float ddz = xi.z - s.z;
        for (int a = -d.nimg; a <= d.nimg; ++a) {
            const float ddx = xi.x - (s.x + (float)a * d.Lx);
            for (int b = -d.nimg; b <= d.nimg; ++b) {
                const float ddy = xi.y - (s.y + (float)b * d.Ly);
                const float r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float u = __builtin_amdgcn_exp2f(-A.alpha_l2e * (r2 * rinv));
                const float ep = ap * u * u, el = al * u, ec = ac * rinv;
                e += ep + el + ec;
                const float sc = (A.alpha * (2.f * ep + el) + ec * rinv) * rinv;   // -dE/dr / r
                fx += sc * ddx; fy += sc * ddy; fz += sc * ddz;
            }
        }
    }
    F = make_float3(fx, fy, fz);
    return e;
}

// CACHE: keep each lane's pre-mixed stencil planes (4 / LPA of them, 16 values each) in
// registers from step to step; this needs blocks of at most 512 threads.
// LPA: lanes per atom (1, 2, 4).  The LPA consecutive lanes of an atom slot hold the same
// position and velocity and integrate identically; they split the atom's non-bonded
// partners, bonded incidences and the replica's torsion terms, and their partial forces and
// energies are summed across them (fixed order, identical on every sub-lane).  With
// LPA = 4 each quad gathers for its own atom; fewer slots per wave mean fewer gather rounds.
template <int STORE, int MODE, bool CACHE, int LPA>
__global__ void __launch_bounds__(CACHE ? 512 : 1024) __attribute__((amdgpu_waves_per_eu(CACHE ? 3 : 1)))
k_replicas(KArgs A) {
    static_assert(LPA == 1 || ((STORE == GFF_STORE_F32 || STORE == GFF_STORE_F16) && MODE != MODE_EVAL),
                  "several lanes per atom only for B-spline relaxation and dynamics");
    constexpr bool FIRE = MODE == MODE_FIRE || MODE == MODE_FIRE_CHECKED || MODE == MODE_FIRE_SCAN;
    constexpr bool WANT_E = MODE != MODE_FIRE && MODE != MODE_FIRE_CHECKED;   // energies in the loop
    extern __shared__ __align__(16) unsigned char smem[];
    const int BT = blockDim.x, tid = threadIdx.x;
    const int NS = BT / LPA;                     // atom slots of the block
    const int slot = tid / LPA, sub = tid & (LPA - 1);
    constexpr int R = 4 / LPA;                   // gather rounds per wave
    // LDS, one float4 slot per lane in each array:
    //   s_pos0/s_pos1  positions (double-buffered by step parity); the buffer of the other
    //                  parity carries the gather results during a step
    //   s_red          per-atom partial sums (float4 FIRE, double2 NVE) and, earlier in the
    //                  step, the gather offsets
    //   s_sum          per-replica sums (index = replica in pack) and, earlier, gather indices
    //   s_plq          per-lane P, L, Q, 1/(m 103.6427)
    //   s_tres         torsion-term results, 2 float4 per term and replica
    //   s_topo         the pack's molecule type: torsion block
    //   s_drift        per-replica NVE drift record (6 doubles)
    //   s_nf           per-replica non-finite flags (NVE)
    float4 *s_pos0 = reinterpret_cast<float4 *>(smem);
    float4 *s_pos1 = s_pos0 + NS;
    float4 *s_red = s_pos1 + NS;
    float4 *s_sum = s_red + NS;
    float4 *s_plq = s_sum + NS;
    float4 *s_tres = s_plq + NS;
    int4 *s_topo = reinterpret_cast<int4 *>(s_tres + 2 * A.tres_max);
    double *s_drift = reinterpret_cast<double *>(s_topo + A.topo_words);
    int *s_nf = reinterpret_cast<int *>(s_drift + 6 * A.max_pack_reps);
    int *s_any = s_nf + NS;
    double2 *s_red64 = reinterpret_cast<double2 *>(s_red);
    float4 *s_gt = s_red;
    int4 *s_gi = reinterpret_cast<int4 *>(s_sum);
    const int N = A.N;
    const int wl = tid & 63, wb = tid - wl, quad_s = wl & 3;
    const int wbs = wb / LPA;                    // the wave's first atom slot
    GridView gv = A.g;
    if constexpr (STORE == GFF_STORE_F32 || STORE == GFF_STORE_F16) fetch_scales(gv);

    for (int pk = blockIdx.x; pk < A.n_packs; pk += gridDim.x) {
        const int4 pinfo = A.packs[pk];
        const TypeInfo ti = A.t.types[pinfo.x];
        const int n = ti.n, nrep = pinfo.y, abase = ti.abase, nt = ti.nt;
        const int lr = slot / n, at = slot - lr * n;
        const bool active = lr < nrep;
        const int rbase = active ? lr * n : 0;
        int rep = 0, g = 0;
        float3 x = make_float3(0.f, 0.f, 0.f), v = make_float3(0.f, 0.f, 0.f);
        float4 me = make_float4(0.f, 0.f, 0.f, 0.f);
        uint4 ex = make_uint4(0u, 0u, 0u, 0u);
        float khalf = 0.f;
        float fdt = 0.f, fal = 0.f; int fnp = 0; unsigned st = GFF_REP_NONFINITE;
        bool held = false;                // FIRE restraint: this atom is held in place
        if (active) {
            rep = A.pack_reps[pinfo.z + lr];
            g = A.atom_off[rep] + at;
            x = make_float3(A.pos[g], A.pos[g + N], A.pos[g + 2 * N]);
            if (MODE != MODE_EVAL) v = make_float3(A.vel[g], A.vel[g + N], A.vel[g + 2 * N]);
            me = A.t.plqm[abase + at];
            ex = A.t.excl[abase + at];
            khalf = A.t.khalf[abase + at];
            st = MODE == MODE_EVAL ? 0u : A.status[rep];
            if (FIRE) { fdt = A.fdt[rep]; fal = A.falpha[rep]; fnp = A.fnpos[rep]; }
            if (FIRE && A.fixed_atom != nullptr && A.fixed_atom[rep] == at) {
                held = true;
                const float *tp = A.path ? A.path + 3 * (size_t)rep * A.n_points : A.fixed_pos + 3 * rep;
                x = make_float3(tp[0], tp[1], tp[2]);
                v = make_float3(0.f, 0.f, 0.f);
            }
        }
        if (sub == 0) s_plq[slot] = me;
        if (tid < NS) s_nf[tid] = 0;
        for (int k = tid; k < ti.blob_words; k += BT) s_topo[k] = A.t.blob[ti.blob_off + k];
        if (MODE == MODE_NVE)
            for (int k = tid; k < 6 * nrep; k += BT) s_drift[k] = 0.0;
        if (tid == 0) { s_any[0] = 0; s_any[1] = 0; s_any[2] = 0; }
        lds_sync();

        unsigned fl = 0;                 // per-lane sticky flags (out of domain, non-finite position)
        float3 F = make_float3(0.f, 0.f, 0.f);
        float e_atom = 0.f, e_grid = 0.f, fnorm = 0.f;
        int steps = 0;
        int pt = 0, spt = 0;             // scan: current point, moves made at it
        const bool entered_conv = (st & GFF_REP_CONVERGED) != 0;
        bool live = active && !(st & GFF_REP_NONFINITE);
        // per-replica sums: a quad of reducer lanes per replica (lane q adds atoms q, q+4, ...,
        // then a quad sum), one lane for molecules of fewer than four atoms
        const int RL = n >= 4 ? 4 : 1;
        const int rr = RL == 4 ? (tid >> 2) : tid, rq = tid - rr * RL;
        const bool reducer = rr < nrep;
        float cm[R][16];                        // cached pre-mixed stencil planes (CACHE)
        int cid[R];                             // their stencil ids (-1: none)
#pragma unroll
        for (int r = 0; r < R; ++r) cid[r] = -1;
        float4 tq[8];                           // trilinear: the cell's pre-mixed corners
        int tcid = -1;                          // their cell (CACHE; -1: none)

        const int total = (MODE == MODE_EVAL) ? 0 : A.n_steps;
        // "any replica of the pack still live" flag of step it lives in slot it % 3: a slot
        // is cleared two steps before it is used again, so a wave that lags behind (no block
        // barrier between two steps' barrier A in some modes) still reads its own step's flag.
        // The slot is derived from the step, not carried from step to step: a loop-carried
        // counter made the register allocator shuffle the cached stencils every step.
        for (int it = 0; it <= total; ++it) {
            const unsigned aslot = (unsigned)it % 3u;
            const int par = it & 1;
            float4 *sp = par ? s_pos1 : s_pos0;
            float4 *s_gres = par ? s_pos0 : s_pos1;
            if (MODE == MODE_NVE && it > 0 && live) {       // velocity Verlet: half kick, drift
                v = v + (0.5f * A.dt * me.w) * F;
                x = x + A.dt * v;
            }
            if (MODE == MODE_LANGEVIN && it > 0 && live) {  // BAOAB: half kick, half drift,
                v = v + (0.5f * A.dt * me.w) * F;            // Ornstein-Uhlenbeck, half drift
                x = x + (0.5f * A.dt) * v;
                const float3 xi = philox_normal3((uint32_t)rep, (uint32_t)at, (uint32_t)it, A.round,
                                                 A.seed_lo, A.seed_hi);
                v = A.lg_c1 * v + (A.lg_c2 * sqrtf(A.kT * me.w)) * xi;
                x = x + (0.5f * A.dt) * v;
            }
            if (live) s_any[aslot] = 1;
            if (tid == 0) s_any[aslot == 2u ? 0u : aslot + 1u] = 0;
            if (sub == 0) sp[slot] = make_float4(x.x, x.y, x.z, 0.f);
            lds_sync();                                          // A: positions visible
            if (s_any[aslot] == 0) break;                        // every replica of the pack is done
            if (MODE == MODE_NVE && live && s_nf[lr]) { st |= GFF_REP_NONFINITE; live = false; }

            float pfx = 0.f, pfy = 0.f, pfz = 0.f, pe = 0.f;    // non-bonded pair sums (CACHE)
            // --- grid: owner hand-off, then four quad-gather rounds within the wave (in the
            // all-atom comparison mode: the direct substrate sum instead)
            if constexpr (STORE == STORE_DIRECT) {
                if (!(__builtin_isfinite(x.x) && __builtin_isfinite(x.y) && __builtin_isfinite(x.z))) {
                    if (live) fl |= GFF_REP_NONFINITE;
                    e_grid = __builtin_nanf("");
                    F = make_float3(e_grid, e_grid, e_grid);
                } else if (live) {
                    e_grid = direct_terms(A, x, me, F);
                } else {
                    e_grid = 0.f;
                    F = make_float3(0.f, 0.f, 0.f);
                }
            } else if constexpr (STORE == STORE_TRI) {
                // per lane: the cell's 8 corners (kept across steps while the atom stays in
                // the cell when CACHE), trilinear weights
                e_grid = 0.f;
                F = make_float3(0.f, 0.f, 0.f);
                if (live) {
                    unsigned fk = 0;
                    const TriKey K = tri_key(gv, x.x, x.y, x.z, fk);
                    fl |= fk;
                    if (K.state == 2) {
                        e_grid = __builtin_nanf("");
                        F = make_float3(e_grid, e_grid, e_grid);
                    } else if (K.state == 0) {
                        const int cell = tri_cell(gv, K);
                        if (!CACHE || cell != tcid) tri_load(gv, K, me.x, me.y, me.z, tq);
                        tcid = cell;
                        e_grid = tri_interp(gv, tq, K, F);
                    }
                }
            } else {
                float4 t;
                unsigned fk = 0;
                GridKey key = grid_key(gv, x.x, x.y, x.z, t, fk);
                if (!live) key.valid = 0;
                else fl |= fk;
                if (sub == 0) {
                    s_gi[slot] = make_int4(key.i, key.j, key.k, key.valid);
                    s_gt[slot] = t;
                }
                wave_sync();
                if constexpr (CACHE) {
                    // stencils stay in registers across steps; a quad reloads its plane
                    // only when its atom has moved to another cell.  The reload of each
                    // half plane is issued before a slice of the non-bonded pair loop and
                    // mixed after it, so the pair work covers the memory latency.
                    const bool pairs = A.include_intra && live;
#pragma unroll
                    for (int rnd = 0; rnd < R; ++rnd) {
                        const int o = wbs + 16 * rnd + (wl >> 2);
                        const int4 ki = s_gi[o];
                        const int id = stencil_id(gv, ki);
                        const bool need = id != cid[rnd] && id >= 0;
                        if constexpr (LPA == 4) {
                            // one cached plane leaves registers to issue the whole reload at
                            // once: one memory latency per step, covered by the pair loop
                            RawNode<STORE> c[8], c2[8];
                            if (need) {
                                const QuadAddr qa = quad_addr<STORE>(gv, ki, quad_s);
                                quad_issue<STORE>(gv, qa, 0, c);
                                quad_issue<STORE>(gv, qa, 2, c2);
                            }
                            if (pairs) pair_range<LPA, WANT_E, FIRE>(A, sp, s_plq, rbase, (2 * rnd) * n / (2 * R),
                                                       (2 * rnd + 2) * n / (2 * R), x, me, ex, sub, pfx, pfy, pfz, pe);
                            if (need) {
                                const float4 po = s_plq[o];
                                quad_mix<STORE>(c, po.x * gv.s0, po.y * gv.s1, po.z * gv.s2, 0, cm[rnd]);
                                quad_mix<STORE>(c2, po.x * gv.s0, po.y * gv.s1, po.z * gv.s2, 2, cm[rnd]);
                            }
                        } else {
                            RawNode<STORE> c[8];
                            if (need) quad_issue<STORE>(gv, quad_addr<STORE>(gv, ki, quad_s), 0, c);
                            if (pairs) pair_range<LPA, WANT_E, FIRE>(A, sp, s_plq, rbase, (2 * rnd) * n / (2 * R),
                                                       (2 * rnd + 1) * n / (2 * R), x, me, ex, sub, pfx, pfy, pfz, pe);
                            if (need) {
                                const float4 po = s_plq[o];
                                quad_mix<STORE>(c, po.x * gv.s0, po.y * gv.s1, po.z * gv.s2, 0, cm[rnd]);
                                quad_issue<STORE>(gv, quad_addr<STORE>(gv, ki, quad_s), 2, c);
                            }
                            if (pairs) pair_range<LPA, WANT_E, FIRE>(A, sp, s_plq, rbase, (2 * rnd + 1) * n / (2 * R),
                                                       (2 * rnd + 2) * n / (2 * R), x, me, ex, sub, pfx, pfy, pfz, pe);
                            if (need) {
                                const float4 po = s_plq[o];
                                quad_mix<STORE>(c, po.x * gv.s0, po.y * gv.s1, po.z * gv.s2, 2, cm[rnd]);
                            }
                        }
                        cid[rnd] = id;
                        const float4 r = quad_contract(cm[rnd], s_gt[o], quad_s, id >= 0);
                        if (quad_s == 0) s_gres[o] = r;
                    }
                } else {
#pragma unroll 1
                    for (int rnd = 0; rnd < R; ++rnd) {
                        const int o = wbs + 16 * rnd + (wl >> 2);
                        const int4 ki = s_gi[o];
                        const float4 ko = s_gt[o];
                        const float4 po = s_plq[o];
                        float m[16];
                        if (ki.w) quad_fetch<STORE>(gv, GridKey{ki.x, ki.y, ki.z, ki.w}, po.x, po.y, po.z, quad_s, m);
                        const float4 r = quad_contract(m, ko, quad_s, ki.w != 0);
                        if (quad_s == 0) s_gres[o] = r;
                    }
                }
                wave_sync();
                const float4 r = s_gres[slot];
                e_grid = r.x;
                F = make_float3(-r.y * gv.idx, -r.z * gv.idy, -r.w * gv.idz);
                if (fk & GFF_REP_NONFINITE) {
                    e_grid = __builtin_nanf("");
                    F = make_float3(e_grid, e_grid, e_grid);
                }
            }
            // --- intramolecular: torsion terms once per term, pairs/bonds/angles per atom
            float e_intra = 0.f;
            // this lane's torsion terms (results to LDS), non-bonded pairs, bonds and angles
            auto intra_terms = [&](float &fx, float &fy, float &fz) {
                if constexpr (FIRE) {
                    // a block-uniform loop (its counter stays scalar): fewer registers in the
                    // FIRE kernels, whose register allocation it suits
                    for (int qb = 0; qb < nt; qb += n * LPA) {
                        const int q = qb + at * LPA + sub;
                        if (q < nt) {
                            float4 oA, oB;
                            e_intra += torsion_term(reinterpret_cast<const TorDef *>(s_topo + ti.o_tor)[q], sp, rbase,
                                                    oA, oB);
                            s_tres[2 * (lr * nt + q)] = oA;
                            s_tres[2 * (lr * nt + q) + 1] = oB;
                        }
                    }
                } else {
                    for (int q = at * LPA + sub; q < nt; q += n * LPA) {
                        float4 oA, oB;
                        e_intra += torsion_term(reinterpret_cast<const TorDef *>(s_topo + ti.o_tor)[q], sp, rbase, oA, oB);
                        s_tres[2 * (lr * nt + q)] = oA;
                        s_tres[2 * (lr * nt + q) + 1] = oB;
                    }
                }
                if constexpr (CACHE && STORE != STORE_TRI) {
                    fx = pfx; fy = pfy; fz = pfz;
                    e_intra += (FIRE ? A.half_inv_alpha : 0.5f) * pe;
                } else {
                    float e = 0.f;
                    pair_range<LPA, WANT_E, FIRE>(A, sp, s_plq, rbase, 0, n, x, me, ex, sub, fx, fy, fz, e);
                    e_intra += (FIRE ? A.half_inv_alpha : 0.5f) * e;
                }
                e_intra += bond_angle_terms<LPA, WANT_E>(A, sp, rbase, abase, at, sub, x, fx, fy, fz);
            };
            // the atom's shares of its incident torsion terms: F_i = A, F_j = -(1+p) A + q B,
            // F_k = p A - (1+q) B, F_l = B (incidence code: term << 2 | slot)
            auto torsion_shares = [&](float &fx, float &fy, float &fz) {
                const int *tinc = reinterpret_cast<const int *>(s_topo + ti.o_tinc);
                if constexpr (MODE == MODE_NVE) {
                    // one branch-free loop per slot group (the incidences are stored grouped)
                    const int4 *itg = reinterpret_cast<const int4 *>(s_topo + ((n + 1) >> 1));
                    const int4 r = itg[at];
                    const int e3 = itg[at + 1].x;
                    const float4 *tr = s_tres + 2 * lr * nt;
                    for (int c = r.x + sub; c < r.y; c += LPA) {
                        const float4 ra = tr[2 * (tinc[c] >> 2)];
                        fx += ra.x; fy += ra.y; fz += ra.z;
                    }
                    for (int c = r.y + sub; c < r.z; c += LPA) {
                        const int q = tinc[c] >> 2;
                        const float4 ra = tr[2 * q], rb = tr[2 * q + 1];
                        const float ca = -(1.f + ra.w);
                        fx += ca * ra.x + rb.w * rb.x; fy += ca * ra.y + rb.w * rb.y; fz += ca * ra.z + rb.w * rb.z;
                    }
                    for (int c = r.z + sub; c < r.w; c += LPA) {
                        const int q = tinc[c] >> 2;
                        const float4 ra = tr[2 * q], rb = tr[2 * q + 1];
                        const float cb = -(1.f + rb.w);
                        fx += ra.w * ra.x + cb * rb.x; fy += ra.w * ra.y + cb * rb.y; fz += ra.w * ra.z + cb * rb.z;
                    }
                    for (int c = r.w + sub; c < e3; c += LPA) {
                        const float4 rb = tr[2 * (tinc[c] >> 2) + 1];
                        fx += rb.x; fy += rb.y; fz += rb.z;
                    }
                } else {
                    // one loop over the incidences, the slot from the code (the FIRE and
                    // Langevin kernels run faster in this form)
                    const int2 itc = reinterpret_cast<const int2 *>(s_topo)[at];
                    for (int c = itc.x + sub; c < itc.x + itc.y; c += LPA) {
                        const int code = tinc[c];
                        const int q = code >> 2, slot = code & 3;
                        const float4 ra = s_tres[2 * (lr * nt + q)], rb = s_tres[2 * (lr * nt + q) + 1];
                        float ca, cb;
                        if (slot == 0) { ca = 1.f; cb = 0.f; }
                        else if (slot == 3) { ca = 0.f; cb = 1.f; }
                        else if (slot == 1) { ca = -(1.f + ra.w); cb = rb.w; }
                        else { ca = ra.w; cb = -(1.f + rb.w); }
                        fx += ca * ra.x + cb * rb.x; fy += ca * ra.y + cb * rb.y; fz += ca * ra.z + cb * rb.z;
                    }
                }
            };
            if (A.include_intra) {
                if constexpr (LPA == 1) {
                    // (this form keeps the register allocation of the cached stencils stable)
                    if (live) {
                        float fx = 0.f, fy = 0.f, fz = 0.f;
                        intra_terms(fx, fy, fz);
                        F = F + make_float3(fx, fy, fz);
                    }
                    lds_sync();                                  // B: torsion results visible
                    if (live) {
                        float fx = 0.f, fy = 0.f, fz = 0.f;
                        torsion_shares(fx, fy, fz);
                        F = F + make_float3(fx, fy, fz);
                    }
                } else {
                    // partial sums of the atom's sub-lanes, summed across them
                    float fx = 0.f, fy = 0.f, fz = 0.f;
                    if (live) intra_terms(fx, fy, fz);
                    fx = sub_sum<LPA>(fx); fy = sub_sum<LPA>(fy); fz = sub_sum<LPA>(fz);
                    e_intra = sub_sum<LPA>(e_intra);
                    if (live) F = F + make_float3(fx, fy, fz);
                    lds_sync();                                  // B: torsion results visible
                    fx = 0.f; fy = 0.f; fz = 0.f;
                    if (live) torsion_shares(fx, fy, fz);
                    fx = sub_sum<LPA>(fx); fy = sub_sum<LPA>(fy); fz = sub_sum<LPA>(fz);
                    if (live) F = F + make_float3(fx, fy, fz);
                }
            }
            if (live) e_atom = e_grid + e_intra;
            if (FIRE && held) F = make_float3(0.f, 0.f, 0.f);   // the restraint's reaction

            if (MODE == MODE_EVAL) break;

            // (step-derived, not loop-carried: a loop-carried counter here makes the register
            // allocator shuffle the cached stencils between registers every step)
            bool between_checks = false;
            if constexpr (MODE == MODE_FIRE_CHECKED) between_checks = it % A.check_every != 0 && it < total;
            if (between_checks) {
                // a move between checks: no sums over the replica, a plain kick and capped
                // move with the current dt (block-uniform condition: no barrier is skipped
                // by some waves only)
                if (live) {
                    v = v + fdt * F;
                    float3 d = fdt * v;
                    const float l2 = dot(d, d);
                    if (l2 > A.max_disp * A.max_disp) d = (A.max_disp * __builtin_amdgcn_rsqf(l2)) * d;
                    x = x + d;
                    steps++;
                }
            } else if (FIRE) {
                constexpr bool scan = MODE == MODE_FIRE_SCAN;
                if (sub == 0) s_red[slot] = make_float4(dot(F, F), dot(F, v), dot(v, v), scan ? e_atom : 0.f);
                lds_sync();                                      // C: partials visible
                if (reducer) {                                   // reducer lanes of replica rr
                    float ff = 0.f, fv = 0.f, vv = 0.f, ee = 0.f;
#pragma unroll 4
                    for (int j = rq; j < n; j += RL) {
                        const float4 r = s_red[rr * n + j];
                        ff += r.x; fv += r.y; vv += r.z; ee += r.w;
                    }
                    if (RL == 4) { ff = quad_sum(ff); fv = quad_sum(fv); vv = quad_sum(vv); ee = quad_sum(ee); }
                    if (rq == 0) s_sum[rr] = make_float4(ff, fv, vv, ee);
                }
                lds_sync();                                      // D: sums visible
                if (live) {
                    const float4 sm = s_sum[lr];
                    const float ff = sm.x, fv = sm.y, vv = sm.z;
                    fnorm = sqrtf(ff);
                    const bool conv = fnorm < A.f_conv;
                    if (!__builtin_isfinite(ff) || !__builtin_isfinite(fv) || !__builtin_isfinite(vv)) {
                        st |= GFF_REP_NONFINITE; live = false;
                    } else if (entered_conv) {
                        live = false;
                    } else if (scan && (conv || spt >= A.mpp)) {
                        // the point is done: record it, then restart FIRE at the next point
                        const size_t o = (size_t)rep * A.n_points + pt;
                        if (at == 0 && sub == 0) {
                            A.E_pts[o] = (double)sm.w;
                            if (A.steps_pts) A.steps_pts[o] = spt;
                            if (A.st_pts) A.st_pts[o] = conv ? GFF_REP_CONVERGED : GFF_REP_MAXSTEPS;
                        }
                        if (A.pos_pts && sub == 0) {
                            const size_t N3 = 3 * (size_t)N;
                            A.pos_pts[pt * N3 + g] = x.x; A.pos_pts[pt * N3 + g + N] = x.y;
                            A.pos_pts[pt * N3 + g + 2 * N] = x.z;
                        }
                        ++pt; spt = 0;
                        if (pt == A.n_points) {
                            if (conv) st |= GFF_REP_CONVERGED;
                            live = false;
                        } else {
                            v = make_float3(0.f, 0.f, 0.f);
                            fdt = A.dt0; fal = A.a0; fnp = 0;
                            if (held) {
                                const float *tp = A.path + 3 * ((size_t)rep * A.n_points + pt);
                                x = make_float3(tp[0], tp[1], tp[2]);
                            }
                        }
                    } else if (!scan && conv) {
                        st |= GFF_REP_CONVERGED; live = false;
                    } else if (scan || it < total) {
                        float a = fal, dt = fdt;
                        const float vn = sqrtf(vv);
                        const float mix = a * vn / fnorm;
                        v = (1.f - a) * v + mix * F;
                        if (fv > 0.f) {
                            fnp += 1;
                            if (fnp > A.nmin) { dt = fminf(dt * A.finc, A.dtmax); a *= A.falpha_f; }
                        } else {
                            dt *= A.fdec; a = A.a0; fnp = 0;
                            v = make_float3(0.f, 0.f, 0.f);
                        }
                        v = v + dt * F;
                        float3 d = dt * v;
                        const float l2 = dot(d, d);
                        if (l2 > A.max_disp * A.max_disp) d = (A.max_disp * __builtin_amdgcn_rsqf(l2)) * d;
                        x = x + d;
                        fdt = dt; fal = a;
                        steps++; spt++;
                    } else {
                        live = false;
                    }
                }
            }

            if (MODE == MODE_NVE) {
                if (live && it > 0) v = v + (0.5f * A.dt * me.w) * F;
                if (A.drift != nullptr && (it % A.drift_every) == 0) {
                    const double ke = (double)khalf * ((double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z);
                    if (sub == 0) s_red64[slot] = live ? make_double2((double)e_atom, ke) : make_double2(0.0, 0.0);
                    lds_sync();                                  // C: partials visible
                    if (reducer && !s_nf[rr]) {                  // reducer lanes of replica rr
                        double ep = 0.0, kk = 0.0;
#pragma unroll 4
                        for (int j = rq; j < n; j += RL) {
                            const double2 r = s_red64[rr * n + j];
                            ep += r.x; kk += r.y;
                        }
                        if (RL == 4) { ep = quad_sum(ep); kk = quad_sum(kk); }
                        const double et = ep + kk;       // identical on the quad's lanes
                        if (rq == 0) {
                            // drift record {E(0), E(last), max |dE|, sum dE, sum step*dE, samples}
                            double *dr = s_drift + 6 * rr;
                            if (!__builtin_isfinite(et)) {
                                s_nf[rr] = 1;
                            } else if (it == 0) {
                                dr[0] = et; dr[1] = et; dr[2] = 0.0; dr[3] = 0.0; dr[4] = 0.0; dr[5] = 1.0;
                            } else {
                                const double de = et - dr[0];
                                dr[1] = et;
                                dr[2] = fmax(dr[2], fabs(de));
                                dr[3] += de; dr[4] += (double)it * de; dr[5] += 1.0;
                            }
                        }
                    }
                }
                if (live && it > 0) steps++;
            }

            if (MODE == MODE_LANGEVIN && live && it > 0) {   // closing half kick
                v = v + (0.5f * A.dt * me.w) * F;
                steps++;
            }
        }

        // ---- outputs: per-atom state, then per-replica sums (FP64) and flags
        lds_sync();       // the last reductions' LDS reads precede these writes
        if (MODE == MODE_NVE && live && s_nf[lr]) { st |= GFF_REP_NONFINITE; live = false; }
        if (sub == 0) s_red64[slot] = make_double2(WANT_E ? (double)e_atom : 0.0, (double)fl);
        lds_sync();
        if (active && sub == 0) {
            if (MODE != MODE_EVAL) {
                A.pos[g] = x.x; A.pos[g + N] = x.y; A.pos[g + 2 * N] = x.z;
                A.vel[g] = v.x; A.vel[g + N] = v.y; A.vel[g + 2 * N] = v.z;
            }
            if (MODE == MODE_EVAL) {
                if (A.F) { A.F[g] = F.x; A.F[g + N] = F.y; A.F[g + 2 * N] = F.z; }
                if (A.E_atom) A.E_atom[g] = e_grid;
            }
            if (at == 0) {
                double es = 0.0; unsigned fo = 0u;
                for (int j = 0; j < n; ++j) {
                    const double2 r = s_red64[rbase + j];
                    es += r.x;
                    fo |= (unsigned)r.y;
                }
                st |= fo;
                if (FIRE && A.f_conv > 0.f && !(st & (GFF_REP_CONVERGED | GFF_REP_NONFINITE)))
                    st |= GFF_REP_MAXSTEPS;
                if (MODE == MODE_EVAL && A.status_in && (A.status_in[rep] & GFF_REP_NONFINITE)) st |= GFF_REP_NONFINITE;
                if (st & GFF_REP_NONFINITE) { es = __builtin_nan(""); fnorm = __builtin_nanf(""); }
                if (WANT_E && A.E_rep) A.E_rep[rep] = es;
                if (A.status) A.status[rep] = st;
                if (MODE != MODE_EVAL) {
                    if (A.fnorm) A.fnorm[rep] = fnorm;
                    if (A.steps) A.steps[rep] = steps;
                }
                if (FIRE) { A.fdt[rep] = fdt; A.falpha[rep] = fal; A.fnpos[rep] = fnp; }
            }
        }
        if (MODE == MODE_NVE && A.drift && reducer && rq == 0) {
            double *d = A.drift + 6 * (size_t)A.pack_reps[pinfo.z + rr];
            const double *dr = s_drift + 6 * rr;
            for (int k = 0; k < 6; ++k) d[k] = dr[k];
        }
        lds_sync();       // LDS is reused by the next pack
    }
}

// Interpolation of independent points (no molecules).  B-spline storages: a quad of lanes
// per point, the replica kernel's gather and contraction (lane s loads the window's plane s
// of the 16 columns, one cache line per column; the quad sums the partial contractions), so
// a wave keeps 16 points' column reads in flight in 16-byte pieces.  Trilinear: a lane per
// point.  Index arithmetic never leaves the grid: x, y wrap, z below the grid is evaluated on
// the first plane, points above the last plane contribute zero, non-finite coordinates give
// NaN without a gather.
template <int STORE>
__global__ void __launch_bounds__(256) k_points(GridView g, int n, const float *pos, const float *plq,
                                                float *F, float *E) {
    unsigned fl = 0;
    if constexpr (STORE != STORE_TRI) {
        const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
        const int p = (int)(t >> 2), s = (int)(t & 3);
        if (p >= n) return;                          // whole quads: p is the same on a quad's lanes
        fetch_scales(g);
        float4 tt;
        const GridKey key = grid_key(g, pos[p], pos[p + n], pos[p + 2 * n], tt, fl);
        float m[16];
        if (key.valid) quad_fetch<STORE>(g, key, plq[p], plq[p + n], plq[p + 2 * n], s, m);
        const float4 r = quad_contract(m, tt, s, key.valid != 0);
        if (s == 0) {
            float e = r.x, fx = -r.y * g.idx, fy = -r.z * g.idy, fz = -r.w * g.idz;
            if (fl & GFF_REP_NONFINITE) e = fx = fy = fz = __builtin_nanf("");
            F[p] = fx; F[p + n] = fy; F[p + 2 * n] = fz;
            if (E) E[p] = e;
        }
    } else {
        const int p = blockIdx.x * blockDim.x + threadIdx.x;
        if (p >= n) return;
        const TriKey K = tri_key(g, pos[p], pos[p + n], pos[p + 2 * n], fl);
        float e = 0.f;
        float3 f = make_float3(0.f, 0.f, 0.f);
        if (K.state == 2) {
            e = __builtin_nanf("");
            f = make_float3(e, e, e);
        } else if (K.state == 0) {
            float4 q[8];
            tri_load(g, K, plq[p], plq[p + n], plq[p + 2 * n], q);
            e = tri_interp(g, q, K, f);
        }
        F[p] = f.x; F[p + n] = f.y; F[p + 2 * n] = f.z;
        if (E) E[p] = e;
    }
}

// ------------------------------------------------------------------ host side
static gff_status make_view(const gff_grid *gr, GridView &g) {
    if (!gr || !gr->d_coef) return GFF_EINVAL;
    if (gr->storage != GFF_STORE_F32 && gr->storage != GFF_STORE_F16 && gr->storage != STORE_TRI)
        return GFF_EUNSUPPORTED;
    if (gr->nx < 4 || gr->ny < 4 || gr->nz < 4) return GFF_EINVAL;
    if (!(gr->dx > 0.f && gr->dy > 0.f && gr->dz > 0.f)) return GFF_EINVAL;
    g.coef = gr->d_coef;
    g.x0 = gr->x0; g.y0 = gr->y0; g.z0 = gr->z0;
    g.idx = 1.f / gr->dx; g.idy = 1.f / gr->dy; g.idz = 1.f / gr->dz;
    g.dx = gr->dx; g.dy = gr->dy; g.dz = gr->dz;
    g.zmax = (float)(gr->nz - 1);
    g.nx = gr->nx; g.ny = gr->ny; g.nzp = col_nodes(gr->nz);
    if (gr->storage == STORE_TRI) {      // unpadded nodes, plain global loads (64-bit addressing)
        g.nzp = gr->nz;
        if ((double)gr->nx * gr->ny * gr->nz >= 2147483647.0) return GFF_EUNSUPPORTED;   // 32-bit cell ids
        g.bytes = 0;
        g.s0 = g.s1 = g.s2 = 1.f;
        g.scale = nullptr;
        return GFF_OK;
    }
    const double bytes = (double)gr->nx * gr->ny * g.nzp * (gr->storage == GFF_STORE_F32 ? 16 : 8);
    if (bytes >= 4294967295.0) return GFF_EUNSUPPORTED;    // 32-bit unsigned buffer offsets
    g.bytes = (unsigned)bytes;
    g.s0 = g.s1 = g.s2 = 1.f;
    g.scale = nullptr;
    if (gr->storage == GFF_STORE_F16) {
        if (!gr->d_scale) return GFF_EINVAL;
        g.scale = gr->d_scale;
    }
    return GFF_OK;
}

static void fill_common(KArgs &A, const gff_topology *topo, const gff_plan *plan) {
    A.t = topo->dev;
    A.alpha = topo->alpha;
    A.alpha_l2e = topo->alpha * 1.4426950408889634f;
    A.half_inv_alpha = 0.5f / topo->alpha;
    A.ke = topo->ke;
    A.packs = plan->d_packs; A.pack_reps = plan->d_pack_reps; A.atom_off = plan->d_atom_off;
    A.n_packs = plan->n_packs; A.N = plan->n_atoms; A.tres_max = plan->tres_max;
    A.max_pack_reps = plan->max_pack_reps; A.topo_words = plan->topo_words;
}

template <int STORE, int MODE, bool CACHE, int LPA>
static void launch_one(int grid, int BT, size_t lds, const KArgs &A, hipStream_t s) {
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)k_replicas<STORE, MODE, CACHE, LPA>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_replicas<STORE, MODE, CACHE, LPA>), dim3(grid), dim3(BT), lds, s, A);
}

// Lanes per atom of the launch: the plan's value for B-spline relaxation and dynamics, one
// for evaluations and the other storages (which then run the plan's packing one lane per atom).
static int launch_lpa(int storage, int mode, const gff_plan *plan) {
    const bool multi = mode != MODE_EVAL && (storage == GFF_STORE_F32 || storage == GFF_STORE_F16);
    return multi ? plan->lanes_per_atom : 1;
}

static size_t launch_lds(const gff_plan *plan, int lpa) {
    return replica_lds_bytes(plan->block_threads / lpa, plan->tres_max, plan->max_pack_reps, plan->topo_words);
}

template <int STORE, int MODE, bool CACHE>
static void launch_lpa_sel(int lpa, int grid, int BT, size_t lds, const KArgs &A, hipStream_t s) {
    if constexpr ((STORE == GFF_STORE_F32 || STORE == GFF_STORE_F16) && MODE != MODE_EVAL) {
        if (lpa == 4) { launch_one<STORE, MODE, CACHE, 4>(grid, BT, lds, A, s); return; }
        if (lpa == 2) { launch_one<STORE, MODE, CACHE, 2>(grid, BT, lds, A, s); return; }
    }
    launch_one<STORE, MODE, CACHE, 1>(grid, BT, lds, A, s);
}

// Relaxation and MD launches keep stencils in registers when the block fits the cached
// variant's register budget (<= 512 threads); single evaluations never reuse a stencil.
template <int MODE>
static gff_status launch_mode(int storage, const gff_plan *plan, KArgs &A, hipStream_t s) {
    const int BT = plan->block_threads;
    const int lpa = launch_lpa(storage, MODE, plan);
    const size_t lds = launch_lds(plan, lpa);
    if (lds > (size_t)plan->lds_limit) return GFF_EUNSUPPORTED;
    const int grid = plan->grid_blocks > 0 ? std::min(plan->grid_blocks, plan->n_packs) : plan->n_packs;
    if (grid <= 0) return GFF_OK;
    constexpr bool can_cache = MODE != MODE_EVAL;
    const bool cache = can_cache && BT <= 512;
    if (storage == STORE_DIRECT) {
        launch_one<STORE_DIRECT, MODE, false, 1>(grid, BT, lds, A, s);
    } else if (storage == STORE_TRI) {
        if (cache) launch_one<STORE_TRI, MODE, can_cache, 1>(grid, BT, lds, A, s);
        else launch_one<STORE_TRI, MODE, false, 1>(grid, BT, lds, A, s);
    } else if (storage == GFF_STORE_F32) {
        if (cache) launch_lpa_sel<GFF_STORE_F32, MODE, can_cache>(lpa, grid, BT, lds, A, s);
        else launch_lpa_sel<GFF_STORE_F32, MODE, false>(lpa, grid, BT, lds, A, s);
    } else {
        if (cache) launch_lpa_sel<GFF_STORE_F16, MODE, can_cache>(lpa, grid, BT, lds, A, s);
        else launch_lpa_sel<GFF_STORE_F16, MODE, false>(lpa, grid, BT, lds, A, s);
    }
    return hip_status(hipGetLastError());
}

template <int STORE, int MODE, bool CACHE, int LPA>
static gff_status occupancy_one(int BT, size_t lds, int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_replicas<STORE, MODE, CACHE, LPA>, BT, lds) ==
                   hipSuccess ? GFF_OK : GFF_EHIP;
}

template <int STORE, int MODE, bool CACHE>
static gff_status occupancy_lpa_sel(int lpa, int BT, size_t lds, int *blocks) {
    if constexpr ((STORE == GFF_STORE_F32 || STORE == GFF_STORE_F16) && MODE != MODE_EVAL) {
        if (lpa == 4) return occupancy_one<STORE, MODE, CACHE, 4>(BT, lds, blocks);
        if (lpa == 2) return occupancy_one<STORE, MODE, CACHE, 2>(BT, lds, blocks);
    }
    return occupancy_one<STORE, MODE, CACHE, 1>(BT, lds, blocks);
}

template <int MODE>
static gff_status occupancy_mode(int storage, int lpa, int BT, size_t lds, int *blocks) {
    constexpr bool can_cache = MODE != MODE_EVAL;
    const bool cache = can_cache && BT <= 512;
    if (storage == STORE_TRI)
        return cache ? occupancy_one<STORE_TRI, MODE, can_cache, 1>(BT, lds, blocks)
                     : occupancy_one<STORE_TRI, MODE, false, 1>(BT, lds, blocks);
    if (storage == GFF_STORE_F32)
        return cache ? occupancy_lpa_sel<GFF_STORE_F32, MODE, can_cache>(lpa, BT, lds, blocks)
                     : occupancy_lpa_sel<GFF_STORE_F32, MODE, false>(lpa, BT, lds, blocks);
    return cache ? occupancy_lpa_sel<GFF_STORE_F16, MODE, can_cache>(lpa, BT, lds, blocks)
                 : occupancy_lpa_sel<GFF_STORE_F16, MODE, false>(lpa, BT, lds, blocks);
}

}  // namespace gff

using namespace gff;

extern "C" gff_status gff_relax_occupancy(const gff_grid *grid, const gff_plan *plan, int mode, int *blocks_per_cu,
                                          size_t *lds_bytes_out) {
    if (!grid || !plan || !blocks_per_cu) return GFF_EINVAL;
    if (grid->storage != GFF_STORE_F32 && grid->storage != GFF_STORE_F16 && grid->storage != STORE_TRI)
        return GFF_EUNSUPPORTED;
    const int BT = plan->block_threads;
    const int kmode = mode == -1 ? MODE_EVAL : (mode == GFF_MODE_FIRE ? MODE_FIRE :
                      (mode == GFF_MODE_NVE ? MODE_NVE : (mode == GFF_MODE_LANGEVIN ? MODE_LANGEVIN : -1)));
    if (kmode < 0) return GFF_EINVAL;
    const int lpa = launch_lpa(grid->storage, kmode, plan);
    const size_t lds = launch_lds(plan, lpa);
    if (lds_bytes_out) *lds_bytes_out = lds;
    if (kmode == MODE_EVAL) return occupancy_mode<MODE_EVAL>(grid->storage, lpa, BT, lds, blocks_per_cu);
    if (kmode == MODE_FIRE) return occupancy_mode<MODE_FIRE>(grid->storage, lpa, BT, lds, blocks_per_cu);
    if (kmode == MODE_NVE) return occupancy_mode<MODE_NVE>(grid->storage, lpa, BT, lds, blocks_per_cu);
    return occupancy_mode<MODE_LANGEVIN>(grid->storage, lpa, BT, lds, blocks_per_cu);
}

static gff_status eval_common(int storage, KArgs &A, const gff_topology *topo, const gff_plan *plan,
                              int include_intra, const float *d_pos, float *d_F, float *d_E_atom, double *d_E_rep,
                              unsigned *d_status, hipStream_t s) {
    fill_common(A, topo, plan);
    A.pos = const_cast<float *>(d_pos);
    A.F = d_F; A.E_atom = d_E_atom; A.E_rep = d_E_rep; A.status = d_status;
    A.include_intra = include_intra;
    return launch_mode<MODE_EVAL>(storage, plan, A, s);
}

static gff_status relax_check(const gff_topology *topo, const gff_plan *plan, const gff_relax_params *p,
                              const gff_state *state, double *d_drift_rep) {
    if (!topo || !plan || !p || !state || !state->d_pos || !state->d_vel || !state->d_status) return GFF_EINVAL;
    if (p->n_steps < 0) return GFF_EINVAL;
    if (p->mode != GFF_MODE_FIRE && p->mode != GFF_MODE_NVE && p->mode != GFF_MODE_LANGEVIN) return GFF_EINVAL;
    if (p->mode == GFF_MODE_FIRE && (!state->d_fire_dt || !state->d_fire_alpha || !state->d_fire_npos))
        return GFF_EINVAL;
    if (p->mode == GFF_MODE_NVE && d_drift_rep && p->drift_every < 1) return GFF_EINVAL;
    if (p->check_every < 0) return GFF_EINVAL;
    if ((state->d_fixed_atom != nullptr) != (state->d_fixed_pos != nullptr)) return GFF_EINVAL;
    if (state->d_fixed_atom && p->mode != GFF_MODE_FIRE) return GFF_EUNSUPPORTED;
    if (p->mode == GFF_MODE_LANGEVIN &&
        (d_drift_rep || !(p->kT >= 0.f) || !(p->gamma >= 0.f) || !std::isfinite(p->kT) || !std::isfinite(p->gamma) ||
         !std::isfinite(p->dt)))
        return GFF_EINVAL;
    return GFF_OK;
}

static gff_status relax_common(int storage, KArgs &A, const gff_topology *topo, const gff_plan *plan,
                               const gff_relax_params *p, const gff_state *state, double *d_E_rep,
                               float *d_fnorm_rep, int *d_steps_rep, double *d_drift_rep, hipStream_t s) {
    fill_common(A, topo, plan);
    A.pos = state->d_pos; A.vel = state->d_vel;
    A.fdt = state->d_fire_dt; A.falpha = state->d_fire_alpha; A.fnpos = state->d_fire_npos;
    A.status = state->d_status;
    A.fixed_atom = state->d_fixed_atom; A.fixed_pos = state->d_fixed_pos;
    A.E_rep = d_E_rep; A.fnorm = d_fnorm_rep; A.steps = d_steps_rep;
    A.drift = p->mode == GFF_MODE_NVE ? d_drift_rep : nullptr;
    A.n_steps = p->n_steps; A.include_intra = p->include_intra;
    A.drift_every = p->drift_every < 1 ? 1 : p->drift_every;
    A.check_every = p->check_every < 1 ? 1 : p->check_every;
    A.nmin = p->fire_nmin;
    A.dt = p->dt; A.f_conv = p->f_conv; A.max_disp = p->max_disp;
    A.finc = p->fire_finc; A.fdec = p->fire_fdec; A.a0 = p->fire_alpha0; A.falpha_f = p->fire_falpha;
    A.dtmax = p->fire_dtmax;
    const double c1 = std::exp(-(double)p->gamma * (double)p->dt);
    A.lg_c1 = (float)c1; A.lg_c2 = (float)std::sqrt(std::max(0.0, 1.0 - c1 * c1)); A.kT = p->kT;
    A.seed_lo = (unsigned)(p->seed & 0xffffffffull); A.seed_hi = (unsigned)(p->seed >> 32); A.round = p->round;
    if (p->mode == GFF_MODE_FIRE) {
        if (A.path) return launch_mode<MODE_FIRE_SCAN>(storage, plan, A, s);
        const gff_status rc = A.check_every > 1 ? launch_mode<MODE_FIRE_CHECKED>(storage, plan, A, s)
                                                : launch_mode<MODE_FIRE>(storage, plan, A, s);
        if (rc != GFF_OK || !d_E_rep) return rc;
        // the energies at the final positions (the relaxation loop forms forces only)
        KArgs E = A;
        E.F = nullptr; E.E_atom = nullptr; E.status = nullptr; E.status_in = state->d_status;
        E.E_rep = d_E_rep;
        return launch_mode<MODE_EVAL>(storage, plan, E, s);
    }
    if (p->mode == GFF_MODE_LANGEVIN) return launch_mode<MODE_LANGEVIN>(storage, plan, A, s);
    return launch_mode<MODE_NVE>(storage, plan, A, s);
}

extern "C" gff_status gff_relax_scan(const gff_grid *grid, const gff_topology *topo, const gff_plan *plan,
                                     const gff_relax_params *p, const gff_state *state, const float *d_path,
                                     int n_points, int moves_per_point, float dt0, double *d_E_points,
                                     int *d_steps_points, unsigned *d_status_points, float *d_pos_points,
                                     double *d_E_rep, float *d_fnorm_rep, int *d_steps_rep, void *stream) {
    if (!p || p->mode != GFF_MODE_FIRE || !d_path || n_points < 1 || moves_per_point < 0 || !d_E_points ||
        !(dt0 > 0.f) || p->check_every > 1)
        return GFF_EINVAL;
    if ((long)n_points * ((long)moves_per_point + 1) >= 2147483647L) return GFF_EINVAL;
    if (!state || !state->d_fixed_atom) return GFF_EINVAL;       // the scanned atom
    gff_relax_params q = *p;
    q.n_steps = n_points * (moves_per_point + 1);
    gff_state t = *state;
    t.d_fixed_pos = d_path;                                     // satisfies the restraint check
    gff_status rc = relax_check(topo, plan, &q, &t, nullptr);
    if (rc != GFF_OK) return rc;
    KArgs A;
    std::memset(&A, 0, sizeof(A));
    if ((rc = make_view(grid, A.g)) != GFF_OK) return rc;
    A.path = d_path; A.n_points = n_points; A.mpp = moves_per_point; A.dt0 = dt0;
    A.E_pts = d_E_points; A.steps_pts = d_steps_points; A.st_pts = d_status_points; A.pos_pts = d_pos_points;
    return relax_common(grid->storage, A, topo, plan, &q, &t, d_E_rep, d_fnorm_rep, d_steps_rep, nullptr,
                        (hipStream_t)stream);
}

static gff_status direct_view(const gff_direct *d, const gff_topology *topo, DirectView &v) {
    if (!d || !topo) return GFF_EINVAL;
    if (d->alpha != topo->alpha) return GFF_EINVAL;           // the factors were formed with alpha
    v.xyza = d->d_xyza; v.bq = d->d_bq; v.n = d->n; v.nimg = d->nimg; v.Lx = d->Lx; v.Ly = d->Ly;
    return GFF_OK;
}

extern "C" gff_status gff_eval_forces(const gff_grid *grid, const gff_topology *topo, const gff_plan *plan,
                                      int include_intra, const float *d_pos, float *d_F, float *d_E_atom,
                                      double *d_E_rep, unsigned *d_status, void *stream) {
    if (!topo || !plan || !d_pos || !d_F) return GFF_EINVAL;
    KArgs A;
    std::memset(&A, 0, sizeof(A));
    gff_status rc = make_view(grid, A.g);
    if (rc != GFF_OK) return rc;
    return eval_common(grid->storage, A, topo, plan, include_intra, d_pos, d_F, d_E_atom, d_E_rep, d_status,
                       (hipStream_t)stream);
}

extern "C" gff_status gff_relax_batch(const gff_grid *grid, const gff_topology *topo, const gff_plan *plan,
                                      const gff_relax_params *p, const gff_state *state,
                                      double *d_E_rep, float *d_fnorm_rep, int *d_steps_rep,
                                      double *d_drift_rep, void *stream) {
    gff_status rc = relax_check(topo, plan, p, state, d_drift_rep);
    if (rc != GFF_OK) return rc;
    KArgs A;
    std::memset(&A, 0, sizeof(A));
    if ((rc = make_view(grid, A.g)) != GFF_OK) return rc;
    return relax_common(grid->storage, A, topo, plan, p, state, d_E_rep, d_fnorm_rep, d_steps_rep, d_drift_rep,
                        (hipStream_t)stream);
}

extern "C" gff_status gff_direct_create(const gff_substrate *sub, float alpha, int n_img, gff_direct **out) {
    if (!sub || !out || sub->n_atoms < 1 || !sub->pos_h || !sub->q_h || !sub->eps_h || !sub->R_h) return GFF_EINVAL;
    if (!(alpha > 0.f) || !(sub->Lx > 0.0) || !(sub->Ly > 0.0) || n_img < 0 || n_img > 64) return GFF_EINVAL;
    const int n = sub->n_atoms;
    std::vector<float4> xyza(n);
    std::vector<float2> bq(n);
    for (int j = 0; j < n; ++j) {
        const double e = sub->eps_h[j], R = sub->R_h[j];
        xyza[j] = make_float4((float)sub->pos_h[3 * j], (float)sub->pos_h[3 * j + 1], (float)sub->pos_h[3 * j + 2],
                              (float)(e * std::exp(2.0 * (double)alpha * R)));
        bq[j] = make_float2((float)(e * std::exp((double)alpha * R)), (float)sub->q_h[j]);
    }
    auto *d = new gff_direct_s();
    d->n = n; d->nimg = n_img; d->alpha = alpha; d->Lx = (float)sub->Lx; d->Ly = (float)sub->Ly;
    d->d_xyza = nullptr; d->d_bq = nullptr;
    if (hipMalloc(&d->d_xyza, n * sizeof(float4)) != hipSuccess ||
        hipMalloc(&d->d_bq, n * sizeof(float2)) != hipSuccess ||
        hipMemcpy(d->d_xyza, xyza.data(), n * sizeof(float4), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->d_bq, bq.data(), n * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) {
        if (d->d_xyza) (void)hipFree(d->d_xyza);
        if (d->d_bq) (void)hipFree(d->d_bq);
        delete d;
        return GFF_EHIP;
    }
    *out = d;
    return GFF_OK;
}

extern "C" void gff_direct_destroy(gff_direct *d) {
    if (!d) return;
    (void)hipFree(d->d_xyza);
    (void)hipFree(d->d_bq);
    delete d;
}

extern "C" gff_status gff_eval_forces_direct(const gff_direct *direct, const gff_topology *topo, const gff_plan *plan,
                                             int include_intra, const float *d_pos, float *d_F, float *d_E_atom,
                                             double *d_E_rep, unsigned *d_status, void *stream) {
    if (!topo || !plan || !d_pos || !d_F) return GFF_EINVAL;
    KArgs A;
    std::memset(&A, 0, sizeof(A));
    gff_status rc = direct_view(direct, topo, A.d);
    if (rc != GFF_OK) return rc;
    return eval_common(STORE_DIRECT, A, topo, plan, include_intra, d_pos, d_F, d_E_atom, d_E_rep, d_status,
                       (hipStream_t)stream);
}

extern "C" gff_status gff_relax_batch_direct(const gff_direct *direct, const gff_topology *topo,
                                             const gff_plan *plan, const gff_relax_params *p,
                                             const gff_state *state, double *d_E_rep, float *d_fnorm_rep,
                                             int *d_steps_rep, double *d_drift_rep, void *stream) {
    gff_status rc = relax_check(topo, plan, p, state, d_drift_rep);
    if (rc != GFF_OK) return rc;
    KArgs A;
    std::memset(&A, 0, sizeof(A));
    if ((rc = direct_view(direct, topo, A.d)) != GFF_OK) return rc;
    return relax_common(STORE_DIRECT, A, topo, plan, p, state, d_E_rep, d_fnorm_rep, d_steps_rep, d_drift_rep,
                        (hipStream_t)stream);
}

extern "C" gff_status gff_interp_points(const gff_grid *grid, int n, const float *d_pos, const float *d_plq,
                                        float *d_F, float *d_E, void *stream) {
    if (n < 0 || (n > 0 && (!d_pos || !d_plq || !d_F))) return GFF_EINVAL;
    GridView g;
    gff_status rc = make_view(grid, g);
    if (rc != GFF_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) return GFF_OK;
    const unsigned blocks = (unsigned)((n + 255L) / 256), quad_blocks = (unsigned)((4L * n + 255) / 256);
    if (grid->storage == GFF_STORE_F32)
        hipLaunchKernelGGL(k_points<GFF_STORE_F32>, dim3(quad_blocks), dim3(256), 0, s, g, n, d_pos, d_plq, d_F, d_E);
    else if (grid->storage == STORE_TRI)
        hipLaunchKernelGGL(k_points<STORE_TRI>, dim3(blocks), dim3(256), 0, s, g, n, d_pos, d_plq, d_F, d_E);
    else
        hipLaunchKernelGGL(k_points<GFF_STORE_F16>, dim3(quad_blocks), dim3(256), 0, s, g, n, d_pos, d_plq, d_F, d_E);
    return hip_status(hipGetLastError());
}
