// Grid construction for gfx950, FP64 throughout (setup path, once per substrate):
//  * Pauli/London channels by direct lattice-image sums (Eq. V_Morse) with cutoff rcut,
//    one thread per node, substrate atoms staged through LDS;
//  * Coulomb channel as the exact 2D-periodic lattice sum above a neutral slab, in its
//    Fourier form (Section "Periodicity and long-range electrostatics"): per reciprocal
//    vector G a structure factor S(G) is formed once, each z plane damps it by
//    exp(-|G| (z - z_top))/|G|, aliases are folded onto the nx x ny lateral bins, and the
//    plane is synthesised by a separable inverse DFT;
//  * exact B-spline coefficients (Section "Interpolation", fitting paragraph) by three
//    separable tridiagonal passes (cyclic in x and y, even-mirror rows in z) with the
//    constant-matrix elimination factors precomputed on the host;
//  * the storage cast into the padded, channel-interleaved, z-fastest evaluation layout.
#include "gff_internal.hpp"
#include <cmath>
#include <cstring>
#include <vector>

namespace gff {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// ------------------------------------------------------------------ Morse channels
struct MorseArgs {
    const double *sp;      // [n][6]: x, y, z, eps, R, Q
    int nsub, nx, ny, nz, KX, KY;
    double x0, y0, z0, dx, dy, dz, Lx, Ly, alpha, rcut2;
    double *V;             // [3][nx][ny][nz]
};

__global__ void __launch_bounds__(256) k_morse(MorseArgs a) {
    __shared__ double s[256 * 6];
    const long node = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)a.nx * a.ny * a.nz;
    const bool ok = node < total;
    const int k = ok ? (int)(node % a.nz) : 0;
    const long ij = ok ? node / a.nz : 0;
    const int j = (int)(ij % a.ny), i = (int)(ij / a.ny);
    const double x = a.x0 + i * a.dx, y = a.y0 + j * a.dy, z = a.z0 + k * a.dz;
    double vp = 0.0, vl = 0.0;
    for (int base = 0; base < a.nsub; base += 256) {
        const int cnt = min(256, a.nsub - base);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt * 6; q += blockDim.x) s[q] = a.sp[(size_t)base * 6 + q];
        __syncthreads();
        for (int q = 0; q < cnt; ++q) {
            const double *p = s + 6 * q;
            double ddx = x - p[0], ddy = y - p[1];
            ddx -= a.Lx * rint(ddx / a.Lx);              // minimum image, then neighbours
            ddy -= a.Ly * rint(ddy / a.Ly);
            const double ddz = z - p[2], dz2 = ddz * ddz;
            if (dz2 >= a.rcut2) continue;
            for (int ax = -a.KX; ax <= a.KX; ++ax) {
                const double ex = ddx + ax * a.Lx, ex2 = ex * ex + dz2;
                if (ex2 >= a.rcut2) continue;
                for (int by = -a.KY; by <= a.KY; ++by) {
                    const double ey = ddy + by * a.Ly;
                    const double r2 = ex2 + ey * ey;
                    if (r2 >= a.rcut2) continue;
                    const double e1 = exp(-a.alpha * (sqrt(r2) - p[4]));
                    vl += p[3] * e1;
                    vp += p[3] * e1 * e1;                // eps e^{-2 alpha (r - R)}
                }
            }
        }
    }
    if (ok) {
        a.V[node] = vp;
        a.V[total + node] = vl;
    }
}

// ------------------------------------------------------------------ Coulomb channel
struct StructArgs {
    const double *sp;        // [n][6]: x, y, z, eps, R, Q
    int nsub, MX, MY;
    double Lx, Ly, gmax, ztop, x0, y0;
    double2 *S;              // [(2MX+1)(2MY+1)], index (m+MX)*(2MY+1) + (n+MY)
};

// S'(G) = exp(i G.(x0,y0)) sum_j Q_j exp(-i G.rho_j) exp(-|G| (z_top - z_j)), zero outside gmax
__global__ void __launch_bounds__(256) k_structure(StructArgs a) {
    const int W = 2 * a.MY + 1;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (2 * a.MX + 1) * W) return;
    const int m = g / W - a.MX, n = g % W - a.MY;
    const double Gx = kTwoPi * m / a.Lx, Gy = kTwoPi * n / a.Ly, G = sqrt(Gx * Gx + Gy * Gy);
    double re = 0.0, im = 0.0;
    if ((m != 0 || n != 0) && G <= a.gmax) {
        for (int j = 0; j < a.nsub; ++j) {
            const double *p = a.sp + 6 * (size_t)j;
            const double q = p[5];
            if (q == 0.0) continue;
            const double damp = q * exp(-G * (a.ztop - p[2]));
            double sn, cs;
            sincos(Gx * (a.x0 - p[0]) + Gy * (a.y0 - p[1]), &sn, &cs);
            re += damp * cs; im += damp * sn;
        }
    }
    a.S[g] = make_double2(re, im);
}

struct BinArgs {
    const double2 *S;
    int MX, MY, nx, ny, nz;
    double Lx, Ly, gmax, ztop, z0, dz, pref;
    double2 *C;              // [nz][nx][ny]
};

// C[k][mm][nn] = pref * sum over aliases (m = mm mod nx, n = nn mod ny) of S'(G) e^{-|G| h_k}/|G|
__global__ void __launch_bounds__(256) k_bins(BinArgs a) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)a.nz * a.nx * a.ny;
    if (t >= total) return;
    const int nn = (int)(t % a.ny), mm = (int)((t / a.ny) % a.nx), k = (int)(t / ((long)a.nx * a.ny));
    const double h = a.z0 + k * a.dz - a.ztop;
    const int W = 2 * a.MY + 1;
    double re = 0.0, im = 0.0;
    // smallest alias >= -MX congruent to mm, likewise for n
    const int m0 = mm - a.nx * ((mm + a.MX) / a.nx);
    const int n0 = nn - a.ny * ((nn + a.MY) / a.ny);
    for (int m = m0; m <= a.MX; m += a.nx) {
        const double Gx = kTwoPi * m / a.Lx;
        for (int n = n0; n <= a.MY; n += a.ny) {
            if (m == 0 && n == 0) continue;
            const double Gy = kTwoPi * n / a.Ly, G = sqrt(Gx * Gx + Gy * Gy);
            if (G > a.gmax) continue;
            const double2 s = a.S[(m + a.MX) * W + (n + a.MY)];
            const double f = exp(-G * h) / G;
            re += s.x * f; im += s.y * f;
        }
    }
    a.C[t] = make_double2(a.pref * re, a.pref * im);
}

// T[k][mm][j] = sum_nn C[k][mm][nn] e^{2 pi i nn j / ny}
__global__ void __launch_bounds__(256) k_dft_y(const double2 *C, const double2 *twy, int nx, int ny, int nz, double2 *T) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nz * nx * ny) return;
    const int j = (int)(t % ny);
    const long row = t / ny;                       // (k, mm)
    const double2 *c = C + row * ny;
    double re = 0.0, im = 0.0;
    int q = 0;                                     // (nn * j) mod ny
    for (int nn = 0; nn < ny; ++nn) {
        const double2 a = c[nn], w = twy[q];
        re += a.x * w.x - a.y * w.y;
        im += a.x * w.y + a.y * w.x;
        q += j; if (q >= ny) q -= ny;
    }
    T[t] = make_double2(re, im);
}

// V[2][i][j][k] = Re sum_mm T[k][mm][j] e^{2 pi i mm i / nx} + dc[k]
__global__ void __launch_bounds__(256) k_dft_x(const double2 *T, const double2 *twx, const double *dc,
                                               int nx, int ny, int nz, double *VC) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nz * nx * ny) return;
    const int j = (int)(t % ny), i = (int)((t / ny) % nx), k = (int)(t / ((long)nx * ny));
    const double2 *c = T + (long)k * nx * ny + j;
    double re = 0.0;
    int q = 0;                                     // (mm * i) mod nx
    for (int mm = 0; mm < nx; ++mm) {
        const double2 a = c[(long)mm * ny], w = twx[q];
        re += a.x * w.x - a.y * w.y;
        q += i; if (q >= nx) q -= nx;
    }
    VC[((long)i * ny + j) * nz + k] = re + dc[k];
}

// ------------------------------------------------------------------ B-spline fit
// Constant tridiagonal system (1/6, 4/6, 1/6) factors: forward-sweep multipliers cp[i] and
// pivots inv[i] (1/pivot); for the cyclic case the Sherman-Morrison vector zsm and factor.
// scal = (vfac0, vfacN): the Sherman-Morrison scalars, on the device beside the arrays.
struct TriFactors { const double *cp, *inv, *lo, *zsm, *scal; int cyclic; };

__device__ __forceinline__ void tri_solve_strided(double *d, long stride, int n, const TriFactors &f) {
    // forward: d'[0] = d[0]*inv0; d'[i] = (d[i] - lo[i] d'[i-1]) inv[i]
    double prev = d[0] * f.inv[0];
    d[0] = prev;
    for (int i = 1; i < n; ++i) {
        const double v = (d[i * stride] - f.lo[i] * prev) * f.inv[i];
        d[i * stride] = v; prev = v;
    }
    for (int i = n - 2; i >= 0; --i) {
        const double v = d[i * stride] - f.cp[i] * prev;
        d[i * stride] = v; prev = v;
    }
    if (f.cyclic) {
        // x = y - (v.y)/(1 + v.z) z with v = (1, 0.., a/gam)
        const double vy = d[0] + f.scal[1] * d[(long)(n - 1) * stride];
        const double s = vy * f.scal[0];
        for (int i = 0; i < n; ++i) d[i * stride] -= s * f.zsm[i];
    }
}

__global__ void __launch_bounds__(256) k_fit_axis(double *B, int nlines, int inner, long stride, long outer_stride,
                                                  int n, TriFactors f) {
    // line index l -> (outer, inner); element e of the line at base + e*stride
    const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlines) return;
    const long o = l / inner, in = l % inner;
    tri_solve_strided(B + o * outer_stride + in, stride, n, f);
}

// ------------------------------------------------------------------ storage cast
__global__ void k_absmax_init(unsigned long long *m) {
    if (threadIdx.x < 3) m[threadIdx.x] = 0ull;
}

__global__ void __launch_bounds__(256) k_absmax(const double *B, long plane, unsigned long long *m) {
    __shared__ unsigned long long s[3][256];
    const int c = blockIdx.y;
    double v = 0.0;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < plane; t += (long)gridDim.x * blockDim.x)
        v = fmax(v, fabs(B[c * plane + t]));
    unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    s[c][threadIdx.x] = bits;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[c][threadIdx.x] = max(s[c][threadIdx.x], s[c][threadIdx.x + w]);
        __syncthreads();
    }
    // non-negative doubles order like their bit patterns; max is exact and order-free
    if (threadIdx.x == 0) atomicMax(m + c, s[c][0]);
}

__global__ void k_scales(const unsigned long long *m, float *scale) {
    if (threadIdx.x != 0) return;
    for (int c = 0; c < 3; ++c) {
        const double v = __longlong_as_double((long long)m[c]);
        float s = 1.f;
        if (v > 0.0) {
            int e;
            const double fr = frexp(v, &e);        // v = fr 2^e, fr in [0.5, 1)
            const int cl = (fr == 0.5) ? e - 1 : e; // ceil(log2 v)
            s = (float)ldexp(1.0, cl - 15);
        }
        scale[c] = s;
    }
    scale[3] = 0.f;
}

__global__ void k_scales_one(float *scale) {
    if (threadIdx.x < 3) scale[threadIdx.x] = 1.f;
    if (threadIdx.x == 3) scale[3] = 0.f;
}

template <int STORE>
__global__ void __launch_bounds__(256) k_pack(const double *B, int nx, int ny, int nz, const float *scale, void *out) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int cn = col_nodes(nz);
    if (t >= (long)nx * ny * cn) return;
    const int q = (int)(t % cn);
    const long ij = t / cn;
    const int p = kZStep * (q / kZBlock) + q % kZBlock;    // padded plane of this slot
    if (p > nz + 2) {                                       // past the last window: never read
        if constexpr (STORE == GFF_STORE_F32) reinterpret_cast<float4 *>(out)[t] = make_float4(0.f, 0.f, 0.f, 0.f);
        else reinterpret_cast<ushort4 *>(out)[t] = make_ushort4(0, 0, 0, 0);
        return;
    }
    int k = p - 1;
    if (k < 0) k = -k;
    if (k > nz - 1) k = 2 * (nz - 1) - k;
    const long plane = (long)nx * ny * nz, idx = ij * nz + k;
    const double b0 = B[idx], b1 = B[plane + idx], b2 = B[2 * plane + idx];
    if constexpr (STORE == GFF_STORE_F32) {
        reinterpret_cast<float4 *>(out)[t] = make_float4((float)b0, (float)b1, (float)b2, 0.f);
    } else {
        // the Pauli channel, whose mixed values dominate near the surface, also keeps the
        // rounding residual of its half (exact in FP64) as a second half in the spare slot
        const double r0 = b0 / (double)scale[0];
        const _Float16 h0 = (_Float16)r0;
        const _Float16 h1 = (_Float16)(b1 / (double)scale[1]);
        const _Float16 h2 = (_Float16)(b2 / (double)scale[2]);
        const _Float16 h3 = (_Float16)(r0 - (double)h0);
        ushort4 u;
        u.x = __builtin_bit_cast(unsigned short, h0); u.y = __builtin_bit_cast(unsigned short, h1);
        u.z = __builtin_bit_cast(unsigned short, h2); u.w = __builtin_bit_cast(unsigned short, h3);
        reinterpret_cast<ushort4 *>(out)[t] = u;
    }
}

// Nodal value and index-space gradient of the fitted model for the trilinear scheme: per
// node and channel E = sum b w_x w_y w_z and dE/du etc. over the 3x3x3 neighbourhood, with
// the cubic B-spline's node weights (1/6, 2/3, 1/6) and derivative weights (-1/2, 0, 1/2);
// x and y wrap, z rows beyond the ends mirror (node -1 -> 1, node nz -> nz-2).  FP64, stored
// FP32.
__global__ void __launch_bounds__(256) k_pack_tri(const double *B, int nx, int ny, int nz, float4 *out) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nx * ny * nz) return;
    const int k = (int)(t % nz);
    const long ij = t / nz;
    const int j = (int)(ij % ny), i = (int)(ij / ny);
    const double w[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0}, d[3] = {-0.5, 0.0, 0.5};
    const long plane = (long)nx * ny * nz;
    double acc[3][4] = {};
    for (int a = 0; a < 3; ++a) {
        const int ii = (i + a - 1 + nx) % nx;
        for (int b = 0; b < 3; ++b) {
            const int jj = (j + b - 1 + ny) % ny;
            for (int c = 0; c < 3; ++c) {
                int kk = k + c - 1;
                if (kk < 0) kk = -kk;
                if (kk > nz - 1) kk = 2 * (nz - 1) - kk;
                const long idx = ((long)ii * ny + jj) * nz + kk;
                const double we = w[a] * w[b] * w[c];
                const double gx = d[a] * w[b] * w[c], gy = w[a] * d[b] * w[c], gz = w[a] * w[b] * d[c];
                for (int ch = 0; ch < 3; ++ch) {
                    const double bb = B[ch * plane + idx];
                    acc[ch][0] += we * bb; acc[ch][1] += gx * bb; acc[ch][2] += gy * bb; acc[ch][3] += gz * bb;
                }
            }
        }
    }
    for (int ch = 0; ch < 3; ++ch)
        out[3 * t + ch] = make_float4((float)acc[ch][0], (float)acc[ch][1], (float)acc[ch][2], (float)acc[ch][3]);
}

// ------------------------------------------------------------------ host helpers
static bool spec_ok(const gff_grid_spec *s) {
    return s && s->nx >= 4 && s->ny >= 4 && s->nz >= 4 && s->dz > 0.0 &&
           (double)s->nx * s->ny * (s->nz + 3) < 2147483647.0;
}

struct CoulombPlan { int MX, MY; double gmax, ztop; size_t S_elems, C_elems; };

static CoulombPlan coulomb_plan(const gff_grid_spec *spec, const gff_substrate *sub) {
    CoulombPlan p{};
    double ztop = -1e300;
    for (int j = 0; j < sub->n_atoms; ++j) ztop = std::max(ztop, sub->pos_h[3 * j + 2]);
    p.ztop = ztop;
    const double h = std::max(spec->z0 - ztop, 0.05);
    p.gmax = 46.1 / h;                                  // exp(-|G| h) < 1e-20 beyond
    p.MX = (int)std::ceil(p.gmax * sub->Lx / kTwoPi);
    p.MY = (int)std::ceil(p.gmax * sub->Ly / kTwoPi);
    p.S_elems = (size_t)(2 * p.MX + 1) * (2 * p.MY + 1);
    p.C_elems = (size_t)spec->nz * spec->nx * spec->ny;
    return p;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace gff

using namespace gff;

extern "C" size_t gff_build_grid_workspace_bytes(const gff_grid_spec *spec, const gff_substrate *sub) {
    if (!spec_ok(spec) || !sub || sub->n_atoms < 1 || !sub->pos_h) return 0;
    CoulombPlan p = coulomb_plan(spec, sub);
    return align256((size_t)sub->n_atoms * 6 * sizeof(double)) + align256(p.S_elems * sizeof(double2)) +
           2 * align256(p.C_elems * sizeof(double2)) + align256((size_t)(spec->nx + spec->ny) * sizeof(double2)) +
           align256((size_t)spec->nz * sizeof(double));
}

extern "C" gff_status gff_build_grid(const gff_substrate *sub, const gff_grid_spec *spec, double *d_V,
                                     void *d_work, size_t work_bytes, void *stream) {
    if (!sub || !spec_ok(spec) || !d_V || sub->n_atoms < 1 || !sub->pos_h || !sub->q_h || !sub->eps_h || !sub->R_h)
        return GFF_EINVAL;
    if (!(sub->Lx > 0 && sub->Ly > 0) || !(spec->alpha > 0) || !(spec->rcut > 0)) return GFF_EINVAL;
    const size_t need = gff_build_grid_workspace_bytes(spec, sub);
    if (!d_work || work_bytes < need) return GFF_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    CoulombPlan cp = coulomb_plan(spec, sub);
    if (spec->z0 <= cp.ztop) return GFF_EINVAL;          // grid must lie above the slab
    const int n = sub->n_atoms;
    std::vector<double> sp(6 * (size_t)n);
    double qsum = 0.0, qz = 0.0;
    for (int j = 0; j < n; ++j) {
        sp[6 * j] = sub->pos_h[3 * j]; sp[6 * j + 1] = sub->pos_h[3 * j + 1]; sp[6 * j + 2] = sub->pos_h[3 * j + 2];
        sp[6 * j + 3] = sub->eps_h[j]; sp[6 * j + 4] = sub->R_h[j]; sp[6 * j + 5] = sub->q_h[j];
        qsum += sub->q_h[j]; qz += sub->q_h[j] * sub->pos_h[3 * j + 2];
    }
    const double ke = spec->k_e > 0 ? spec->k_e : kDefaultKe;
    const double dx = sub->Lx / spec->nx, dy = sub->Ly / spec->ny;
    char *w = static_cast<char *>(d_work);
    double *d_sp = reinterpret_cast<double *>(w); w += align256((size_t)n * 6 * sizeof(double));
    double2 *d_S = reinterpret_cast<double2 *>(w); w += align256(cp.S_elems * sizeof(double2));
    double2 *d_C = reinterpret_cast<double2 *>(w); w += align256(cp.C_elems * sizeof(double2));
    double2 *d_T = reinterpret_cast<double2 *>(w); w += align256(cp.C_elems * sizeof(double2));
    double2 *d_tw = reinterpret_cast<double2 *>(w); w += align256((size_t)(spec->nx + spec->ny) * sizeof(double2));
    double *d_dc = reinterpret_cast<double *>(w);
    // twiddles e^{2 pi i q / N} for both axes and the G = 0 plane constants
    std::vector<double2> tw(spec->nx + spec->ny);
    for (int q = 0; q < spec->nx; ++q) tw[q] = make_double2(std::cos(kTwoPi * q / spec->nx), std::sin(kTwoPi * q / spec->nx));
    for (int q = 0; q < spec->ny; ++q)
        tw[spec->nx + q] = make_double2(std::cos(kTwoPi * q / spec->ny), std::sin(kTwoPi * q / spec->ny));
    const double A = sub->Lx * sub->Ly, pref = kTwoPi * ke / A;
    std::vector<double> dc(spec->nz);
    for (int k = 0; k < spec->nz; ++k) dc[k] = pref * (qz - (spec->z0 + k * spec->dz) * qsum);
    // the staging copies are tiny and come from pageable host memory (setup path)
    hipError_t e = hipMemcpyAsync(d_sp, sp.data(), sp.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_dc, dc.data(), dc.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return GFF_EHIP;

    MorseArgs ma;
    ma.sp = d_sp; ma.nsub = n; ma.nx = spec->nx; ma.ny = spec->ny; ma.nz = spec->nz;
    ma.KX = (int)std::ceil(spec->rcut / sub->Lx); ma.KY = (int)std::ceil(spec->rcut / sub->Ly);
    ma.x0 = spec->x0; ma.y0 = spec->y0; ma.z0 = spec->z0; ma.dx = dx; ma.dy = dy; ma.dz = spec->dz;
    ma.Lx = sub->Lx; ma.Ly = sub->Ly; ma.alpha = spec->alpha; ma.rcut2 = spec->rcut * spec->rcut; ma.V = d_V;
    const long total = (long)spec->nx * spec->ny * spec->nz;
    hipLaunchKernelGGL(k_morse, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, ma);

    StructArgs sa;
    sa.sp = d_sp; sa.nsub = n; sa.MX = cp.MX; sa.MY = cp.MY; sa.Lx = sub->Lx; sa.Ly = sub->Ly;
    sa.gmax = cp.gmax; sa.ztop = cp.ztop; sa.x0 = spec->x0; sa.y0 = spec->y0; sa.S = d_S;
    hipLaunchKernelGGL(k_structure, dim3((unsigned)((cp.S_elems + 255) / 256)), dim3(256), 0, s, sa);

    BinArgs ba;
    ba.S = d_S; ba.MX = cp.MX; ba.MY = cp.MY; ba.nx = spec->nx; ba.ny = spec->ny; ba.nz = spec->nz;
    ba.Lx = sub->Lx; ba.Ly = sub->Ly; ba.gmax = cp.gmax; ba.ztop = cp.ztop; ba.z0 = spec->z0; ba.dz = spec->dz;
    ba.pref = pref; ba.C = d_C;
    const unsigned nb = (unsigned)((cp.C_elems + 255) / 256);
    hipLaunchKernelGGL(k_bins, dim3(nb), dim3(256), 0, s, ba);
    hipLaunchKernelGGL(k_dft_y, dim3(nb), dim3(256), 0, s, (const double2 *)d_C, (const double2 *)(d_tw + spec->nx),
                       spec->nx, spec->ny, spec->nz, d_T);
    hipLaunchKernelGGL(k_dft_x, dim3(nb), dim3(256), 0, s, (const double2 *)d_T, (const double2 *)d_tw,
                       (const double *)d_dc, spec->nx, spec->ny, spec->nz, d_V + 2 * total);
    return hip_status(hipGetLastError());
}

// ------------------------------------------------------------------ fit
namespace gff {
// Elimination factors of the constant (1/6, 4/6, 1/6) system of size n, one thread per axis
// (a short sequential recurrence).  cyclic: the Sherman-Morrison split A = T + u v^T with
// u = (gam, 0.., a), v = (1, 0.., a/gam), gam = -4/6; mirror: rows 0 and n-1 have
// off-diagonal 2/6.  Outputs: lo, cp (forward-sweep multipliers), inv (1/pivot), zsm
// (T^-1 u, cyclic only) and scal = (vfac0, vfacN).
struct AxisOut { double *lo, *cp, *inv, *zsm, *scal; int n, cyclic; };
struct FactorArgs { AxisOut ax[3]; };

__global__ void k_tri_factors(FactorArgs fa) {
    if (threadIdx.x >= 3) return;
    const AxisOut o = fa.ax[threadIdx.x];
    const int n = o.n;
    const double a = 1.0 / 6.0, b = 4.0 / 6.0, gam = -b;
    auto diag = [&](int i) {
        if (o.cyclic) return i == 0 ? b - gam : (i == n - 1 ? b - a * a / gam : b);
        return b;
    };
    auto upper = [&](int i) { return (!o.cyclic && i == 0) ? 2.0 / 6.0 : a; };
    for (int i = 0; i < n; ++i) o.lo[i] = (!o.cyclic && i == n - 1) ? 2.0 / 6.0 : a;
    double piv = diag(0);
    o.inv[0] = 1.0 / piv;
    o.cp[0] = upper(0) / piv;
    for (int i = 1; i < n; ++i) {
        piv = diag(i) - o.lo[i] * o.cp[i - 1];
        o.inv[i] = 1.0 / piv;
        o.cp[i] = upper(i) / piv;
    }
    if (o.cyclic) {
        // z = T^-1 u by the same forward and backward sweeps
        double prev = gam * o.inv[0];
        o.zsm[0] = prev;
        for (int i = 1; i < n; ++i) {
            const double u = (i == n - 1) ? a : 0.0;
            prev = (u - o.lo[i] * prev) * o.inv[i];
            o.zsm[i] = prev;
        }
        for (int i = n - 2; i >= 0; --i) o.zsm[i] -= o.cp[i] * o.zsm[i + 1];
        const double vfacN = a / gam;
        o.scal[0] = 1.0 / (1.0 + o.zsm[0] + vfacN * o.zsm[n - 1]);
        o.scal[1] = vfacN;
    } else {
        for (int i = 0; i < n; ++i) o.zsm[i] = 0.0;
        o.scal[0] = 0.0; o.scal[1] = 0.0;
    }
}
}  // namespace gff

extern "C" size_t gff_fit_workspace_bytes(const gff_grid_spec *spec) {
    if (!spec_ok(spec)) return 0;
    return 3 * (4 * align256((size_t)std::max(spec->nx, std::max(spec->ny, spec->nz)) * sizeof(double)) + 256);
}

extern "C" gff_status gff_fit_bspline(const gff_grid_spec *spec, const double *d_V, double *d_B, void *d_work,
                                      size_t work_bytes, void *stream) {
    if (!spec_ok(spec) || !d_V || !d_B || d_V == d_B) return GFF_EINVAL;
    const size_t need = gff_fit_workspace_bytes(spec);
    if (!d_work || work_bytes < need) return GFF_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const int nx = spec->nx, ny = spec->ny, nz = spec->nz;
    const long plane = (long)nx * ny * nz;
    hipError_t e = hipMemcpyAsync(d_B, d_V, 3 * plane * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return GFF_EHIP;
    const int L = std::max(nx, std::max(ny, nz));
    char *w = static_cast<char *>(d_work);
    // factors computed on the device in the workspace (x, y cyclic; z mirror rows)
    TriFactors F[3];
    FactorArgs fa;
    const int ns[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        double *arr[4];
        for (int q = 0; q < 4; ++q) { arr[q] = reinterpret_cast<double *>(w); w += align256((size_t)L * sizeof(double)); }
        double *scal = reinterpret_cast<double *>(w);
        w += 256;
        fa.ax[a] = AxisOut{arr[0], arr[1], arr[2], arr[3], scal, ns[a], a < 2 ? 1 : 0};
        F[a] = TriFactors{arr[1], arr[2], arr[0], arr[3], scal, a < 2 ? 1 : 0};
    }
    hipLaunchKernelGGL(k_tri_factors, dim3(1), dim3(64), 0, s, fa);
    for (int c = 0; c < 3; ++c) {
        double *Bc = d_B + c * plane;
        {   // along x: lines (j,k), element stride ny*nz
            const int nl = ny * nz;
            hipLaunchKernelGGL(k_fit_axis, dim3((nl + 255) / 256), dim3(256), 0, s, Bc, nl, nl, (long)ny * nz, 0L, nx, F[0]);
        }
        {   // along y: lines (i,k), element stride nz, outer stride ny*nz
            const int nl = nx * nz;
            hipLaunchKernelGGL(k_fit_axis, dim3((nl + 255) / 256), dim3(256), 0, s, Bc, nl, nz, (long)nz, (long)ny * nz, ny, F[1]);
        }
        {   // along z: lines (i,j), contiguous
            const int nl = nx * ny;
            hipLaunchKernelGGL(k_fit_axis, dim3((nl + 255) / 256), dim3(256), 0, s, Bc, nl, 1, 1L, (long)nz, nz, F[2]);
        }
    }
    return hip_status(hipGetLastError());
}

extern "C" size_t gff_grid_bytes(const gff_grid_spec *spec, int storage) {
    if (!spec_ok(spec)) return 0;
    const size_t nodes = (size_t)spec->nx * spec->ny * col_nodes(spec->nz);
    if (storage == GFF_STORE_F32) return nodes * 4 * sizeof(float);
    if (storage == GFF_STORE_F16) return nodes * 4 * sizeof(uint16_t);
    if (storage == GFF_STORE_TRILINEAR) return (size_t)spec->nx * spec->ny * spec->nz * 3 * sizeof(float4);
    return 0;
}

extern "C" gff_status gff_pack_grid(const gff_grid_spec *spec, const double *d_B, int storage, void *d_coef,
                                    float *d_scale, void *stream) {
    if (!spec_ok(spec) || !d_B || !d_coef) return GFF_EINVAL;
    if (storage != GFF_STORE_F32 && storage != GFF_STORE_F16 && storage != GFF_STORE_TRILINEAR)
        return GFF_EUNSUPPORTED;
    if (storage == GFF_STORE_F16 && !d_scale) return GFF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const long nodes = (long)spec->nx * spec->ny * col_nodes(spec->nz);
    const unsigned nb = (unsigned)((nodes + 255) / 256);
    if (storage == GFF_STORE_F32) {
        if (d_scale) hipLaunchKernelGGL(k_scales_one, dim3(1), dim3(64), 0, s, d_scale);
        hipLaunchKernelGGL(k_pack<GFF_STORE_F32>, dim3(nb), dim3(256), 0, s, d_B, spec->nx, spec->ny, spec->nz,
                           (const float *)nullptr, d_coef);
    } else if (storage == GFF_STORE_TRILINEAR) {
        if (d_scale) hipLaunchKernelGGL(k_scales_one, dim3(1), dim3(64), 0, s, d_scale);
        const long n3 = (long)spec->nx * spec->ny * spec->nz;
        hipLaunchKernelGGL(k_pack_tri, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, d_B, spec->nx, spec->ny,
                           spec->nz, static_cast<float4 *>(d_coef));
    } else {
        // the per-channel maxima are accumulated in the last 24 bytes of d_coef, which the
        // pack kernel overwrites afterwards (stream order: init, max, scales, pack)
        unsigned long long *d_max = reinterpret_cast<unsigned long long *>(
            static_cast<char *>(d_coef) + gff_grid_bytes(spec, GFF_STORE_F16) - 32);
        const long plane = (long)spec->nx * spec->ny * spec->nz;
        hipLaunchKernelGGL(k_absmax_init, dim3(1), dim3(64), 0, s, d_max);
        hipLaunchKernelGGL(k_absmax, dim3(256, 3), dim3(256), 0, s, d_B, plane, d_max);
        hipLaunchKernelGGL(k_scales, dim3(1), dim3(64), 0, s, (const unsigned long long *)d_max, d_scale);
        hipLaunchKernelGGL(k_pack<GFF_STORE_F16>, dim3(nb), dim3(256), 0, s, d_B, spec->nx, spec->ny, spec->nz,
                           (const float *)d_scale, d_coef);
    }
    return hip_status(hipGetLastError());
}
