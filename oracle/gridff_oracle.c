/*
 * FP64 CPU oracle for the GridFF hot path.  TEST INFRASTRUCTURE ONLY: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load it;
 * the HIP library never links or calls it, and the two share no code.
 *
 * Plain, slow, direct implementations of what the method computes, each written
 * from the paper's definitions (GridFF, arXiv 2508.15522):
 *   - substrate channels V^P, V^L by direct lattice-image sums
 *       (Section "Principles", Eq. V_Morse), V^C as the 2D-periodic Coulomb
 *       lattice sum (Section "Periodicity and long-range electrostatics"),
 *       evaluated by 2D Ewald summation and, above the slab, by its Fourier form;
 *   - the cubic B-spline basis and the tricubic tensor-product model as a plain
 *       64-term sum (Section "Interpolation", Eqs. Bspline1D and Bspline);
 *   - the exact B-spline coefficient fit (Section "Interpolation", fitting
 *       paragraph: the linear system the paper solves iteratively is solved
 *       exactly here);
 *   - per-atom mixing E_i = P_i V^P + L_i V^L + Q_i V^C (Eqs. E_Coulomb,
 *       E_Morse, V_Morse);
 *   - the intramolecular force field (bond, angle, torsion, Morse + Coulomb
 *       non-bonded beyond 1-3), FIRE relaxation (Bitzek et al. 2006, as used in
 *       Section "Accuracy and performance tests on CPU"), velocity-Verlet NVE;
 *   - Philox4x32-10 (Salmon et al. 2011) and uniform pose proposals.
 * Everything is double precision.  OpenMP only distributes independent replicas
 * or points; no result depends on the thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Thread count of the OpenMP loops (timing only: no result depends on it); n <= 0 restores
 * the count the process started with.  Returns the count in force before the call. */
int orc_set_threads(int n) {
    static int initial = 0;
    const int before = omp_get_max_threads();
    if (initial == 0) initial = before;
    omp_set_num_threads(n > 0 ? n : initial);
    return before;
}

/* ------------------------------------------------------------------ helpers */
static long pmod(long a, long n) { long r = a % n; return r < 0 ? r + n : r; }
static double dot3(const double *a, const double *b) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }
static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1]*b[2] - a[2]*b[1]; c[1] = a[2]*b[0] - a[0]*b[2]; c[2] = a[0]*b[1] - a[1]*b[0];
}

/* All-atom molecule-substrate energy of the comparison in Section "Configuration sampling
 * on GPU": a plain sum over every substrate atom of the cell and of its lateral periodic
 * images (a, b) with |a|, |b| <= nimg (nimg = 1: the cell and its 8 neighbours, 9 cells),
 * no cutoff and no Ewald treatment.  Per point with mixing (P, L, Q):
 *   E = sum_j sum_ab [ P eps_j e^{2 alpha R_j} e^{-2 alpha r} + L eps_j e^{alpha R_j} e^{-alpha r}
 *                      + k_e Q q_j / r ],
 * the same Pauli/London factorisation as the grids (Eq. V_Morse), and F = -grad E. */
void orc_direct_images(int nsub, const double *spos, const double *sq, const double *seps, const double *sR,
                       double Lx, double Ly, double alpha, double ke, int nimg,
                       int npts, const double *pts, const double *plq, double *E, double *F)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int p = 0; p < npts; ++p) {
        const double *r = pts + 3 * p;
        const double P = plq[3 * p], L = plq[3 * p + 1], Q = plq[3 * p + 2];
        double e = 0, f[3] = {0, 0, 0};
        for (int j = 0; j < nsub; ++j) {
            const double aP = seps[j] * exp(2.0 * alpha * sR[j]), aL = seps[j] * exp(alpha * sR[j]);
            for (int a = -nimg; a <= nimg; ++a)
                for (int b = -nimg; b <= nimg; ++b) {
                    const double d[3] = { r[0] - spos[3*j] - a * Lx, r[1] - spos[3*j+1] - b * Ly,
                                          r[2] - spos[3*j+2] };
                    const double dist = sqrt(dot3(d, d));
                    const double ep = P * aP * exp(-2.0 * alpha * dist);
                    const double el = L * aL * exp(-alpha * dist);
                    const double ec = ke * Q * sq[j] / dist;
                    e += ep + el + ec;
                    const double g = 2.0 * alpha * ep + alpha * el + ec / dist;   /* -dE/dr */
                    for (int c = 0; c < 3; ++c) f[c] += g * d[c] / dist;
                }
        }
        E[p] = e;
        for (int c = 0; c < 3; ++c) F[3 * p + c] = f[c];
    }
}

/* Scaled complementary error function erfcx(x) = exp(x^2) erfc(x).  For x < 5 from
 * the library erfc; above, from the Laplace continued fraction
 * erfc(x) = exp(-x^2)/sqrt(pi) * 1/(x + (1/2)/(x + 1/(x + (3/2)/(x + 2/(x + ...))))). */
double orc_erfcx(double x) {
    if (x < 5.0) return exp(x * x) * erfc(x);
    double f = x;                       /* evaluate the fraction bottom-up */
    for (int k = 60; k >= 1; --k) f = x + 0.5 * k / f;
    return 1.0 / (sqrt(M_PI) * f);
}
/* exp(a) * erfc(x) without overflow/underflow of the separate factors */
static double exp_erfc(double a, double x) {
    if (x < 5.0) return exp(a) * erfc(x);
    return exp(a - x * x) * orc_erfcx(x);
}

/* ============================================================ substrate channels */
/* V^P(r) = sum_j sum_n eps_j exp(-2 alpha (|r - r_j - n| - R_j)),
 * V^L(r) = sum_j sum_n eps_j exp(-alpha (|r - r_j - n| - R_j)),
 * over all lateral images n = (a Lx, b Ly) with |r - r_j - n| < rcut.
 * Gradients with respect to r.  (Eq. V_Morse) */
void orc_morse_direct(int nsub, const double *spos, const double *seps, const double *sR,
                      double Lx, double Ly, double alpha, double rcut,
                      int npts, const double *pts, double *VP, double *VL, double *gP, double *gL)
{
    int KX = (int)ceil(rcut / Lx) + 1, KY = (int)ceil(rcut / Ly) + 1;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int p = 0; p < npts; ++p) {
        const double *r = pts + 3 * p;
        double vp = 0, vl = 0, gp[3] = {0, 0, 0}, gl[3] = {0, 0, 0};
        for (int j = 0; j < nsub; ++j) {
            for (int a = -KX; a <= KX; ++a)
                for (int b = -KY; b <= KY; ++b) {
                    double d[3] = { r[0] - spos[3*j] - a * Lx, r[1] - spos[3*j+1] - b * Ly, r[2] - spos[3*j+2] };
                    double dist = sqrt(dot3(d, d));
                    if (dist >= rcut) continue;
                    double el = seps[j] * exp(-alpha * (dist - sR[j]));
                    double ep = seps[j] * exp(-2.0 * alpha * (dist - sR[j]));
                    vp += ep; vl += el;
                    for (int c = 0; c < 3; ++c) {
                        gp[c] += -2.0 * alpha * ep * d[c] / dist;
                        gl[c] += -alpha * el * d[c] / dist;
                    }
                }
        }
        VP[p] = vp; VL[p] = vl;
        if (gP) for (int c = 0; c < 3; ++c) gP[3*p+c] = gp[c];
        if (gL) for (int c = 0; c < 3; ++c) gL[3*p+c] = gl[c];
    }
}

/* 2D Ewald sum (Parry 1975; Heyes, Barber & Clarke 1977) of the Coulomb potential of
 * a charge-neutral slab periodic in x,y (rectangular cell Lx x Ly, area A):
 *   V(r) = k_e sum_j Q_j { sum_n erfc(eta d)/d
 *        + (pi/A) sum_{G!=0} cos(G.(rho-rho_j))/|G| [e^{G z} erfc(G/2eta + eta z) + e^{-G z} erfc(G/2eta - eta z)]
 *        - (2 pi/A) [ z erf(eta z) + exp(-eta^2 z^2)/(eta sqrt(pi)) ] },   z = z_r - z_j.
 * Real-space images with eta d < 6.2 and reciprocal vectors with |G|/(2 eta) < 6.2 are kept
 * (omitted terms < 1e-17 relative).  Gradient analytic. */
void orc_coulomb_ewald2d(int nsub, const double *spos, const double *sq, double Lx, double Ly,
                         double ke, double eta, int npts, const double *pts, double *V, double *g)
{
    const double A = Lx * Ly, rreal = 6.2 / eta, gmax = 2.0 * eta * 6.2;
    int KX = (int)ceil(rreal / Lx) + 1, KY = (int)ceil(rreal / Ly) + 1;
    int MX = (int)ceil(gmax * Lx / (2 * M_PI)), MY = (int)ceil(gmax * Ly / (2 * M_PI));
    #pragma omp parallel for schedule(dynamic, 4)
    for (int p = 0; p < npts; ++p) {
        const double *r = pts + 3 * p;
        double v = 0, gr[3] = {0, 0, 0};
        for (int j = 0; j < nsub; ++j) {
            double qj = sq[j];
            double rx = r[0] - spos[3*j], ry = r[1] - spos[3*j+1], z = r[2] - spos[3*j+2];
            /* real space */
            for (int a = -KX; a <= KX; ++a)
                for (int b = -KY; b <= KY; ++b) {
                    double d[3] = { rx - a * Lx, ry - b * Ly, z };
                    double dist = sqrt(dot3(d, d));
                    if (eta * dist >= 6.2) continue;
                    double f = erfc(eta * dist) / dist;
                    double df = -erfc(eta * dist) / (dist * dist)
                                - 2.0 * eta / sqrt(M_PI) * exp(-eta * eta * dist * dist) / dist;
                    v += qj * f;
                    for (int c = 0; c < 3; ++c) gr[c] += qj * df * d[c] / dist;
                }
            /* reciprocal space, G != 0 */
            for (int m = -MX; m <= MX; ++m)
                for (int n = -MY; n <= MY; ++n) {
                    if (m == 0 && n == 0) continue;
                    double Gx = 2 * M_PI * m / Lx, Gy = 2 * M_PI * n / Ly, G = sqrt(Gx*Gx + Gy*Gy);
                    if (G / (2 * eta) >= 6.2) continue;
                    double hp = exp_erfc(G * z, G / (2 * eta) + eta * z);
                    double hm = exp_erfc(-G * z, G / (2 * eta) - eta * z);
                    double ph = Gx * rx + Gy * ry, cs = cos(ph), sn = sin(ph);
                    double pref = M_PI / A / G * qj;
                    v += pref * cs * (hp + hm);
                    gr[0] += -pref * sn * Gx * (hp + hm);
                    gr[1] += -pref * sn * Gy * (hp + hm);
                    gr[2] += pref * cs * G * (hp - hm);
                }
            /* G = 0 */
            v += -2 * M_PI / A * qj * (z * erf(eta * z) + exp(-eta * eta * z * z) / (eta * sqrt(M_PI)));
            gr[2] += -2 * M_PI / A * qj * erf(eta * z);
        }
        V[p] = ke * v;
        if (g) for (int c = 0; c < 3; ++c) g[3*p+c] = ke * gr[c];
    }
}

/* Above a neutral, zero-dipole slab (z_r above every substrate atom) the same lattice sum
 * is V(r) = (2 pi k_e/A) sum_{G!=0} sum_j Q_j cos(G.(rho - rho_j)) exp(-|G|(z_r - z_j))/|G|.
 * Reciprocal vectors are kept while exp(-|G| dzmin) > 1e-20, dzmin the smallest height of a
 * point above the top atom. */
void orc_coulomb_fourier_above(int nsub, const double *spos, const double *sq, double Lx, double Ly,
                               double ke, int npts, const double *pts, double *V, double *g)
{
    const double A = Lx * Ly;
    double ztop = -1e300, zmin = 1e300;
    for (int j = 0; j < nsub; ++j) if (spos[3*j+2] > ztop) ztop = spos[3*j+2];
    for (int p = 0; p < npts; ++p) if (pts[3*p+2] < zmin) zmin = pts[3*p+2];
    double h = zmin - ztop; if (h < 0.05) h = 0.05;
    double gmax = 46.1 / h;
    int MX = (int)ceil(gmax * Lx / (2 * M_PI)), MY = (int)ceil(gmax * Ly / (2 * M_PI));
    #pragma omp parallel for schedule(dynamic, 4)
    for (int p = 0; p < npts; ++p) {
        const double *r = pts + 3 * p;
        double v = 0, gr[3] = {0, 0, 0};
        for (int m = -MX; m <= MX; ++m)
            for (int n = -MY; n <= MY; ++n) {
                if (m == 0 && n == 0) continue;
                double Gx = 2 * M_PI * m / Lx, Gy = 2 * M_PI * n / Ly, G = sqrt(Gx*Gx + Gy*Gy);
                if (G > gmax) continue;
                for (int j = 0; j < nsub; ++j) {
                    double ph = Gx * (r[0] - spos[3*j]) + Gy * (r[1] - spos[3*j+1]);
                    double e = sq[j] * exp(-G * (r[2] - spos[3*j+2])) / G;
                    v += cos(ph) * e;
                    gr[0] += -sin(ph) * Gx * e; gr[1] += -sin(ph) * Gy * e; gr[2] += -G * cos(ph) * e;
                }
            }
        double pref = 2 * M_PI * ke / A;
        V[p] = pref * v;
        if (g) for (int c = 0; c < 3; ++c) g[3*p+c] = pref * gr[c];
    }
}

/* ============================================================ cubic B-spline */
/* B(t) of Eq. Bspline and its derivative */
double orc_bspline_B(double t) {
    double a = fabs(t);
    if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
    if (a < 2.0) { double u = 2.0 - a; return u * u * u / 6.0; }
    return 0.0;
}
double orc_bspline_dB(double t) {
    double a = fabs(t), s = t < 0 ? -1.0 : 1.0;
    if (a < 1.0) return s * (-2.0 * a + 1.5 * a * a);
    if (a < 2.0) { double u = 2.0 - a; return -s * 0.5 * u * u; }
    return 0.0;
}

/* Tridiagonal solve with sub/diag/super (lo, di, up), Thomas algorithm, in place on d. */
static void thomas(int n, const double *lo, const double *di, const double *up, double *d, double *work) {
    double *c = work;
    c[0] = up[0] / di[0];
    d[0] = d[0] / di[0];
    for (int i = 1; i < n; ++i) {
        double m = di[i] - lo[i] * c[i-1];
        c[i] = up[i] / m;
        d[i] = (d[i] - lo[i] * d[i-1]) / m;
    }
    for (int i = n - 2; i >= 0; --i) d[i] -= c[i] * d[i+1];
}

/* Periodic system (b[i-1] + 4 b[i] + b[i+1]) / 6 = v[i] (indices mod n), solved with the
 * Sherman-Morrison correction of the cyclic tridiagonal matrix. */
static void solve_cyclic(int n, double *v) {
    double *lo = malloc(sizeof(double) * n), *di = malloc(sizeof(double) * n), *up = malloc(sizeof(double) * n);
    double *u = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    const double a = 1.0 / 6.0, b = 4.0 / 6.0;
    double gam = -b;                        /* A = T + u v^T, u = (gam,0..0,a), v = (1,0..0,a/gam) */
    for (int i = 0; i < n; ++i) { lo[i] = a; di[i] = b; up[i] = a; u[i] = 0; }
    di[0] = b - gam; di[n-1] = b - a * a / gam;
    u[0] = gam; u[n-1] = a;
    thomas(n, lo, di, up, v, w);
    thomas(n, lo, di, up, u, w);
    double vy = v[0] + a / gam * v[n-1], vz = u[0] + a / gam * u[n-1];
    double f = vy / (1.0 + vz);
    for (int i = 0; i < n; ++i) v[i] -= f * u[i];
    free(lo); free(di); free(up); free(u); free(w);
}

/* Even-mirror system: rows 0 and n-1 read (4 b0 + 2 b1)/6 and (2 b_{n-2} + 4 b_{n-1})/6,
 * the interior rows (b[i-1] + 4 b[i] + b[i+1])/6. */
static void solve_mirror(int n, double *v) {
    double *lo = malloc(sizeof(double) * n), *di = malloc(sizeof(double) * n), *up = malloc(sizeof(double) * n);
    double *w = malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) { lo[i] = 1.0 / 6.0; di[i] = 4.0 / 6.0; up[i] = 1.0 / 6.0; }
    up[0] = 2.0 / 6.0; lo[n-1] = 2.0 / 6.0;
    thomas(n, lo, di, up, v, w);
    free(lo); free(di); free(up); free(w);
}

/* Coefficients b of one channel, layout [nx][ny][nz] (z fastest): the B-spline model
 * reproduces V at every node, periodic in x and y, even-mirror in z.  In place on V->B. */
void orc_fit_bspline(int nx, int ny, int nz, const double *V, double *B) {
    size_t N = (size_t)nx * ny * nz;
    memcpy(B, V, N * sizeof(double));
    #pragma omp parallel
    {
        double *line = malloc(sizeof(double) * (nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz)));
        #pragma omp for
        for (long jk = 0; jk < (long)ny * nz; ++jk) {        /* along x */
            long j = jk / nz, k = jk % nz;
            for (int i = 0; i < nx; ++i) line[i] = B[((size_t)i * ny + j) * nz + k];
            solve_cyclic(nx, line);
            for (int i = 0; i < nx; ++i) B[((size_t)i * ny + j) * nz + k] = line[i];
        }
        #pragma omp for
        for (long ik = 0; ik < (long)nx * nz; ++ik) {        /* along y */
            long i = ik / nz, k = ik % nz;
            for (int j = 0; j < ny; ++j) line[j] = B[((size_t)i * ny + j) * nz + k];
            solve_cyclic(ny, line);
            for (int j = 0; j < ny; ++j) B[((size_t)i * ny + j) * nz + k] = line[j];
        }
        #pragma omp for
        for (long ij = 0; ij < (long)nx * ny; ++ij) {        /* along z */
            for (int k = 0; k < nz; ++k) line[k] = B[(size_t)ij * nz + k];
            solve_mirror(nz, line);
            for (int k = 0; k < nz; ++k) B[(size_t)ij * nz + k] = line[k];
        }
        free(line);
    }
}

/* Tricubic B-spline model of three channels B[3][nx][ny][nz] (x, y periodic, z even mirror)
 * at points r, mixed per point with (P, L, Q): E = P V^P + L V^L + Q V^C, F = -grad E.
 * Written as the plain 64-term sum over the 4x4x4 stencil (Eq. Bspline1D in each axis).
 * Domain rules: below the first z node the model is evaluated on the first z node and the
 * point is flagged (flag bit 2); strictly above the last z node the channels are zero.
 * Non-finite coordinates give NaN outputs and flag bit 4.  chanE (nullable, [n][3]) receives
 * the unmixed channel values. */
void orc_bspline_eval(int nx, int ny, int nz, double x0, double y0, double z0,
                      double dx, double dy, double dz, const double *B,
                      int n, const double *pos, const double *plq,
                      double *E, double *F, int *flag, double *chanE)
{
    size_t plane = (size_t)nx * ny * nz;
    #pragma omp parallel for schedule(static)
    for (int p = 0; p < n; ++p) {
        const double *r = pos + 3 * p;
        int fl = 0;
        double e3[3] = {0, 0, 0}, g3[3][3] = {{0,0,0},{0,0,0},{0,0,0}};
        if (!isfinite(r[0]) || !isfinite(r[1]) || !isfinite(r[2])) {
            E[p] = NAN; F[3*p] = F[3*p+1] = F[3*p+2] = NAN; flag[p] = 4;
            if (chanE) chanE[3*p] = chanE[3*p+1] = chanE[3*p+2] = NAN;
            continue;
        }
        double u = (r[0] - x0) / dx, v = (r[1] - y0) / dy, w = (r[2] - z0) / dz;
        if (w < 0) { w = 0; fl |= 2; }
        if (w <= nz - 1) {
            double fu = floor(u), fv = floor(v), fw = floor(w);
            double tu = u - fu, tv = v - fv, tw = w - fw;
            long i = pmod((long)fu, nx), j = pmod((long)fv, ny), k = (long)fw;
            for (int a = -1; a <= 2; ++a) {
                double wx = orc_bspline_B(tu - a), dwx = orc_bspline_dB(tu - a) / dx;
                long ii = pmod(i + a, nx);
                for (int b = -1; b <= 2; ++b) {
                    double wy = orc_bspline_B(tv - b), dwy = orc_bspline_dB(tv - b) / dy;
                    long jj = pmod(j + b, ny);
                    for (int c = -1; c <= 2; ++c) {
                        double wz = orc_bspline_B(tw - c), dwz = orc_bspline_dB(tw - c) / dz;
                        long kk = k + c;
                        if (kk < 0) kk = -kk;
                        if (kk > nz - 1) kk = 2 * (nz - 1) - kk;
                        size_t idx = ((size_t)ii * ny + jj) * nz + kk;
                        for (int ch = 0; ch < 3; ++ch) {
                            double bb = B[ch * plane + idx];
                            e3[ch] += wx * wy * wz * bb;
                            g3[ch][0] += dwx * wy * wz * bb;
                            g3[ch][1] += wx * dwy * wz * bb;
                            g3[ch][2] += wx * wy * dwz * bb;
                        }
                    }
                }
            }
        }
        const double *m = plq + 3 * p;
        E[p] = m[0] * e3[0] + m[1] * e3[1] + m[2] * e3[2];
        for (int c = 0; c < 3; ++c) F[3*p+c] = -(m[0] * g3[0][c] + m[1] * g3[1][c] + m[2] * g3[2][c]);
        flag[p] = fl;
        if (chanE) for (int ch = 0; ch < 3; ++ch) chanE[3*p+ch] = e3[ch];
    }
}

/* ============================================================ intramolecular force field */
typedef struct {
    int n;
    const double *eps, *R, *q;      /* [n] */
    int nb; const int *bonds; const double *bk, *br0;                 /* [nb][2] */
    int na; const int *angles; const double *ak, *acos0;              /* [na][3], vertex in the middle */
    int nt; const int *tors; const double *tV; const int *tn; const double *tphi0; /* [nt][4] */
    double alpha, ke;
} orc_mol;

/* 1 if atoms i and j are at most two bonds apart (or i == j) */
static void exclusion_matrix(const orc_mol *m, unsigned char *ex) {
    int n = m->n;
    unsigned char *adj = calloc((size_t)n * n, 1);
    for (int b = 0; b < m->nb; ++b) {
        int i = m->bonds[2*b], j = m->bonds[2*b+1];
        adj[i*n+j] = adj[j*n+i] = 1;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            int e = (i == j) || adj[i*n+j];
            for (int k = 0; k < n && !e; ++k) if (adj[i*n+k] && adj[k*n+j]) e = 1;
            ex[i*n+j] = (unsigned char)e;
        }
    free(adj);
}

/* Energy and forces of one molecule (no substrate).  Terms:
 *   bond  1/2 k (r - r0)^2
 *   angle 1/2 k (cos th - cos th0)^2
 *   torsion 1/2 V (1 - cos(n phi - phi0)), phi the IUPAC dihedral
 *   non-bonded, pairs more than two bonds apart:
 *        eps_i eps_j [exp(-2 alpha (r - R_i - R_j)) - 2 exp(-alpha (r - R_i - R_j))] + k_e Q_i Q_j / r.
 * F may be NULL.  `ex` is the n*n exclusion matrix or NULL (then computed). */
double orc_intra(const orc_mol *m, const double *x, double *F, const unsigned char *ex_in)
{
    int n = m->n;
    double E = 0;
    if (F) memset(F, 0, sizeof(double) * 3 * n);
    unsigned char *ex = (unsigned char *)ex_in;
    if (!ex) { ex = malloc((size_t)n * n); exclusion_matrix(m, ex); }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            if (ex[i*n+j]) continue;
            double d[3] = { x[3*i] - x[3*j], x[3*i+1] - x[3*j+1], x[3*i+2] - x[3*j+2] };
            double r = sqrt(dot3(d, d));
            double s = r - m->R[i] - m->R[j], ee = m->eps[i] * m->eps[j];
            double e2 = exp(-2 * m->alpha * s), e1 = exp(-m->alpha * s);
            double qq = m->ke * m->q[i] * m->q[j];
            E += ee * (e2 - 2 * e1) + qq / r;
            double dEdr = ee * (-2 * m->alpha * e2 + 2 * m->alpha * e1) - qq / (r * r);
            if (F) for (int c = 0; c < 3; ++c) { F[3*i+c] -= dEdr * d[c] / r; F[3*j+c] += dEdr * d[c] / r; }
        }
    for (int b = 0; b < m->nb; ++b) {
        int i = m->bonds[2*b], j = m->bonds[2*b+1];
        double d[3] = { x[3*i] - x[3*j], x[3*i+1] - x[3*j+1], x[3*i+2] - x[3*j+2] };
        double r = sqrt(dot3(d, d));
        E += 0.5 * m->bk[b] * (r - m->br0[b]) * (r - m->br0[b]);
        double g = m->bk[b] * (r - m->br0[b]) / r;
        if (F) for (int c = 0; c < 3; ++c) { F[3*i+c] -= g * d[c]; F[3*j+c] += g * d[c]; }
    }
    for (int t = 0; t < m->na; ++t) {
        int i = m->angles[3*t], j = m->angles[3*t+1], k = m->angles[3*t+2];
        double a[3], b[3];
        for (int c = 0; c < 3; ++c) { a[c] = x[3*i+c] - x[3*j+c]; b[c] = x[3*k+c] - x[3*j+c]; }
        double la = sqrt(dot3(a, a)), lb = sqrt(dot3(b, b));
        double cs = dot3(a, b) / (la * lb);
        double de = m->ak[t] * (cs - m->acos0[t]);
        E += 0.5 * m->ak[t] * (cs - m->acos0[t]) * (cs - m->acos0[t]);
        if (F) for (int c = 0; c < 3; ++c) {
            double gi = b[c] / (la * lb) - cs * a[c] / (la * la);
            double gk = a[c] / (la * lb) - cs * b[c] / (lb * lb);
            F[3*i+c] -= de * gi; F[3*k+c] -= de * gk; F[3*j+c] += de * (gi + gk);
        }
    }
    for (int t = 0; t < m->nt; ++t) {
        int i = m->tors[4*t], j = m->tors[4*t+1], k = m->tors[4*t+2], l = m->tors[4*t+3];
        double b1[3], b2[3], b3[3], mm[3], nn[3];
        for (int c = 0; c < 3; ++c) {
            b1[c] = x[3*j+c] - x[3*i+c]; b2[c] = x[3*k+c] - x[3*j+c]; b3[c] = x[3*l+c] - x[3*k+c];
        }
        cross3(b1, b2, mm); cross3(b2, b3, nn);
        double lb2 = sqrt(dot3(b2, b2)), m2 = dot3(mm, mm), n2 = dot3(nn, nn);
        if (m2 < 1e-20 || n2 < 1e-20) continue;   /* collinear: dihedral undefined, term dropped */
        double phi = atan2(lb2 * dot3(b1, nn), dot3(mm, nn));
        double arg = m->tn[t] * phi - m->tphi0[t];
        E += 0.5 * m->tV[t] * (1 - cos(arg));
        double dEdphi = 0.5 * m->tV[t] * m->tn[t] * sin(arg);
        if (F) {
            double gi[3], gl[3], p = dot3(b1, b2) / (lb2 * lb2), q = dot3(b3, b2) / (lb2 * lb2);
            for (int c = 0; c < 3; ++c) { gi[c] = -lb2 / m2 * mm[c]; gl[c] = lb2 / n2 * nn[c]; }
            for (int c = 0; c < 3; ++c) {
                double gj = -(1 + p) * gi[c] + q * gl[c];
                double gk = p * gi[c] - (1 + q) * gl[c];
                F[3*i+c] -= dEdphi * gi[c]; F[3*j+c] -= dEdphi * gj;
                F[3*k+c] -= dEdphi * gk;    F[3*l+c] -= dEdphi * gl[c];
            }
        }
    }
    if (!ex_in) free(ex);
    return E;
}

/* Trilinear interpolation of stored nodal energies and forces, the earlier scheme the paper
 * contrasts its B-splines with (Section "Interpolation": E, Fx, Fy, Fz stored and interpolated
 * independently, so the force is not the gradient of the energy).  N[c][i][j][k][4] holds
 * (E, Fx, Fy, Fz) of channel c at node (i, j, k).  Per point: u = (x - x0)/dx, i = floor(u)
 * mod nx, t_x = u - floor(u) (same for y); w = (z - z0)/dz, below 0 evaluated at 0 with flag
 * 2, above nz - 1 zero; k = min(floor(w), nz - 2), t_z = w - k.  Each of the 8 corners has
 * weight prod (t or 1 - t); E = sum_c m_c E_c, F = sum_c m_c F_c with (m_c) = (P, L, Q). */
void orc_trilinear_eval(int nx, int ny, int nz, double x0, double y0, double z0, double dx, double dy, double dz,
                        const double *N, int n, const double *pos, const double *plq, double *E, double *F,
                        int *flag)
{
    const size_t chan = (size_t)nx * ny * nz * 4;
    #pragma omp parallel for schedule(static)
    for (int p = 0; p < n; ++p) {
        const double *r = pos + 3 * p, *m = plq + 3 * p;
        int fl = 0;
        double acc[4] = {0, 0, 0, 0};
        if (!isfinite(r[0]) || !isfinite(r[1]) || !isfinite(r[2])) {
            E[p] = NAN; F[3*p] = F[3*p+1] = F[3*p+2] = NAN; flag[p] = 4;
            continue;
        }
        double u = (r[0] - x0) / dx, v = (r[1] - y0) / dy, w = (r[2] - z0) / dz;
        if (w < 0) { w = 0; fl |= 2; }
        if (w <= nz - 1) {
            const double fu = floor(u), fv = floor(v);
            double fw = floor(w);
            if (fw > nz - 2) fw = nz - 2;
            const double t[3] = {u - fu, v - fv, w - fw};
            const long i0 = pmod((long)fu, nx), j0 = pmod((long)fv, ny), k0 = (long)fw;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int c = 0; c < 2; ++c) {
                        const double wt = (a ? t[0] : 1 - t[0]) * (b ? t[1] : 1 - t[1]) * (c ? t[2] : 1 - t[2]);
                        const size_t node = ((size_t)pmod(i0 + a, nx) * ny + pmod(j0 + b, ny)) * nz + (k0 + c);
                        for (int ch = 0; ch < 3; ++ch)
                            for (int q = 0; q < 4; ++q) acc[q] += wt * m[ch] * N[ch * chan + 4 * node + q];
                    }
        }
        E[p] = acc[0]; F[3*p] = acc[1]; F[3*p+1] = acc[2]; F[3*p+2] = acc[3];
        flag[p] = fl;
    }
}

/* ============================================================ whole-replica force */
typedef struct {
    int nx, ny, nz; double x0, y0, z0, dx, dy, dz; const double *B;
    const double *N;          /* if not NULL: trilinear nodal table [3][nx][ny][nz][4] instead of B */
} orc_grid;

/* Total energy and force of one replica: grid model (mixing with P_i, L_i, Q_i; B-spline,
 * or the trilinear table when the grid carries one) plus the intramolecular field if `intra`.  Returns status bits (2 out of domain, 4 non-finite). */
static int replica_force(const orc_grid *g, const orc_mol *m, const double *plq, int intra,
                         const unsigned char *ex, const double *x, double *F, double *E_out,
                         double *Eatom, double *Ftmp)
{
    int n = m->n, st = 0;
    int *fl = malloc(sizeof(int) * n);
    double *Ea = Eatom ? Eatom : malloc(sizeof(double) * n);
    if (g->N)
        orc_trilinear_eval(g->nx, g->ny, g->nz, g->x0, g->y0, g->z0, g->dx, g->dy, g->dz, g->N,
                           n, x, plq, Ea, F, fl);
    else
        orc_bspline_eval(g->nx, g->ny, g->nz, g->x0, g->y0, g->z0, g->dx, g->dy, g->dz, g->B,
                         n, x, plq, Ea, F, fl, NULL);
    double E = 0;
    for (int i = 0; i < n; ++i) { E += Ea[i]; st |= fl[i]; }
    if (intra) {
        E += orc_intra(m, x, Ftmp, ex);
        for (int i = 0; i < 3 * n; ++i) F[i] += Ftmp[i];
    }
    if (!isfinite(E)) st |= 4;
    for (int i = 0; i < 3 * n; ++i) if (!isfinite(F[i])) st |= 4;
    *E_out = E;
    free(fl); if (!Eatom) free(Ea);
    return st;
}

/* Mixing coefficients of Eq. V_Morse: P = eps e^{2 alpha R}, L = -2 eps e^{alpha R}, and Q. */
void orc_mixing(int n, const double *eps, const double *R, const double *q, double alpha, double *plq) {
    for (int i = 0; i < n; ++i) {
        plq[3*i] = eps[i] * exp(2 * alpha * R[i]);
        plq[3*i+1] = -2 * eps[i] * exp(alpha * R[i]);
        plq[3*i+2] = q[i];
    }
}

typedef struct {
    int n_types;
    const int *natoms;            /* [n_types] */
    const int *atom_off;          /* [n_types+1] offsets into the per-atom arrays below */
    const double *eps, *R, *q, *mass;
    const int *bond_off, *angle_off, *tors_off;     /* [n_types+1] */
    const int *bonds; const double *bk, *br0;
    const int *angles; const double *ak, *acos0;
    const int *tors; const double *tV; const int *tn; const double *tphi0;
    double alpha, ke;
} orc_types;

static orc_mol type_mol(const orc_types *T, int t) {
    orc_mol m;
    int a0 = T->atom_off[t];
    m.n = T->natoms[t]; m.eps = T->eps + a0; m.R = T->R + a0; m.q = T->q + a0;
    m.nb = T->bond_off[t+1] - T->bond_off[t]; m.bonds = T->bonds + 2 * T->bond_off[t];
    m.bk = T->bk + T->bond_off[t]; m.br0 = T->br0 + T->bond_off[t];
    m.na = T->angle_off[t+1] - T->angle_off[t]; m.angles = T->angles + 3 * T->angle_off[t];
    m.ak = T->ak + T->angle_off[t]; m.acos0 = T->acos0 + T->angle_off[t];
    m.nt = T->tors_off[t+1] - T->tors_off[t]; m.tors = T->tors + 4 * T->tors_off[t];
    m.tV = T->tV + T->tors_off[t]; m.tn = T->tn + T->tors_off[t]; m.tphi0 = T->tphi0 + T->tors_off[t];
    m.alpha = T->alpha; m.ke = T->ke;
    return m;
}

/* Energy/force of a batch of replicas at fixed positions.  pos/F: [n_atoms_total][3];
 * atom_off[n_rep+1]; E_rep[n_rep]; E_atom[n_atoms_total] (grid part only, nullable). */
void orc_eval_batch(const orc_grid *g, const orc_types *T, int intra, int n_rep, const int *rep_type,
                    const int *atom_off, const double *pos, double *F, double *E_rep, double *E_atom,
                    int *status)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < n_rep; ++r) {
        int t = rep_type[r];
        orc_mol m = type_mol(T, t);
        int n = m.n, a0 = atom_off[r];
        double *plq = malloc(sizeof(double) * 3 * n), *Ft = malloc(sizeof(double) * 3 * n);
        unsigned char *ex = malloc((size_t)n * n);
        exclusion_matrix(&m, ex);
        orc_mixing(n, m.eps, m.R, m.q, T->alpha, plq);
        status[r] = replica_force(g, &m, plq, intra, ex, pos + 3 * a0, F + 3 * a0, E_rep + r,
                                  E_atom ? E_atom + a0 : NULL, Ft);
        free(plq); free(Ft); free(ex);
    }
}

/* ============================================================ FIRE and NVE */
typedef struct {
    int n_steps; double dt0, f_conv, max_disp, finc, fdec, alpha0, falpha, dtmax; int nmin;
    int intra;
    int check_every;            /* global decisions every k-th move (<= 1: every move) */
} orc_fire_params;

/* FIRE (Bitzek et al. 2006) for each replica, unit masses.  Each iteration: evaluate F and E
 * at x; if |F|_2 (whole 3N vector) < f_conv mark converged (bit 1) and stop; otherwise
 * P = F.v; v <- (1-a) v + a |v| F/|F|; if P > 0 { npos++; if npos > Nmin: dt <- min(dt finc,
 * dtmax), a <- a falpha } else { dt <- dt fdec, a <- a0, v <- 0, npos <- 0 }; v <- v + F dt;
 * dx = v dt, each atom's step scaled down to |dx_i| <= max_disp; x <- x + dx.  After n_steps
 * moves the state is evaluated once more (and tested).  Non-finite replicas freeze (bit 4) and
 * report NaN; replicas converged on entry are evaluated once and not moved.
 * Not converged after n_steps with f_conv > 0: bit 8.  State arrays are in/out.
 * Restraint (the manipulation scans of the paper's relaxed detachment and dragging: one atom
 * held, the rest relaxed): if fixed_atom is given and 0 <= fixed_atom[r] < n, that atom is
 * placed at fixed_pos[r] on entry, its velocity is zero and its force is replaced by zero
 * (the restraint's reaction), so it never moves and takes no part in |F|, F.v or the mixing;
 * the energy is the whole replica's.
 * Check cadence (the paper's GPU sampler downloads the state every 100 steps to test the
 * force norm and to zero the velocities when P < 0, Section "Configuration sampling on GPU"):
 * with check_every = k > 1 the steps above that need sums over the replica (convergence test,
 * P, mixing, dt/alpha adaptation, restart) are taken only on moves it = 0, k, 2k, ... and at
 * the final evaluation; every other move is a plain kick v <- v + F dt and capped move with
 * the current dt. */
void orc_fire_batch(const orc_grid *g, const orc_types *T, const orc_fire_params *prm, int n_rep,
                    const int *rep_type, const int *atom_off, double *pos, double *vel,
                    double *fdt, double *falpha, int *fnpos, int *status,
                    double *E_rep, double *fnorm_rep, int *steps_rep,
                    const int *fixed_atom, const double *fixed_pos)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < n_rep; ++r) {
        orc_mol m = type_mol(T, rep_type[r]);
        int n = m.n, a0 = atom_off[r];
        double *x = pos + 3 * a0, *v = vel + 3 * a0;
        double *plq = malloc(sizeof(double) * 3 * n), *F = malloc(sizeof(double) * 3 * n);
        double *Ft = malloc(sizeof(double) * 3 * n);
        unsigned char *ex = malloc((size_t)n * n);
        exclusion_matrix(&m, ex);
        orc_mixing(n, m.eps, m.R, m.q, T->alpha, plq);
        int st = status[r], steps = 0;
        double E = 0, fn = 0;
        if (st & 4) { E = NAN; fn = NAN; }
        const int fa = (fixed_atom && fixed_atom[r] >= 0 && fixed_atom[r] < n) ? fixed_atom[r] : -1;
        if (fa >= 0)
            for (int c = 0; c < 3; ++c) { x[3*fa+c] = fixed_pos[3*r+c]; v[3*fa+c] = 0; }
        for (int it = 0; it <= prm->n_steps && !(st & 4); ++it) {
            st |= replica_force(g, &m, plq, prm->intra, ex, x, F, &E, NULL, Ft);
            if (fa >= 0) F[3*fa] = F[3*fa+1] = F[3*fa+2] = 0;
            if (prm->check_every > 1 && it % prm->check_every != 0 && it < prm->n_steps) {
                const double dt = fdt[r];          /* no sums over the replica on this move */
                for (int i = 0; i < 3 * n; ++i) v[i] += F[i] * dt;
                for (int i = 0; i < n; ++i) {
                    double d[3] = { v[3*i] * dt, v[3*i+1] * dt, v[3*i+2] * dt };
                    double l = sqrt(dot3(d, d));
                    double s = l > prm->max_disp ? prm->max_disp / l : 1.0;
                    for (int c = 0; c < 3; ++c) x[3*i+c] += d[c] * s;
                }
                steps++;
                continue;
            }
            double ff = 0, fv = 0, vv = 0;
            for (int i = 0; i < 3 * n; ++i) { ff += F[i] * F[i]; fv += F[i] * v[i]; vv += v[i] * v[i]; }
            fn = sqrt(ff);
            if (st & 4) break;
            if (st & 1) break;                 /* converged on entry: report only */
            if (fn < prm->f_conv) { st |= 1; break; }
            if (it == prm->n_steps) break;
            double a = falpha[r], dt = fdt[r];
            double vn = sqrt(vv);
            for (int i = 0; i < 3 * n; ++i) v[i] = (1 - a) * v[i] + a * vn * F[i] / fn;
            if (fv > 0) {
                fnpos[r] += 1;
                if (fnpos[r] > prm->nmin) { dt = fmin(dt * prm->finc, prm->dtmax); a *= prm->falpha; }
            } else {
                dt *= prm->fdec; a = prm->alpha0; fnpos[r] = 0;
                for (int i = 0; i < 3 * n; ++i) v[i] = 0;
            }
            for (int i = 0; i < 3 * n; ++i) v[i] += F[i] * dt;
            for (int i = 0; i < n; ++i) {
                double d[3] = { v[3*i] * dt, v[3*i+1] * dt, v[3*i+2] * dt };
                double l = sqrt(dot3(d, d));
                double s = l > prm->max_disp ? prm->max_disp / l : 1.0;
                for (int c = 0; c < 3; ++c) x[3*i+c] += d[c] * s;
            }
            fdt[r] = dt; falpha[r] = a;
            steps++;
        }
        if (prm->f_conv > 0 && !(st & 1) && !(st & 4)) st |= 8;
        status[r] = st; E_rep[r] = E; fnorm_rep[r] = fn; steps_rep[r] = steps;
        free(plq); free(F); free(Ft); free(ex);
    }
}

/* Velocity-Verlet NVE with masses in amu, velocities in A/fs, dt in fs:
 * a = F / (m * 103.6426965...) [A/fs^2]  (1 amu A^2 fs^-2 = 103.6427 eV).
 * F at the start positions is evaluated first; every step: v += a dt/2; x += v dt; F(x);
 * v += a dt/2.  Total energy E_pot + sum m v^2/2 is sampled at steps s = 0, k, 2k, ... and
 * accumulated in drift[6] = {E(0), E(last sample), max|E(s)-E(0)|, sum dE, sum s dE, samples}.
 * Non-finite replicas freeze (bit 4). */
void orc_nve_batch(const orc_grid *g, const orc_types *T, int n_steps, double dt, int intra,
                   int drift_every, int n_rep, const int *rep_type, const int *atom_off,
                   double *pos, double *vel, int *status, double *E_rep, double *drift)
{
    const double conv = 103.6426965268;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < n_rep; ++r) {
        int t = rep_type[r];
        orc_mol m = type_mol(T, t);
        int n = m.n, a0 = atom_off[r];
        const double *mass = T->mass + T->atom_off[t];
        double *x = pos + 3 * a0, *v = vel + 3 * a0;
        double *plq = malloc(sizeof(double) * 3 * n), *F = malloc(sizeof(double) * 3 * n);
        double *Ft = malloc(sizeof(double) * 3 * n);
        unsigned char *ex = malloc((size_t)n * n);
        exclusion_matrix(&m, ex);
        orc_mixing(n, m.eps, m.R, m.q, T->alpha, plq);
        int st = status[r];
        double E = 0, *dr = drift ? drift + 6 * r : NULL;
        if (!(st & 4)) st |= replica_force(g, &m, plq, intra, ex, x, F, &E, NULL, Ft);
        for (int s = 0; s <= n_steps && !(st & 4); ++s) {
            if (s > 0) {
                for (int i = 0; i < n; ++i) for (int c = 0; c < 3; ++c) {
                    v[3*i+c] += 0.5 * dt * F[3*i+c] / (mass[i] * conv);
                    x[3*i+c] += dt * v[3*i+c];
                }
                st |= replica_force(g, &m, plq, intra, ex, x, F, &E, NULL, Ft);
                if (st & 4) break;
                for (int i = 0; i < n; ++i) for (int c = 0; c < 3; ++c)
                    v[3*i+c] += 0.5 * dt * F[3*i+c] / (mass[i] * conv);
            }
            if (dr && s % drift_every == 0) {
                double ke = 0;
                for (int i = 0; i < n; ++i) ke += 0.5 * mass[i] * conv * dot3(v + 3 * i, v + 3 * i);
                double et = E + ke;
                if (s == 0) { dr[0] = et; dr[2] = 0; dr[3] = 0; dr[4] = 0; dr[5] = 0; }
                double de = et - dr[0];
                dr[1] = et;
                if (fabs(de) > dr[2]) dr[2] = fabs(de);
                dr[3] += de; dr[4] += s * de; dr[5] += 1;
            }
        }
        status[r] = st; E_rep[r] = E;
        free(plq); free(F); free(Ft); free(ex);
    }
}

/* ============================================================ Philox4x32-10 and proposals */
/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11): per round
 * (hi0,lo0) = M0*c0, (hi1,lo1) = M1*c2, c <- (hi1^c1^k0, lo1, hi0^c3^k1, lo0); the key is
 * bumped by the Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0, hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0; c1 = lo1; c2 = hi0 ^ c3 ^ k1; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Langevin dynamics, the thermal perturbation of the paper's minima hopping (Section
 * "Configuration sampling on GPU": 1000 steps at 300 K before each relaxation), integrated
 * by the BAOAB splitting (Leimkuhler & Matthews 2013); the paper names no scheme.  Per step
 *   v += dt/2 F/m;  x += dt/2 v;  v = c1 v + c2 sqrt(kT/m) xi;  x += dt/2 v;  F = F(x);
 *   v += dt/2 F/m,   c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2),
 * masses in amu (m -> m * 103.6427 eV fs^2/A^2).  The normals xi of replica id r, atom a,
 * step s (1-based) come from Philox4x32-10 with counter (r, a, s, round) and key (seed low,
 * seed high): with u_k = ((x_k >> 9) + 1/2) 2^-23 (exact in single precision, never 0 or 1),
 * xi_x = sqrt(-2 ln u0) cos(2 pi u1),
 * xi_y = sqrt(-2 ln u0) sin(2 pi u1), xi_z = sqrt(-2 ln u2) cos(2 pi u3).  A replica whose
 * energy becomes non-finite is frozen with status bit 4. */
void orc_langevin_batch(const orc_grid *g, const orc_types *T, int n_steps, double dt, double kT, double gamma,
                        uint64_t seed, uint32_t round, int intra, int n_rep, const int *rep_type, const int *rep_id,
                        const int *atom_off, double *pos, double *vel, int *status, double *E_rep)
{
    const double conv = 103.6426965268;
    const double c1 = exp(-gamma * dt), c2 = sqrt(1.0 - c1 * c1);
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    #pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < n_rep; ++r) {
        int t = rep_type[r];
        orc_mol m = type_mol(T, t);
        int n = m.n, a0 = atom_off[r];
        const double *mass = T->mass + T->atom_off[t];
        double *x = pos + 3 * a0, *v = vel + 3 * a0;
        double *plq = malloc(sizeof(double) * 3 * n), *F = malloc(sizeof(double) * 3 * n);
        double *Ft = malloc(sizeof(double) * 3 * n);
        unsigned char *ex = malloc((size_t)n * n);
        exclusion_matrix(&m, ex);
        orc_mixing(n, m.eps, m.R, m.q, T->alpha, plq);
        int st = status[r];
        double E = 0;
        if (!(st & 4)) st |= replica_force(g, &m, plq, intra, ex, x, F, &E, NULL, Ft);
        for (int s = 1; s <= n_steps && !(st & 4); ++s) {
            for (int i = 0; i < n; ++i) {
                const double mi = mass[i] * conv, sig = sqrt(kT / mi);
                const uint32_t ctr[4] = {(uint32_t)rep_id[r], (uint32_t)i, (uint32_t)s, round};
                uint32_t o[4];
                orc_philox4x32_10(ctr, key, o);
                double u[4];
                for (int k = 0; k < 4; ++k) u[k] = ((double)(o[k] >> 9) + 0.5) / 8388608.0;
                const double r0 = sqrt(-2.0 * log(u[0])), r2 = sqrt(-2.0 * log(u[2]));
                const double xi[3] = {r0 * cos(2.0 * M_PI * u[1]), r0 * sin(2.0 * M_PI * u[1]),
                                      r2 * cos(2.0 * M_PI * u[3])};
                for (int c = 0; c < 3; ++c) {
                    v[3*i+c] += 0.5 * dt * F[3*i+c] / mi;
                    x[3*i+c] += 0.5 * dt * v[3*i+c];
                    v[3*i+c] = c1 * v[3*i+c] + c2 * sig * xi[c];
                    x[3*i+c] += 0.5 * dt * v[3*i+c];
                }
            }
            st |= replica_force(g, &m, plq, intra, ex, x, F, &E, NULL, Ft);
            if (st & 4) break;
            for (int i = 0; i < n; ++i) for (int c = 0; c < 3; ++c)
                v[3*i+c] += 0.5 * dt * F[3*i+c] / (mass[i] * conv);
        }
        status[r] = st; E_rep[r] = E;
        free(plq); free(F); free(Ft); free(ex);
    }
}

/* uniform in [0,1) from the top 24 bits */
static double u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* Uniform proposal DOF for replica r: counter (r, block, round, 0), key (seed lo, hi).
 * Block 0 gives (u, v, h, s1), block 1 (s2, s3, t0, t1), block b >= 2 torsions
 * t_{2b-2..}.  Output per replica: [u, v, h, qw, qx, qy, qz, phi_0..phi_{T-1}]:
 *   lateral fractions u, v in [0,1), height h = hlo + (hhi-hlo) U,
 *   unit quaternion by Shoemake's method from (s1, s2, s3),
 *   torsions phi_k = 2 pi U. */
void orc_propose_uniform(int n_rep, int T, uint64_t seed, uint32_t round, double hlo, double hhi,
                         double *dof /* [n_rep][7+T] */)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (int r = 0; r < n_rep; ++r) {
        int nb = 2 + (T > 2 ? (T - 2 + 3) / 4 : 0);
        double u[64];
        for (int b = 0; b < nb; ++b) {
            uint32_t ctr[4] = { (uint32_t)r, (uint32_t)b, round, 0u }, o[4];
            orc_philox4x32_10(ctr, key, o);
            for (int k = 0; k < 4; ++k) u[4*b+k] = u01(o[k]);
        }
        double *d = dof + (size_t)r * (7 + T);
        d[0] = u[0]; d[1] = u[1]; d[2] = hlo + (hhi - hlo) * u[2];
        double s1 = u[3], s2 = u[4], s3 = u[5];
        double a = sqrt(1 - s1), b = sqrt(s1);
        d[3] = b * cos(2 * M_PI * s3);        /* w */
        d[4] = a * sin(2 * M_PI * s2);        /* x */
        d[5] = a * cos(2 * M_PI * s2);        /* y */
        d[6] = b * sin(2 * M_PI * s3);        /* z */
        for (int k = 0; k < T; ++k) d[7 + k] = 2 * M_PI * u[6 + k];
    }
}

/* IUPAC dihedral of four points */
static double dihedral(const double *pi, const double *pj, const double *pk, const double *pl) {
    double b1[3], b2[3], b3[3], mm[3], nn[3];
    for (int c = 0; c < 3; ++c) { b1[c] = pj[c] - pi[c]; b2[c] = pk[c] - pj[c]; b3[c] = pl[c] - pk[c]; }
    cross3(b1, b2, mm); cross3(b2, b3, nn);
    return atan2(sqrt(dot3(b2, b2)) * dot3(b1, nn), dot3(mm, nn));
}
double orc_dihedral(const double *p4) { return dihedral(p4, p4 + 3, p4 + 6, p4 + 9); }

/* rotate point p about the axis through o with unit direction k by angle t (Rodrigues) */
static void rot_axis(double *p, const double *o, const double *k, double t) {
    double v[3] = { p[0] - o[0], p[1] - o[1], p[2] - o[2] }, kv[3];
    cross3(k, v, kv);
    double kd = dot3(k, v), c = cos(t), s = sin(t);
    for (int i = 0; i < 3; ++i) p[i] = o[i] + v[i] * c + kv[i] * s + k[i] * kd * (1 - c);
}

/* Pose from DOF (layout of orc_propose_uniform) for a molecule with reference geometry
 * ref[n][3] and T rotatable torsions (quad[T][4], mask[T][n]):
 *   1. set each torsion in order: rotate the masked atoms about the j->k axis so that the
 *      dihedral of quad becomes phi_k;
 *   2. rotate about the centroid by the unit quaternion (w,x,y,z);
 *   3. translate: centroid to (u Lx, v Ly) laterally, lowest atom to z_top + h. */
void orc_pose(int n, const double *ref, int T, const int *quad, const unsigned char *mask,
              const double *d, double Lx, double Ly, double z_top, double *out)
{
    memcpy(out, ref, sizeof(double) * 3 * n);
    for (int k = 0; k < T; ++k) {
        const int *q = quad + 4 * k;
        double cur = dihedral(out + 3*q[0], out + 3*q[1], out + 3*q[2], out + 3*q[3]);
        double ax[3] = { out[3*q[2]] - out[3*q[1]], out[3*q[2]+1] - out[3*q[1]+1], out[3*q[2]+2] - out[3*q[1]+2] };
        double l = sqrt(dot3(ax, ax));
        for (int c = 0; c < 3; ++c) ax[c] /= l;
        double o[3] = { out[3*q[1]], out[3*q[1]+1], out[3*q[1]+2] };
        double t = d[7 + k] - cur;
        for (int i = 0; i < n; ++i) if (mask[k * n + i]) rot_axis(out + 3 * i, o, ax, t);
    }
    double cen[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) for (int c = 0; c < 3; ++c) cen[c] += out[3*i+c] / n;
    double w = d[3], x = d[4], y = d[5], z = d[6];
    double Rm[9] = { 1 - 2*(y*y + z*z), 2*(x*y - z*w),     2*(x*z + y*w),
                     2*(x*y + z*w),     1 - 2*(x*x + z*z), 2*(y*z - x*w),
                     2*(x*z - y*w),     2*(y*z + x*w),     1 - 2*(x*x + y*y) };
    double zmin = 1e300;
    for (int i = 0; i < n; ++i) {
        double p[3] = { out[3*i] - cen[0], out[3*i+1] - cen[1], out[3*i+2] - cen[2] };
        for (int c = 0; c < 3; ++c) out[3*i+c] = Rm[3*c] * p[0] + Rm[3*c+1] * p[1] + Rm[3*c+2] * p[2];
        if (out[3*i+2] < zmin) zmin = out[3*i+2];
    }
    for (int i = 0; i < n; ++i) {
        out[3*i] += d[0] * Lx; out[3*i+1] += d[1] * Ly; out[3*i+2] += z_top + d[2] - zmin;
    }
}
