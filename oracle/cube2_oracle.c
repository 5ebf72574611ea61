/*
 * cube2_oracle.c -- plain FP64 CPU reference of the CUBE2 force computation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP path and is deliberately slow and literal: every loop follows
 * one definition of the paper, with no blocking, fusion or reordering.
 *
 * Conventions (readings of the paper, section 2.1):
 *  - lengths in fine mesh cells; a level with spacing H (in fine cells) works
 *    in its own grid units y = x / H and has n = n_fine / H nodes per side;
 *  - node n sits at position n (0-based, periodic mod n); cell i = [i, i+1);
 *  - meshes are stored [z][y][x] with x fastest;
 *  - particle arrays are SoA: x[d*N + i], d = 0 (x), 1 (y), 2 (z);
 *  - coupling constants G*m are left to the caller (the paper drops them).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ */
/* Softening profile and reference force, section 2.1.1               */
/* ------------------------------------------------------------------ */

/* eq. (1): density profile of a softened particle, unit mass. */
double orc_profile(double r, double b)
{
    if (r < b / 2) return 48.0 * (b / 2 - r) / (M_PI * pow(b, 4));
    return 0.0;
}

/* eq. (2): force magnitude between two eq.(1) profiles at distance r.
 * The pair law of eq. (4d) subtracts two of these, which cancel as r
 * approaches b_f (both tend to 1/r^2), so they are evaluated in x87 extended
 * precision (64-bit significand) and the difference is rounded once. */
typedef long double xreal;

static xreal refforce_x(xreal r, xreal b)
{
    if (r >= b) return 1.0L / (r * r);
    xreal b2 = b * b, b3 = b2 * b, b4 = b3 * b, b5 = b4 * b, b6 = b5 * b,
          b7 = b6 * b, b8 = b7 * b;
    xreal r2 = r * r, r3 = r2 * r, r4 = r3 * r, r5 = r4 * r, r6 = r5 * r;
    if (r < b / 2)
        return 64.0L * r / (5.0L * b3) - 256.0L * r3 / (5.0L * b5) + 32.0L * r4 / b6
             + 1536.0L * r5 / (35.0L * b7) - 192.0L * r6 / (5.0L * b8);
    return 3.0L / (35.0L * r2) - 32.0L / (5.0L * b2) + 256.0L * r / (5.0L * b3)
         - 96.0L * r2 / b4 + 256.0L * r3 / (5.0L * b5) + 32.0L * r4 / b6
         - 1536.0L * r5 / (35.0L * b7) + 64.0L * r6 / (5.0L * b8);
}

/* d/dr of eq. (2), term by term. */
static xreal refforce_dr_x(xreal r, xreal b)
{
    if (r >= b) return -2.0L / (r * r * r);
    xreal b2 = b * b, b3 = b2 * b, b4 = b3 * b, b5 = b4 * b, b6 = b5 * b,
          b7 = b6 * b, b8 = b7 * b;
    xreal r2 = r * r, r3 = r2 * r, r4 = r3 * r, r5 = r4 * r;
    if (r < b / 2)
        return 64.0L / (5.0L * b3) - 768.0L * r2 / (5.0L * b5) + 128.0L * r3 / b6
             + 1536.0L * r4 / (7.0L * b7) - 1152.0L * r5 / (5.0L * b8);
    return -6.0L / (35.0L * r3) + 256.0L / (5.0L * b3) - 192.0L * r / b4
         + 768.0L * r2 / (5.0L * b5) + 128.0L * r3 / b6 - 1536.0L * r4 / (7.0L * b7)
         + 384.0L * r5 / (5.0L * b8);
}

double orc_refforce(double r, double b) { return (double)refforce_x(r, b); }

/* R(r_i, b) for an array of separations (the same evaluation as orc_refforce). */
void orc_refforce_many(int64_t N, const double *r, double b, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) out[i] = (double)refforce_x(r[i], b);
}
double orc_refforce_dr(double r, double b) { return (double)refforce_dr_x(r, b); }

/* eq. (13): Fourier transform of eq.(1).  b <= 0 stands for b = infinity,
 * where S vanishes (b_0 = infinity, so the coarsest level is untruncated).
 * For small u = kb/2 the closed form cancels; its Taylor series is used. */
double orc_profile_k(double k, double b)
{
    if (!(b > 0.0) || isinf(b)) return 0.0;
    double u = 0.5 * k * b;
    if (u < 1.0) {
        double u2 = u * u;
        return 1.0 - u2 / 15.0 + u2 * u2 / 560.0 - u2 * u2 * u2 / 37800.0
             + u2 * u2 * u2 * u2 / 3991680.0
             - u2 * u2 * u2 * u2 * u2 / 605404800.0
             + u2 * u2 * u2 * u2 * u2 * u2 / 124540416000.0
             - u2 * u2 * u2 * u2 * u2 * u2 * u2 / 33345696384000.0;
    }
    return 12.0 / pow(u, 4) * (2.0 - 2.0 * cos(u) - u * sin(u));
}

/* ------------------------------------------------------------------ */
/* Optimized Green's function, eqs. (9)-(13)                           */
/* ------------------------------------------------------------------ */

static double sinc(double x)
{
    if (fabs(x) < 1e-4) return 1.0 - x * x / 6.0 + x * x * x * x / 120.0;
    return sin(x) / x;
}

/* sin(2 pi m / n), exactly zero where it vanishes mathematically. */
static double sin_frac(long m, long n)
{
    long mm = ((m % n) + n) % n;
    if ((2 * mm) % n == 0) return 0.0;
    return sin(2.0 * M_PI * (double)mm / (double)n);
}

/*
 * G_alpha at the mesh wave number k = 2 pi (m1, m2, m3) / n (level grid
 * units), eq. (11):
 *     G = D(k) . sum_n W^2(k_n) R*(k_n) / ( |D(k)|^2 [sum_n W^2(k_n)]^2 )
 * with k_n = k + 2 pi n, |n_d| <= nmax, the assignment window
 * W(k) = prod_d sinc(k_d/2)^p (p = 2 for CIC, p = 3 for TSC, eq. (9)),
 * the finite-difference operator D_d(k) = i (4/3 sin k_d - 1/6 sin 2k_d)
 * (eq. (10), one component per axis), and the target force of the level,
 * eq. (12) with the Newtonian 4 pi restored:
 *     R(k) = -4 pi i k [S^2(|k|, b_a) - S^2(|k|, b_prev)] / |k|^2.
 * Where |D|^2 = 0 (every k_d in {0, pi}), G = 0.  With iso_L > 0 the target
 * force is the one truncated at r = iso_L (appendix A): R(k) is multiplied
 * by 1 - sinc(|k| iso_L), for a mesh of twice that length (isolated
 * boundaries).
 */
double orc_green_point(int n, int m1, int m2, int m3, double b_a, double b_prev,
                       int nmax, int p, double iso_L)
{
    int m[3] = {m1, m2, m3};
    double k[3], d[3], dd = 0.0;
    for (int a = 0; a < 3; ++a) {
        k[a] = 2.0 * M_PI * (double)m[a] / (double)n;
        d[a] = 4.0 / 3.0 * sin_frac(m[a], n) - 1.0 / 6.0 * sin_frac(2L * m[a], n);
        dd += d[a] * d[a];
    }
    if (dd == 0.0) return 0.0;
    double U = 0.0, V = 0.0;
    for (int n1 = -nmax; n1 <= nmax; ++n1)
        for (int n2 = -nmax; n2 <= nmax; ++n2)
            for (int n3 = -nmax; n3 <= nmax; ++n3) {
                double kn[3] = {k[0] + 2.0 * M_PI * n1, k[1] + 2.0 * M_PI * n2,
                                k[2] + 2.0 * M_PI * n3};
                double W = 1.0;
                for (int a = 0; a < 3; ++a) W *= pow(sinc(0.5 * kn[a]), p);
                double W2 = W * W;
                U += W2;
                double kk = kn[0] * kn[0] + kn[1] * kn[1] + kn[2] * kn[2];
                if (kk == 0.0) continue;
                double kmag = sqrt(kk);
                double sa = orc_profile_k(kmag, b_a), sp = orc_profile_k(kmag, b_prev);
                double dS2 = sa * sa - sp * sp;
                /* isolated boundaries (appendix A, eq. A2): the target force
                 * truncated at r = L has the transform [1 - sinc(k L)] R(k) */
                if (iso_L > 0.0) dS2 *= 1.0 - sinc(kmag * iso_L);
                /* D . R* with D = i d and R* = +4 pi i k_n dS2 / k_n^2 */
                double dk = d[0] * kn[0] + d[1] * kn[1] + d[2] * kn[2];
                V += W2 * dk * dS2 / kk;
            }
    return -4.0 * M_PI * V / (dd * U * U);
}

/* Octant table G[m3][m2][m1], m_d in [0, n/2]. */
void orc_green_table(int n, double b_a, double b_prev, int nmax, int p, double iso_L,
                     double *out)
{
    int h = n / 2 + 1;
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int m3 = 0; m3 < h; ++m3)
        for (int m2 = 0; m2 < h; ++m2)
            for (int m1 = 0; m1 < h; ++m1)
                out[((size_t)m3 * h + m2) * h + m1] =
                    orc_green_point(n, m1, m2, m3, b_a, b_prev, nmax, p, iso_L);
}

/* Sum over aliases of W^2 in one dimension (used by the identity checks). */
double orc_alias_w2_1d(double k, int nmax, int p)
{
    double s = 0.0;
    for (int a = -nmax; a <= nmax; ++a) s += pow(sinc(0.5 * (k + 2.0 * M_PI * a)), 2 * p);
    return s;
}

/* ------------------------------------------------------------------ */
/* CIC assignment and interpolation (section 2.1.2 with the CIC kernel) */
/* ------------------------------------------------------------------ */

static inline long wrapi(long i, long n) { i %= n; return i < 0 ? i + n : i; }
static inline size_t midx(long x, long y, long z, long n)
{
    return ((size_t)wrapi(z, n) * n + wrapi(y, n)) * n + wrapi(x, n);
}

/* Cell index j and fractional offset f of coordinate x (fine cells) on a
 * level of spacing H.  With quant != 0 the fraction is truncated to 15 bits,
 * the fixed-point reading used by the integer deposit. */
static inline void cic_coord(double x, double H, int quant, long *j, double *f)
{
    double y = x / H;
    double fl = floor(y);
    double fr = y - fl;
    if (quant) fr = floor(fr * 32768.0) / 32768.0;
    *j = (long)fl;
    *f = fr;
}

/* Exact integer CIC deposit: acc[(j+s) mod n] += prod_d w_d(s_d) with
 * w(0) = 2^15 - f, w(1) = f and f the 15-bit in-cell fraction.  The density
 * in particle masses per level cell is acc * 2^-45. */
void orc_deposit_fx(int64_t N, const double *x, int n, double H, uint64_t *acc)
{
    for (int64_t i = 0; i < N; ++i) {
        long j[3];
        uint64_t w[3][2];
        for (int d = 0; d < 3; ++d) {
            double f;
            cic_coord(x[d * N + i], H, 1, &j[d], &f);
            uint64_t fi = (uint64_t)(f * 32768.0);
            w[d][0] = 32768u - fi;
            w[d][1] = fi;
        }
        for (int sz = 0; sz < 2; ++sz)
            for (int sy = 0; sy < 2; ++sy)
                for (int sx = 0; sx < 2; ++sx)
                    acc[midx(j[0] + sx, j[1] + sy, j[2] + sz, n)] +=
                        w[0][sx] * w[1][sy] * w[2][sz];
    }
}

/* Floating-point CIC deposit, unit mass per particle. */
void orc_deposit(int64_t N, const double *x, int n, double H, int quant, double *rho)
{
    for (int64_t i = 0; i < N; ++i) {
        long j[3];
        double w[3][2];
        for (int d = 0; d < 3; ++d) {
            double f;
            cic_coord(x[d * N + i], H, quant, &j[d], &f);
            w[d][0] = 1.0 - f;
            w[d][1] = f;
        }
        for (int sz = 0; sz < 2; ++sz)
            for (int sy = 0; sy < 2; ++sy)
                for (int sx = 0; sx < 2; ++sx)
                    rho[midx(j[0] + sx, j[1] + sy, j[2] + sz, n)] +=
                        w[0][sx] * w[1][sy] * w[2][sz];
    }
}

/* ------------------------------------------------------------------ */
/* TSC assignment and interpolation (eq. 5)                            */
/* ------------------------------------------------------------------ */

/* eq. (5): W(x) = 3/4 - x^2 for |x| <= 1/2, (3/2 - |x|)^2 / 2 for
 * 1/2 <= |x| <= 3/2, 0 beyond, x the distance to a node in level cells.
 * A particle at y (level units) has nearest node n0 = floor(y + 1/2) and
 * d = y - n0 in [-1/2, 1/2); nodes n0-1, n0, n0+1 get (1/2 - d)^2/2,
 * 3/4 - d^2, (1/2 + d)^2/2.  With quant != 0 the in-cell fraction of y is
 * first truncated to 15 bits (as for CIC), so d = m 2^-15 with integer m in
 * [-2^14, 2^14). */
static inline void tsc_coord(double x, double H, int quant, long *n0, long *m, double *d)
{
    double y = x / H;
    double fl = floor(y);
    double fr = y - fl;
    if (quant) fr = floor(fr * 32768.0) / 32768.0;
    if (fr < 0.5) {
        *n0 = (long)fl;
        *d = fr;
    } else {
        *n0 = (long)fl + 1;
        *d = fr - 1.0;
    }
    *m = (long)floor(*d * 32768.0);
}

/* The fixed-point TSC weights (units 2^-16) for d = m 2^-15: the outer two
 * are the eq. (5) values rounded to nearest (ties up), the centre one takes
 * the remainder so that the three sum to exactly 2^16. */
static inline void tsc_weights_fx(long m, uint64_t w[3])
{
    const uint64_t a = (uint64_t)(16384 - m), b = (uint64_t)(16384 + m);
    w[0] = (a * a + 16384u) >> 15;
    w[2] = (b * b + 16384u) >> 15;
    w[1] = 65536u - w[0] - w[2];
}

static inline void tsc_weights(long m, double d, int quant, double w[3])
{
    if (quant) {
        uint64_t wi[3];
        tsc_weights_fx(m, wi);
        for (int k = 0; k < 3; ++k) w[k] = (double)wi[k] / 65536.0;
    } else {
        w[0] = 0.5 * (0.5 - d) * (0.5 - d);
        w[1] = 0.75 - d * d;
        w[2] = 0.5 * (0.5 + d) * (0.5 + d);
    }
}

/* Exact integer TSC deposit: acc[n0 + s - 1] += prod_d W_d(s_d), s_d in
 * {0, 1, 2}, with the fixed-point weights above; density = acc * 2^-48. */
void orc_deposit_tsc_fx(int64_t N, const double *x, int n, double H, uint64_t *acc)
{
    for (int64_t i = 0; i < N; ++i) {
        long n0[3];
        uint64_t w[3][3];
        for (int d = 0; d < 3; ++d) {
            long m;
            double dd;
            tsc_coord(x[d * N + i], H, 1, &n0[d], &m, &dd);
            tsc_weights_fx(m, w[d]);
        }
        for (int sz = 0; sz < 3; ++sz)
            for (int sy = 0; sy < 3; ++sy)
                for (int sx = 0; sx < 3; ++sx)
                    acc[midx(n0[0] + sx - 1, n0[1] + sy - 1, n0[2] + sz - 1, n)] +=
                        w[0][sx] * w[1][sy] * w[2][sz];
    }
}

/* Floating-point TSC deposit, unit mass per particle. */
void orc_deposit_tsc(int64_t N, const double *x, int n, double H, int quant, double *rho)
{
    for (int64_t i = 0; i < N; ++i) {
        long n0[3];
        double w[3][3];
        for (int d = 0; d < 3; ++d) {
            long m;
            double dd;
            tsc_coord(x[d * N + i], H, quant, &n0[d], &m, &dd);
            tsc_weights(m, dd, quant, w[d]);
        }
        for (int sz = 0; sz < 3; ++sz)
            for (int sy = 0; sy < 3; ++sy)
                for (int sx = 0; sx < 3; ++sx)
                    rho[midx(n0[0] + sx - 1, n0[1] + sy - 1, n0[2] + sz - 1, n)] +=
                        w[0][sx] * w[1][sy] * w[2][sz];
    }
}

/* TSC interpolation with the deposit's weights: acc_i += sum_s W_s E(n0+s-1). */
void orc_interp_tsc(int64_t N, const double *x, int n, double H, int quant,
                    const double *E, double *acc)
{
    size_t n3 = (size_t)n * n * n;
#pragma omp parallel for
    for (int64_t i = 0; i < N; ++i) {
        long n0[3];
        double w[3][3];
        for (int d = 0; d < 3; ++d) {
            long m;
            double dd;
            tsc_coord(x[d * N + i], H, quant, &n0[d], &m, &dd);
            tsc_weights(m, dd, quant, w[d]);
        }
        for (int sz = 0; sz < 3; ++sz)
            for (int sy = 0; sy < 3; ++sy)
                for (int sx = 0; sx < 3; ++sx) {
                    double W = w[0][sx] * w[1][sy] * w[2][sz];
                    size_t c = midx(n0[0] + sx - 1, n0[1] + sy - 1, n0[2] + sz - 1, n);
                    for (int d = 0; d < 3; ++d) acc[d * N + i] += W * E[d * n3 + c];
                }
    }
}

/* eq. (7) with the physical sign: E_d(n) = -[(2/3)(phi(n+e_d) - phi(n-e_d))
 *                                     - (1/12)(phi(n+2e_d) - phi(n-2e_d))]. */
void orc_fd_force(int n, const double *phi, double *E)
{
    size_t n3 = (size_t)n * n * n;
#pragma omp parallel for collapse(2)
    for (long z = 0; z < n; ++z)
        for (long y = 0; y < n; ++y)
            for (long x = 0; x < n; ++x) {
                size_t c = midx(x, y, z, n);
                E[0 * n3 + c] = -(2.0 / 3.0 * (phi[midx(x + 1, y, z, n)] - phi[midx(x - 1, y, z, n)])
                                - 1.0 / 12.0 * (phi[midx(x + 2, y, z, n)] - phi[midx(x - 2, y, z, n)]));
                E[1 * n3 + c] = -(2.0 / 3.0 * (phi[midx(x, y + 1, z, n)] - phi[midx(x, y - 1, z, n)])
                                - 1.0 / 12.0 * (phi[midx(x, y + 2, z, n)] - phi[midx(x, y - 2, z, n)]));
                E[2 * n3 + c] = -(2.0 / 3.0 * (phi[midx(x, y, z + 1, n)] - phi[midx(x, y, z - 1, n)])
                                - 1.0 / 12.0 * (phi[midx(x, y, z + 2, n)] - phi[midx(x, y, z - 2, n)]));
            }
}

/* Transpose of orc_fd_force: phibar(m) = sum_d (2/3)(Eb_d(m+e_d) - Eb_d(m-e_d))
 *                                         - (1/12)(Eb_d(m+2e_d) - Eb_d(m-2e_d)). */
void orc_fd_force_adjoint(int n, const double *Eb, double *phibar)
{
    size_t n3 = (size_t)n * n * n;
#pragma omp parallel for collapse(2)
    for (long z = 0; z < n; ++z)
        for (long y = 0; y < n; ++y)
            for (long x = 0; x < n; ++x) {
                double s = 0.0;
                s += 2.0 / 3.0 * (Eb[0 * n3 + midx(x + 1, y, z, n)] - Eb[0 * n3 + midx(x - 1, y, z, n)])
                   - 1.0 / 12.0 * (Eb[0 * n3 + midx(x + 2, y, z, n)] - Eb[0 * n3 + midx(x - 2, y, z, n)]);
                s += 2.0 / 3.0 * (Eb[1 * n3 + midx(x, y + 1, z, n)] - Eb[1 * n3 + midx(x, y - 1, z, n)])
                   - 1.0 / 12.0 * (Eb[1 * n3 + midx(x, y + 2, z, n)] - Eb[1 * n3 + midx(x, y - 2, z, n)]);
                s += 2.0 / 3.0 * (Eb[2 * n3 + midx(x, y, z + 1, n)] - Eb[2 * n3 + midx(x, y, z - 1, n)])
                   - 1.0 / 12.0 * (Eb[2 * n3 + midx(x, y, z + 2, n)] - Eb[2 * n3 + midx(x, y, z - 2, n)]);
                phibar[midx(x, y, z, n)] += s;
            }
}

/* CIC interpolation with the deposit's weights: acc_i += sum_s W_s E(j+s).
 * E holds three meshes [d][z][y][x].  No unit conversion here. */
void orc_interp(int64_t N, const double *x, int n, double H, int quant,
                const double *E, double *acc)
{
    size_t n3 = (size_t)n * n * n;
#pragma omp parallel for
    for (int64_t i = 0; i < N; ++i) {
        long j[3];
        double w[3][2];
        for (int d = 0; d < 3; ++d) {
            double f;
            cic_coord(x[d * N + i], H, quant, &j[d], &f);
            w[d][0] = 1.0 - f;
            w[d][1] = f;
        }
        for (int sz = 0; sz < 2; ++sz)
            for (int sy = 0; sy < 2; ++sy)
                for (int sx = 0; sx < 2; ++sx) {
                    double W = w[0][sx] * w[1][sy] * w[2][sz];
                    size_t c = midx(j[0] + sx, j[1] + sy, j[2] + sz, n);
                    for (int d = 0; d < 3; ++d) acc[d * N + i] += W * E[d * n3 + c];
                }
    }
}

/* Adjoint of orc_interp with respect to the meshes: Eb(j+s) += W_s abar_i. */
void orc_interp_adjoint_mesh(int64_t N, const double *x, int n, double H, int quant,
                             const double *abar, double *Eb)
{
    size_t n3 = (size_t)n * n * n;
    for (int64_t i = 0; i < N; ++i) {
        long j[3];
        double w[3][2];
        for (int d = 0; d < 3; ++d) {
            double f;
            cic_coord(x[d * N + i], H, quant, &j[d], &f);
            w[d][0] = 1.0 - f;
            w[d][1] = f;
        }
        for (int sz = 0; sz < 2; ++sz)
            for (int sy = 0; sy < 2; ++sy)
                for (int sx = 0; sx < 2; ++sx) {
                    double W = w[0][sx] * w[1][sy] * w[2][sz];
                    size_t c = midx(j[0] + sx, j[1] + sy, j[2] + sz, n);
                    for (int d = 0; d < 3; ++d) Eb[d * n3 + c] += W * abar[d * N + i];
                }
    }
}

/* Gradient of the CIC weights: dW_s/dx_d = (1/H) (s_d ? +1 : -1) prod_{e!=d} w_e.
 * At cell faces the left-continuous value is used (weights of the cell that
 * holds the particle). */
static inline void cic_grad(const double w[3][2], int sx, int sy, int sz, double H,
                            double g[3])
{
    int s[3] = {sx, sy, sz};
    for (int d = 0; d < 3; ++d) {
        double v = (s[d] ? 1.0 : -1.0) / H;
        for (int e = 0; e < 3; ++e)
            if (e != d) v *= w[e][s[e]];
        g[d] = v;
    }
}

/* Position adjoint of the interpolation: xbar_i += sum_s grad W_s (abar_i . E(j+s)). */
void orc_interp_adjoint_pos(int64_t N, const double *x, int n, double H, int quant,
                            const double *E, const double *abar, double *xbar)
{
    size_t n3 = (size_t)n * n * n;
#pragma omp parallel for
    for (int64_t i = 0; i < N; ++i) {
        long j[3];
        double w[3][2];
        for (int d = 0; d < 3; ++d) {
            double f;
            cic_coord(x[d * N + i], H, quant, &j[d], &f);
            w[d][0] = 1.0 - f;
            w[d][1] = f;
        }
        for (int sz = 0; sz < 2; ++sz)
            for (int sy = 0; sy < 2; ++sy)
                for (int sx = 0; sx < 2; ++sx) {
                    size_t c = midx(j[0] + sx, j[1] + sy, j[2] + sz, n);
                    double dot = 0.0;
                    for (int d = 0; d < 3; ++d) dot += abar[d * N + i] * E[d * n3 + c];
                    double g[3];
                    cic_grad(w, sx, sy, sz, H, g);
                    for (int d = 0; d < 3; ++d) xbar[d * N + i] += g[d] * dot;
                }
    }
}

/* Position adjoint of the deposit: xbar_i += sum_s grad W_s rhobar(j+s). */
void orc_deposit_adjoint_pos(int64_t N, const double *x, int n, double H, int quant,
                             const double *rhobar, double *xbar)
{
#pragma omp parallel for
    for (int64_t i = 0; i < N; ++i) {
        long j[3];
        double w[3][2];
        for (int d = 0; d < 3; ++d) {
            double f;
            cic_coord(x[d * N + i], H, quant, &j[d], &f);
            w[d][0] = 1.0 - f;
            w[d][1] = f;
        }
        for (int sz = 0; sz < 2; ++sz)
            for (int sy = 0; sy < 2; ++sy)
                for (int sx = 0; sx < 2; ++sx) {
                    double rb = rhobar[midx(j[0] + sx, j[1] + sy, j[2] + sz, n)];
                    double g[3];
                    cic_grad(w, sx, sy, sz, H, g);
                    for (int d = 0; d < 3; ++d) xbar[d * N + i] += g[d] * rb;
                }
    }
}

/* TSC versions of the three adjoints above (eq. 5).  The weights are the
 * forward's; their derivative with respect to the particle coordinate is
 * that of the continuous eq. (5) at the (quantised) offset d from the
 * nearest node, per axis in level units:
 *   dW(n0-1)/dy = -(1/2 - d),  dW(n0)/dy = -2 d,  dW(n0+1)/dy = 1/2 + d,
 * divided by H for fine-cell coordinates (the fixed-point rounding of the
 * weights is taken as the identity, as the quantisation of positions is). */
static inline void tsc_setup(double xv, double H, int quant, long *n0, double w[3], double dw[3])
{
    long m;
    double d;
    tsc_coord(xv, H, quant, n0, &m, &d);
    tsc_weights(m, d, quant, w);
    dw[0] = -(0.5 - d) / H;
    dw[1] = -2.0 * d / H;
    dw[2] = (0.5 + d) / H;
}

/* Adjoint of orc_interp_tsc with respect to the meshes: Eb(n0+s-1) += W_s abar_i. */
void orc_interp_adjoint_mesh_tsc(int64_t N, const double *x, int n, double H, int quant,
                                 const double *abar, double *Eb)
{
    size_t n3 = (size_t)n * n * n;
    for (int64_t i = 0; i < N; ++i) {
        long n0[3];
        double w[3][3], dw[3][3];
        for (int d = 0; d < 3; ++d) tsc_setup(x[d * N + i], H, quant, &n0[d], w[d], dw[d]);
        for (int sz = 0; sz < 3; ++sz)
            for (int sy = 0; sy < 3; ++sy)
                for (int sx = 0; sx < 3; ++sx) {
                    double W = w[0][sx] * w[1][sy] * w[2][sz];
                    size_t c = midx(n0[0] + sx - 1, n0[1] + sy - 1, n0[2] + sz - 1, n);
                    for (int d = 0; d < 3; ++d) Eb[d * n3 + c] += W * abar[d * N + i];
                }
    }
}

/* grad W_s = (dW_x w_y w_z, w_x dW_y w_z, w_x w_y dW_z) for the node offsets s. */
static inline void tsc_grad(const double w[3][3], const double dw[3][3], int sx, int sy, int sz,
                            double g[3])
{
    g[0] = dw[0][sx] * w[1][sy] * w[2][sz];
    g[1] = w[0][sx] * dw[1][sy] * w[2][sz];
    g[2] = w[0][sx] * w[1][sy] * dw[2][sz];
}

/* Position adjoint of the TSC interpolation: xbar_i += sum_s grad W_s (abar_i . E(n0+s-1)). */
void orc_interp_adjoint_pos_tsc(int64_t N, const double *x, int n, double H, int quant,
                                const double *E, const double *abar, double *xbar)
{
    size_t n3 = (size_t)n * n * n;
#pragma omp parallel for
    for (int64_t i = 0; i < N; ++i) {
        long n0[3];
        double w[3][3], dw[3][3];
        for (int d = 0; d < 3; ++d) tsc_setup(x[d * N + i], H, quant, &n0[d], w[d], dw[d]);
        for (int sz = 0; sz < 3; ++sz)
            for (int sy = 0; sy < 3; ++sy)
                for (int sx = 0; sx < 3; ++sx) {
                    size_t c = midx(n0[0] + sx - 1, n0[1] + sy - 1, n0[2] + sz - 1, n);
                    double dot = 0.0;
                    for (int d = 0; d < 3; ++d) dot += abar[d * N + i] * E[d * n3 + c];
                    double g[3];
                    tsc_grad(w, dw, sx, sy, sz, g);
                    for (int d = 0; d < 3; ++d) xbar[d * N + i] += g[d] * dot;
                }
    }
}

/* Position adjoint of the TSC deposit: xbar_i += sum_s grad W_s rhobar(n0+s-1). */
void orc_deposit_adjoint_pos_tsc(int64_t N, const double *x, int n, double H, int quant,
                                 const double *rhobar, double *xbar)
{
#pragma omp parallel for
    for (int64_t i = 0; i < N; ++i) {
        long n0[3];
        double w[3][3], dw[3][3];
        for (int d = 0; d < 3; ++d) tsc_setup(x[d * N + i], H, quant, &n0[d], w[d], dw[d]);
        for (int sz = 0; sz < 3; ++sz)
            for (int sy = 0; sy < 3; ++sy)
                for (int sx = 0; sx < 3; ++sx) {
                    double rb = rhobar[midx(n0[0] + sx - 1, n0[1] + sy - 1, n0[2] + sz - 1, n)];
                    double g[3];
                    tsc_grad(w, dw, sx, sy, sz, g);
                    for (int d = 0; d < 3; ++d) xbar[d * N + i] += g[d] * rb;
                }
    }
}

/* ------------------------------------------------------------------ */
/* PP: eq. (4d) with the PM3 softening replaced by the fine one         */
/* ------------------------------------------------------------------ */

/* g(r) = [R(r, b_pp) - R(r, b_f)] / r for 0 < r < b_f, else 0. */
static xreal pp_g_x(xreal r, xreal b_pp, xreal b_f)
{
    if (!(r > 0.0L) || r >= b_f) return 0.0L;
    return (refforce_x(r, b_pp) - refforce_x(r, b_f)) / r;
}

/* g'(r) */
static xreal pp_dg_x(xreal r, xreal b_pp, xreal b_f)
{
    if (!(r > 0.0L) || r >= b_f) return 0.0L;
    xreal R = refforce_x(r, b_pp) - refforce_x(r, b_f);
    xreal dR = refforce_dr_x(r, b_pp) - refforce_dr_x(r, b_f);
    return dR / r - R / (r * r);
}

double orc_pp_g(double r, double b_pp, double b_f) { return (double)pp_g_x(r, b_pp, b_f); }
double orc_pp_dg(double r, double b_pp, double b_f) { return (double)pp_dg_x(r, b_pp, b_f); }

/* g at the squared separation r2 (exact in FP64 for quantised positions). */
static inline double pp_g_r2(double r2, double b_pp, double b_f)
{
    return (double)pp_g_x(sqrtl((xreal)r2), b_pp, b_f);
}

static inline double minimg(double d, double L)
{
    if (d >= 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

/* Brute force O(N^2) minimum-image pair sum: acc_i += sum_j g(r_ij) (x_j - x_i). */
void orc_pp_brute(int64_t N, const double *x, double L, double b_pp, double b_f, double *acc)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        double a[3] = {0, 0, 0};
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            double D[3], r2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                D[d] = minimg(x[d * N + j] - x[d * N + i], L);
                r2 += D[d] * D[d];
            }
            double g = pp_g_r2(r2, b_pp, b_f);
            for (int d = 0; d < 3; ++d) a[d] += g * D[d];
        }
        for (int d = 0; d < 3; ++d) acc[d * N + i] += a[d];
    }
}

/* Linked-list cells of side >= b_f over the periodic box of side L. */
typedef struct { int nc; double cs; int64_t *head, *next; } cells_t;

static int cells_build(int64_t N, const double *x, double L, double b_f, cells_t *c)
{
    c->nc = (int)floor(L / b_f);
    if (c->nc < 3) return 0;
    c->cs = L / c->nc;
    size_t nc3 = (size_t)c->nc * c->nc * c->nc;
    c->head = (int64_t *)malloc(nc3 * sizeof(int64_t));
    c->next = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    for (size_t k = 0; k < nc3; ++k) c->head[k] = -1;
    for (int64_t i = N - 1; i >= 0; --i) {
        long ci[3];
        for (int d = 0; d < 3; ++d) ci[d] = wrapi((long)floor(x[d * N + i] / c->cs), c->nc);
        size_t k = midx(ci[0], ci[1], ci[2], c->nc);
        c->next[i] = c->head[k];
        c->head[k] = i;
    }
    return 1;
}

static void cells_free(cells_t *c) { free(c->head); free(c->next); }

/* PP sum over the 27 neighbouring linked-list cells; same pair set as the
 * brute force because the cell side is at least the cutoff. */
void orc_pp(int64_t N, const double *x, double L, double b_pp, double b_f, double *acc)
{
    cells_t c;
    if (!cells_build(N, x, L, b_f, &c)) { orc_pp_brute(N, x, L, b_pp, b_f, acc); return; }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) {
        long ci[3];
        for (int d = 0; d < 3; ++d) ci[d] = wrapi((long)floor(x[d * N + i] / c.cs), c.nc);
        double a[3] = {0, 0, 0};
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox)
                    for (int64_t j = c.head[midx(ci[0] + ox, ci[1] + oy, ci[2] + oz, c.nc)]; j >= 0;
                         j = c.next[j]) {
                        if (j == i) continue;
                        double D[3], r2 = 0.0;
                        for (int d = 0; d < 3; ++d) {
                            D[d] = minimg(x[d * N + j] - x[d * N + i], L);
                            r2 += D[d] * D[d];
                        }
                        double g = pp_g_r2(r2, b_pp, b_f);
                        for (int d = 0; d < 3; ++d) a[d] += g * D[d];
                    }
        for (int d = 0; d < 3; ++d) acc[d * N + i] += a[d];
    }
    cells_free(&c);
}

/* PP for a subset of target particles (indices idx[0..M)), sources all N. */
void orc_pp_subset(int64_t N, const double *x, double L, double b_pp, double b_f,
                   int64_t M, const int64_t *idx, double *acc /* 3*M */)
{
    cells_t c;
    int have = cells_build(N, x, L, b_f, &c);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < M; ++t) {
        int64_t i = idx[t];
        double a[3] = {0, 0, 0};
        if (have) {
            long ci[3];
            for (int d = 0; d < 3; ++d) ci[d] = wrapi((long)floor(x[d * N + i] / c.cs), c.nc);
            for (int oz = -1; oz <= 1; ++oz)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int ox = -1; ox <= 1; ++ox)
                        for (int64_t j = c.head[midx(ci[0] + ox, ci[1] + oy, ci[2] + oz, c.nc)];
                             j >= 0; j = c.next[j]) {
                            if (j == i) continue;
                            double D[3], r2 = 0.0;
                            for (int d = 0; d < 3; ++d) {
                                D[d] = minimg(x[d * N + j] - x[d * N + i], L);
                                r2 += D[d] * D[d];
                            }
                            double g = pp_g_r2(r2, b_pp, b_f);
                            for (int d = 0; d < 3; ++d) a[d] += g * D[d];
                        }
        } else {
            for (int64_t j = 0; j < N; ++j) {
                if (j == i) continue;
                double D[3], r2 = 0.0;
                for (int d = 0; d < 3; ++d) {
                    D[d] = minimg(x[d * N + j] - x[d * N + i], L);
                    r2 += D[d] * D[d];
                }
                double g = pp_g_r2(r2, b_pp, b_f);
                for (int d = 0; d < 3; ++d) a[d] += g * D[d];
            }
        }
        for (int d = 0; d < 3; ++d) acc[d * M + t] = a[d];
    }
    if (have) cells_free(&c);
}

/* Number of ordered pairs with 0 < r < b_f (the PP work count). */
int64_t orc_pp_count(int64_t N, const double *x, double L, double b_f)
{
    cells_t c;
    int64_t total = 0;
    if (!cells_build(N, x, L, b_f, &c)) return -1;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t i = 0; i < N; ++i) {
        long ci[3];
        for (int d = 0; d < 3; ++d) ci[d] = wrapi((long)floor(x[d * N + i] / c.cs), c.nc);
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox)
                    for (int64_t j = c.head[midx(ci[0] + ox, ci[1] + oy, ci[2] + oz, c.nc)]; j >= 0;
                         j = c.next[j]) {
                        if (j == i) continue;
                        double r2 = 0.0;
                        for (int d = 0; d < 3; ++d) {
                            double D = minimg(x[d * N + j] - x[d * N + i], L);
                            r2 += D * D;
                        }
                        if (r2 > 0.0 && r2 < b_f * b_f) total++;
                    }
    }
    cells_free(&c);
    return total;
}

/* Adjoint of the PP sum for one particle k: with J(D) = g(r) I + g'(r) D D^T / r
 * (symmetric, even), out = sum_j J(D_kj) (abar_j - abar_k), D_kj = x_j - x_k,
 * over the 27 linked-list cells around k (all N particles without cells). */
static void pp_adjoint_one(int64_t k, int64_t N, const double *x, double L, double b_pp,
                           double b_f, const double *abar, const cells_t *c, int have,
                           double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    long ck[3] = {0, 0, 0};
    if (have)
        for (int d = 0; d < 3; ++d) ck[d] = wrapi((long)floor(x[d * N + k] / c->cs), c->nc);
    int64_t jlist_end = have ? 27 : 1;
    for (int64_t cell = 0; cell < jlist_end; ++cell) {
        int64_t j;
        if (have) {
            int ox = (int)(cell % 3) - 1, oy = (int)((cell / 3) % 3) - 1, oz = (int)(cell / 9) - 1;
            j = c->head[midx(ck[0] + ox, ck[1] + oy, ck[2] + oz, c->nc)];
        } else {
            j = 0;
        }
        for (; have ? j >= 0 : j < N; j = have ? c->next[j] : j + 1) {
            if (j == k) continue;
            double D[3], r2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                D[d] = minimg(x[d * N + j] - x[d * N + k], L);
                r2 += D[d] * D[d];
            }
            xreal rx = sqrtl((xreal)r2);
            if (!(rx > 0.0L) || rx >= b_f) continue;
            double r = (double)rx;
            double g = (double)pp_g_x(rx, b_pp, b_f), gp = (double)pp_dg_x(rx, b_pp, b_f);
            double u[3], Du = 0.0;
            for (int d = 0; d < 3; ++d) {
                u[d] = abar[d * N + j] - abar[d * N + k];
                Du += D[d] * u[d];
            }
            for (int d = 0; d < 3; ++d) out[d] += g * u[d] + gp * D[d] * Du / r;
        }
    }
}

/* Adjoint of the PP sum: xbar_k += sum_j J(D_kj) (abar_j - abar_k). */
void orc_pp_adjoint(int64_t N, const double *x, double L, double b_pp, double b_f,
                    const double *abar, double *xbar)
{
    cells_t c;
    int have = cells_build(N, x, L, b_f, &c);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < N; ++k) {
        double out[3];
        pp_adjoint_one(k, N, x, L, b_pp, b_f, abar, &c, have, out);
        for (int d = 0; d < 3; ++d) xbar[d * N + k] += out[d];
    }
    if (have) cells_free(&c);
}

/* The same adjoint for the target particles idx[0..M) only (sources all N):
 * xbar[d*M + t] = (sum_j J(D_kj) (abar_j - abar_k))_d with k = idx[t]. */
void orc_pp_adjoint_subset(int64_t N, const double *x, double L, double b_pp, double b_f,
                           const double *abar, int64_t M, const int64_t *idx, double *xbar)
{
    cells_t c;
    int have = cells_build(N, x, L, b_f, &c);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < M; ++t) {
        double out[3];
        pp_adjoint_one(idx[t], N, x, L, b_pp, b_f, abar, &c, have, out);
        for (int d = 0; d < 3; ++d) xbar[d * M + t] = out[d];
    }
    if (have) cells_free(&c);
}
