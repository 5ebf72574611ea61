// green.hip -- FP64 construction of the optimized Green's function (eq. 11)
// and the FFT twiddle tables; runs once per context (cube2_init_tables).
//
// For the level mesh with n nodes and wave vector k = 2 pi m / n:
//   G(k) = -4 pi sum_a W^2(k_a) (d . k_a) dS2(|k_a|) / |k_a|^2
//          / ( |d|^2 [sum_a W^2(k_a)]^2 )
// with k_a = k + 2 pi a, |a_d| <= nmax (section 2.1.2: max |n| <= 2),
// W(k) = prod_d sinc^p(k_d / 2) (eq. 9: p = 2 for CIC, 3 for TSC),
// d_d = 4/3 sin k_d - 1/6 sin 2 k_d (eq. 10, D = i d),
// dS2 = S^2(|k|, b_a) - S^2(|k|, b_prev) (eq. 12; S of eq. 13; S(k, inf) = 0).
// This is eq. (11) with D . R* = -4 pi (d . k_a) dS2 / k_a^2.  G = 0 where
// |d| = 0.  With isolated boundaries (appendix A) the untruncated level's
// dS2 is multiplied by 1 - sinc(|k_a| L), L half the mesh length.  The table is stored as FP32 over the octant |m_d| <= n/2 (and,
// for the FP64 plain form, a second time in FP64).
#include "common.hpp"

namespace cube2 {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// S(k, b) of eq. (13) as a function of u = k b / 2:  12 (2 - 2cos u - u sin u) / u^4.
// Below u = 0.75 the Taylor polynomial in u^2 is used (the closed form
// cancels); its coefficients are 12 (-1)^(j+1) (2 - 2j) / (2j)!.
__device__ double profile_k(double u) {
    if (u < 0.75) {
        const double t = u * u;
        return 1.0 + t * (-1.0 / 15.0 + t * (1.0 / 560.0 + t * (-1.0 / 37800.0 +
               t * (1.0 / 3991680.0 + t * (-1.0 / 605404800.0 + t * (1.0 / 124540416000.0))))));
    }
    const double u2 = u * u;
    return 12.0 * (2.0 - 2.0 * cos(u) - u * sin(u)) / (u2 * u2);
}

template <typename T>
__global__ void green_kernel(T *__restrict__ out, int n, double ba, double bprev, int nmax,
                             int p, double iso_L) {
    const int h = n / 2 + 1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)h * h * h) return;
    const int m[3] = {(int)(idx % h), (int)((idx / h) % h), (int)(idx / ((int64_t)h * h))};

    double d[3], dd = 0.0, k[3];
    for (int a = 0; a < 3; ++a) {
        const double f = (double)m[a] / (double)n;
        k[a] = 2.0 * kPi * f;
        d[a] = (4.0 / 3.0) * sinpi(2.0 * f) - (1.0 / 6.0) * sinpi(4.0 * f);
        dd += d[a] * d[a];
    }
    if (dd == 0.0) {
        out[idx] = T(0);
        return;
    }
    // Per-axis alias windows w[a][j] = sinc^(2p)((k_a + 2 pi j)/2), j = -nmax..nmax
    // (W^2 of eq. 9: p = 2 for CIC, 3 for TSC).
    double w[3][9];
    for (int a = 0; a < 3; ++a)
        for (int j = -nmax; j <= nmax; ++j) {
            const double t = (double)m[a] / (double)n + (double)j;  // (k + 2 pi j)/2 = pi t
            const double s = (t == 0.0) ? 1.0 : sinpi(t) / (kPi * t);
            const double s2 = s * s;
            w[a][j + nmax] = p == 3 ? s2 * s2 * s2 : s2 * s2;
        }
    double U = 0.0, V = 0.0;
    for (int jz = -nmax; jz <= nmax; ++jz)
        for (int jy = -nmax; jy <= nmax; ++jy)
            for (int jx = -nmax; jx <= nmax; ++jx) {
                const double W2 = w[0][jx + nmax] * w[1][jy + nmax] * w[2][jz + nmax];
                U += W2;
                const double kx = k[0] + 2.0 * kPi * jx, ky = k[1] + 2.0 * kPi * jy,
                             kz = k[2] + 2.0 * kPi * jz;
                const double kk = kx * kx + ky * ky + kz * kz;
                if (kk == 0.0) continue;
                const double km = sqrt(kk);
                const double sa = profile_k(0.5 * km * ba);
                const double sp = bprev > 0.0 ? profile_k(0.5 * km * bprev) : 0.0;
                // isolated boundaries (appendix A): the target force truncated
                // at r = iso_L, whose transform is [1 - sinc(k iso_L)] R(k)
                const double iso = iso_L > 0.0 ? 1.0 - sin(km * iso_L) / (km * iso_L) : 1.0;
                V += W2 * (d[0] * kx + d[1] * ky + d[2] * kz) * (sa * sa - sp * sp) * iso / kk;
            }
    out[idx] = (T)(-4.0 * kPi * V / (dd * U * U));
}

// W_n^m = exp(-2 pi i m / n), m = 0..n-1, from FP64.
// The octant table g[mz][my][kx] re-laid out for the z pass of the FFT:
// gz[my][kx / 16][mz][kx % 16], kx padded to the spectrum pitch with zeros,
// so that each z-line workgroup (16 adjacent kx, one ky) reads one
// contiguous block.
__global__ void green_zorder_kernel(const float *__restrict__ g, float *__restrict__ gz, int h,
                                    int ngrp) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)h * ngrp * h * 16) return;
    const int c = (int)(idx & 15);
    const int64_t r = idx >> 4;
    const int mz = (int)(r % h), grp = (int)((r / h) % ngrp), my = (int)(r / ((int64_t)h * ngrp));
    const int kx = grp * 16 + c;
    gz[idx] = kx < h ? g[((int64_t)mz * h + my) * h + kx] : 0.0f;
}

__global__ void twiddle_kernel(float2 *__restrict__ tw, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const double f = 2.0 * (double)m / (double)n;
    tw[m] = make_float2((float)cospi(f), (float)(-sinpi(f)));
}

__global__ void twiddle64_kernel(double2 *__restrict__ tw, int n) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const double f = 2.0 * (double)m / (double)n;
    tw[m] = make_double2(cospi(f), -sinpi(f));
}

}  // namespace

int launch_green(cube2_ctx *ctx, hipStream_t s) {
    for (int l = 0; l < ctx->n_levels; ++l) {
        const Level &L = ctx->lv[l];
        float2 *tw = reinterpret_cast<float2 *>(ctx->tables + L.tw_off);
        twiddle_kernel<<<(L.n + 255) / 256, 256, 0, s>>>(tw, L.n);
        CUBE2_LAUNCH_CHECK();
        const int64_t h = L.n / 2 + 1;
        const int64_t pts = h * h * h;
        float *g = reinterpret_cast<float *>(ctx->tables + L.g_off);
        const double ba = L.b_a / L.H;
        const double bp = L.b_prev > 0.0 ? L.b_prev / L.H : -1.0;
        // isolated boundaries: the untruncated level's force is cut at half the box
        const double iso_L = (ctx->isolated && bp <= 0.0) ? 0.5 * L.n : 0.0;
        green_kernel<float><<<(unsigned)((pts + 255) / 256), 256, 0, s>>>(
            g, L.n, ba, bp, ctx->cfg.alias_nmax, ctx->tsc ? 3 : 2, iso_L);
        CUBE2_LAUNCH_CHECK();
        const int ngrp = L.pitch / 16;
        const int64_t zpts = h * ngrp * h * 16;
        green_zorder_kernel<<<(unsigned)((zpts + 255) / 256), 256, 0, s>>>(
            g, reinterpret_cast<float *>(ctx->tables + L.gz_off), (int)h, ngrp);
        CUBE2_LAUNCH_CHECK();
        if (ctx->fp64) {
            twiddle64_kernel<<<(L.n + 255) / 256, 256, 0, s>>>(
                reinterpret_cast<double2 *>(ctx->tables + L.tw64_off), L.n);
            CUBE2_LAUNCH_CHECK();
            green_kernel<double><<<(unsigned)((pts + 255) / 256), 256, 0, s>>>(
                reinterpret_cast<double *>(ctx->tables + L.g64_off), L.n, ba, bp,
                ctx->cfg.alias_nmax, ctx->tsc ? 3 : 2, iso_L);
            CUBE2_LAUNCH_CHECK();
        }
    }
    return CUBE2_OK;
}

}  // namespace cube2
