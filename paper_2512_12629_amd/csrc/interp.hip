// interp.hip -- finite-difference force (eq. 7) and CIC interpolation back to
// the particles (section 2.1.2, steps 3 and 4) for both PM levels in one
// sweep over the cell-sorted particles.
//
// One workgroup per tile (8^3 IOS cells = 16^3 fine cells).  It stages in LDS
// the fine potential on the tile plus a halo (2 nodes for the stencil below,
// 3 above: the CIC upper node plus the stencil), and the coarse potential on
// the tile's coarse footprint with the same halo.  Each particle then reads
// the 6 potential values along each axis around its 2x2 CIC footprint and
// forms E = -[(2/3)(phi(+1) - phi(-1)) - (1/12)(phi(+2) - phi(-2))] at its two
// nodes per axis, weighted with the deposit's 15-bit integer weights.
// With TSC assignment (eq. 5) each particle has three nodes per axis around
// its nearest node, with the deposit's 16-bit weights, and the staged tiles
// carry one more halo node on each side.
// The kernel is templated on the real type: float for the production path,
// double for the FP64 plain form.
#include "common.hpp"

namespace cube2 {
namespace {

// TSC: nodes n0-1..n0+1 with n0 in [0, 16/H] plus the stencil: 3 below, 4 above
template <int P> struct InterpGeo {
    static constexpr int HLO = P == 3 ? 3 : 2;                 // halo below the tile
    static constexpr int FS = kTileFine + (P == 3 ? 7 : 5);    // 21 or 23
    static constexpr int CSMAX = kTileFine / 2 + (P == 3 ? 7 : 5);
};

// The FD force at the particle's two nodes along one axis, CIC-weighted
// (w0 E(j) + w1 E(j+1)), is one 6-tap filter over phi(j-2..j+3); its taps
// depend only on the axis weights, so they are formed once per particle and
// axis.  With E(i) = -[c1 (phi(i+1) - phi(i-1)) - c2 (phi(i+2) - phi(i-2))],
// c1 = 2/3, c2 = 1/12, the taps are
//   -c2 w0, c1 w0 - c2 w1, c1 w1, -c1 w0, c2 w0 - c1 w1, c2 w1.
template <typename T> struct Taps { T t[6]; };

template <typename T>
__device__ __forceinline__ Taps<T> axis_taps(T w0, T w1) {
    const T c1 = T(2.0 / 3.0), c2 = T(1.0 / 12.0);
    const T a = c1 * w0, b = c2 * w0, c = c1 * w1, d = c2 * w1;
    return Taps<T>{{-b, a - d, c, -a, b - c, d}};
}

// One line of the filter: p points at phi(j) on that axis, st is the axis
// stride in LDS.
template <typename T>
__device__ __forceinline__ T axis_line(const T *p, int st, const Taps<T> &k) {
    T r = p[-2 * st] * k.t[0];
    r = fma(p[-st], k.t[1], r);
    r = fma(p[0], k.t[2], r);
    r = fma(p[st], k.t[3], r);
    r = fma(p[2 * st], k.t[4], r);
    return fma(p[3 * st], k.t[5], r);
}

// CIC-weighted force of a staged potential tile P (side S) at the particle
// whose lower CIC node is (jx, jy, jz) in tile coordinates.
template <typename T>
__device__ __forceinline__ void gather(const T *P, int S, int jx, int jy, int jz,
                                       const T (&wx)[2], const T (&wy)[2], const T (&wz)[2],
                                       T &ax, T &ay, T &az) {
    const int SS = S * S;
    const Taps<T> kx = axis_taps(wx[0], wx[1]), ky = axis_taps(wy[0], wy[1]),
                  kz = axis_taps(wz[0], wz[1]);
    ax = ay = az = T(0);
#pragma unroll
    for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
            // x: nodes (jx.., jy+s1, jz+s2)
            ax = fma(wy[s1] * wz[s2], axis_line(P + (jz + s2) * SS + (jy + s1) * S + jx, 1, kx), ax);
            // y: nodes (jx+s1, jy.., jz+s2)
            ay = fma(wx[s1] * wz[s2], axis_line(P + (jz + s2) * SS + jy * S + jx + s1, S, ky), ay);
            // z: nodes (jx+s1, jy+s2, jz..)
            az = fma(wx[s1] * wy[s2], axis_line(P + jz * SS + (jy + s2) * S + jx + s1, SS, kz), az);
        }
}

// FD force at the particle's three TSC nodes along one axis (n0-1, n0, n0+1),
// weighted; p points at phi(n0) on that axis, st is the axis stride in LDS.
template <typename T>
__device__ __forceinline__ T axis_force3(const T *p, int st, const T (&w)[3]) {
    const T pm3 = p[-3 * st], pm2 = p[-2 * st], pm1 = p[-st], p0 = p[0], p1 = p[st],
            p2 = p[2 * st], p3 = p[3 * st];
    const T c1 = T(2.0 / 3.0), c2 = T(1.0 / 12.0);
    const T e0 = -(c1 * (p0 - pm2) - c2 * (p1 - pm3));
    const T e1 = -(c1 * (p1 - pm1) - c2 * (p2 - pm2));
    const T e2 = -(c1 * (p2 - p0) - c2 * (p3 - pm1));
    return w[0] * e0 + w[1] * e1 + w[2] * e2;
}

// TSC-weighted force of a staged potential tile P (side S) at the particle
// whose nearest node is (nx, ny, nz) in LDS coordinates.
template <typename T>
__device__ __forceinline__ void gather3(const T *P, int S, int nx, int ny, int nz,
                                        const T (&wx)[3], const T (&wy)[3], const T (&wz)[3],
                                        T &ax, T &ay, T &az) {
    const int SS = S * S;
    ax = ay = az = T(0);
    // the outer loop stays rolled: unrolled, the 189 window reads of the nine
    // lines per axis need 256 registers and spill
#pragma unroll 1
    for (int s1 = 0; s1 < 3; ++s1)
#pragma unroll
        for (int s2 = 0; s2 < 3; ++s2) {
            ax += wy[s1] * wz[s2] * axis_force3(P + (nz - 1 + s2) * SS + (ny - 1 + s1) * S + nx, 1, wx);
            ay += wx[s1] * wz[s2] * axis_force3(P + (nz - 1 + s2) * SS + ny * S + nx - 1 + s1, S, wy);
            az += wx[s1] * wy[s2] * axis_force3(P + nz * SS + (ny - 1 + s2) * S + nx - 1 + s1, SS, wz);
        }
}

// At least two waves per SIMD: left alone, the compiler gives the two-level
// TSC gather all 256 VGPRs and one wave per SIMD.  FINE = false gathers the
// coarse level only (the tile+buffer mode computes the fine level per tile).
// HS > 0 fixes log2 of the coarse ratio at compile time (the coarse tile's
// LDS strides then fold into immediate offsets); HS = 0 reads it from hshift.
template <bool TWO, int P, typename T, bool FINE = true, int HS = 0>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void interp_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs, int n, int n_f, int nt,
    const T *__restrict__ phi_f, const T *__restrict__ phi_c, int n_c, int hshift_arg, T scale_f,
    T scale_c, T *__restrict__ acc, int accumulate) {
    constexpr int FS = InterpGeo<P>::FS, HLO = InterpGeo<P>::HLO, CSM = InterpGeo<P>::CSMAX;
    __shared__ T pf[FINE ? FS * FS * FS : 1];
    __shared__ T pc[TWO ? CSM * CSM * CSM : 1];
    __shared__ uint32_t cst[kTileCells + 1];

    int tx, ty, tz;
    tile_of_block(blockIdx.x, nt, tx, ty, tz);
    const int tid = threadIdx.x;
    const int hshift = HS > 0 ? HS : hshift_arg;
    const uint32_t key0 = (uint32_t)((tz * nt + ty) * nt + tx) * kTileCells;
    stage_cell_starts<kBlock>(cst, cs, key0);
    const int ax0 = tx * kTileFine, ay0 = ty * kTileFine, az0 = tz * kTileFine;
    if (FINE) stage_block<FS, kBlock>(pf, phi_f, n_f, ax0 - HLO, ay0 - HLO, az0 - HLO);
    const int CS = (kTileFine >> hshift) + FS - kTileFine;
    if (TWO) {
        const int cx0 = (ax0 >> hshift) - HLO, cy0 = (ay0 >> hshift) - HLO,
                  cz0 = (az0 >> hshift) - HLO;
        switch (hshift) {
            case 1: stage_block<kTileFine / 2 + FS - kTileFine, kBlock>(pc, phi_c, n_c, cx0, cy0, cz0); break;
            case 2: stage_block<kTileFine / 4 + FS - kTileFine, kBlock>(pc, phi_c, n_c, cx0, cy0, cz0); break;
            default: stage_block<kTileFine / 8 + FS - kTileFine, kBlock>(pc, phi_c, n_c, cx0, cy0, cz0); break;
        }
    }
    __syncthreads();
    const uint32_t p0 = cst[0], p1 = cst[kTileCells];
    const T inv = T(1.0 / 32768.0);
    // two particles per thread at a time (one for TSC, whose gather needs
    // more registers): the cell searches and all position loads are issued
    // before the first particle is processed
    constexpr int kBatch = P == 3 ? 1 : 2;
    for (uint32_t pb = p0 + tid; pb < p1; pb += kBlock * kBatch) {
        int ub[kBatch];
        uint32_t ob[kBatch][3];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            // searched for every lane (past the end: the last particle) so
            // that the searches of the batch interleave outside any branch
            const uint32_t p = pb + k * kBlock;
            const int u = seg_search_n<kTileCells>(cst, p < p1 ? p : p1 - 1);
            ub[k] = p < p1 ? u : -1;
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            if (ub[k] < 0) continue;
#pragma unroll
            for (int d = 0; d < 3; ++d) ob[k][d] = pos[(int64_t)d * n + pb + k * kBlock];
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            if (ub[k] < 0) continue;
            const uint32_t p = pb + k * kBlock;
            const int u = ub[k];
            const int uc[3] = {u & 7, (u >> 3) & 7, u >> 6};
            int jf[3], jc[3];
            T a[3];
            if (P == 3) {
                T wf[3][3], wc[3][3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const uint32_t o = ob[k][d];
                    // nearest node n0 = fine cell + hi, in LDS coordinates
                    jf[d] = 2 * uc[d] + (int)(o >> 15) + tsc_axis<T>((int)(o & 0x7FFFu), wf[d]) + HLO;
                    if (TWO) {
                        const uint32_t q = ((uint32_t)uc[d] << 16) + o;  // tile-relative, 2^-15 units
                        const uint32_t y = q >> hshift;
                        jc[d] = (int)(y >> kFracBits) + tsc_axis<T>((int)(y & 0x7FFFu), wc[d]) + HLO;
                    }
                }
                a[0] = a[1] = a[2] = T(0);
                if (FINE) {
                    gather3(pf, FS, jf[0], jf[1], jf[2], wf[0], wf[1], wf[2], a[0], a[1], a[2]);
                    a[0] *= scale_f;
                    a[1] *= scale_f;
                    a[2] *= scale_f;
                }
                if (TWO) {
                    T c[3];
                    gather3(pc, CS, jc[0], jc[1], jc[2], wc[0], wc[1], wc[2], c[0], c[1], c[2]);
                    a[0] += scale_c * c[0];
                    a[1] += scale_c * c[1];
                    a[2] += scale_c * c[2];
                }
            } else {
                T wf[3][2], wc[3][2];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const uint32_t o = ob[k][d];
                    const int f = (int)(o & 0x7FFFu);
                    jf[d] = 2 * uc[d] + (int)(o >> 15) + HLO;
                    wf[d][1] = (T)f * inv;
                    wf[d][0] = (T)(32768 - f) * inv;
                    if (TWO) {
                        const uint32_t q = ((uint32_t)uc[d] << 16) + o;  // tile-relative, 2^-15 units
                        const int fc = (int)((q >> hshift) & 0x7FFFu);
                        jc[d] = (int)(q >> (kFracBits + hshift)) + HLO;
                        wc[d][1] = (T)fc * inv;
                        wc[d][0] = (T)(32768 - fc) * inv;
                    }
                }
                a[0] = a[1] = a[2] = T(0);
                if (FINE) {
                    gather(pf, FS, jf[0], jf[1], jf[2], wf[0], wf[1], wf[2], a[0], a[1], a[2]);
                    a[0] *= scale_f;
                    a[1] *= scale_f;
                    a[2] *= scale_f;
                }
                if (TWO) {
                    T c[3];
                    gather(pc, CS, jc[0], jc[1], jc[2], wc[0], wc[1], wc[2], c[0], c[1], c[2]);
                    a[0] += scale_c * c[0];
                    a[1] += scale_c * c[1];
                    a[2] += scale_c * c[2];
                }
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                T *dst = acc + (int64_t)d * n + p;
                *dst = accumulate ? *dst + a[d] : a[d];
            }
        }
    }
}

}  // namespace

// levels: bit 0 the fine level, bit 1 the coarse level (if the context has one)
template <int P, typename T>
void launch_interp_kernel(cube2_ctx *ctx, unsigned blocks, const uint16_t *pos, const uint32_t *cs,
                          int64_t n, const T *phi_f, const T *phi_c, double gm, T *acc,
                          int accumulate, int levels, hipStream_t s) {
    const int nt = ctx->nt;
    const bool fine = (levels & 1) != 0, coarse = ctx->n_levels > 1 && (levels & 2) != 0;
    if (coarse && !fine) {
        const Level &C = ctx->lv[1];
        interp_kernel<true, P, T, false><<<blocks, kBlock, 0, s>>>(
            pos, cs, (int)n, ctx->n_f, nt, nullptr, phi_c, C.n, C.hshift, T(0),
            (T)(gm / ((double)C.H * C.H)), acc, accumulate);
    } else if (coarse) {
        const Level &C = ctx->lv[1];
        auto *k = C.hshift == 2 ? interp_kernel<true, P, T, true, 2> : interp_kernel<true, P, T>;
        k<<<blocks, kBlock, 0, s>>>(pos, cs, (int)n, ctx->n_f, nt, phi_f, phi_c, C.n, C.hshift,
                                    (T)gm, (T)(gm / ((double)C.H * C.H)), acc, accumulate);
    } else {
        interp_kernel<false, P, T><<<blocks, kBlock, 0, s>>>(pos, cs, (int)n, ctx->n_f, nt, phi_f,
                                                             nullptr, 1, 0, (T)gm, T(0), acc,
                                                             accumulate);
    }
}

template <typename T>
int interp_levels(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                  const T *phi_f, const T *phi_c, T *acc, int accumulate, int levels,
                  hipStream_t s) {
    const int nt = ctx->nt;
    const unsigned blocks = (unsigned)(nt * nt * nt);
    const double gm = ctx->cfg.g_newton * ctx->cfg.m_p;
    if (ctx->tsc)
        launch_interp_kernel<3, T>(ctx, blocks, pos, cs, n, phi_f, phi_c, gm, acc, accumulate,
                                   levels, s);
    else
        launch_interp_kernel<2, T>(ctx, blocks, pos, cs, n, phi_f, phi_c, gm, acc, accumulate,
                                   levels, s);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

int launch_interp(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                  const float *phi_f, const float *phi_c, float *acc, int accumulate,
                  hipStream_t s) {
    return interp_levels<float>(ctx, pos, cs, n, phi_f, phi_c, acc, accumulate, 3, s);
}

int launch_interp_levels(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                         const float *phi_f, const float *phi_c, float *acc, int accumulate,
                         int levels, hipStream_t s) {
    return interp_levels<float>(ctx, pos, cs, n, phi_f, phi_c, acc, accumulate, levels, s);
}

int launch_interp64(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                    const double *phi_f, const double *phi_c, double *acc, int accumulate,
                    hipStream_t s) {
    return interp_levels<double>(ctx, pos, cs, n, phi_f, phi_c, acc, accumulate, 3, s);
}

}  // namespace cube2
