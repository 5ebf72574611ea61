// fp64.hip -- pieces of the FP64 plain form that have no FP32 twin:
//   * the density in FP64: the deposit's exact uint64 accumulator times its
//     unit (2^-45 for CIC, 2^-48 for TSC);
//   * the PP force (eq. 4d) in FP64, one thread per particle looping over its
//     neighbour IOS cells (27, or 125 for b_f > 2) in HBM, with the pair
//     law of eq. (2) evaluated
//     from the FP64 rows of the same exact piecewise-polynomial table that
//     the FP32 kernel uses (re-expanded on the host in FP64).
// It favours plainness over speed: it is the yardstick the FP32 path is
// compared against at sizes the host oracle cannot reach.
#include "common.hpp"

namespace cube2 {
namespace {

__global__ void fx_to_f64_kernel(uint64_t *buf, int64_t m, double unit) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const double v = (double)buf[i] * unit;
    buf[i] = (uint64_t)__double_as_longlong(v);
}

__global__ __launch_bounds__(kBlock) void pp64_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs, int n, int nt,
    const double *__restrict__ rows, int K, double kinv, double gm, double *__restrict__ acc,
    int accumulate, int reach) {
    __shared__ uint32_t cst[kTileCells + 1];
    int tx, ty, tz;
    tile_of_block(blockIdx.x, nt, tx, ty, tz);
    const int n_ios = nt * kTileIos;
    const uint32_t key0 = (uint32_t)((tz * nt + ty) * nt + tx) * kTileCells;
    for (int i = threadIdx.x; i <= kTileCells; i += kBlock) cst[i] = cs[key0 + i];
    __syncthreads();
    const uint32_t p0 = cst[0], p1 = cst[kTileCells];
    for (uint32_t p = p0 + threadIdx.x; p < p1; p += kBlock) {
        const int u = seg_search_n<kTileCells>(cst, p);
        const int c[3] = {tx * kTileIos + (u & 7), ty * kTileIos + ((u >> 3) & 7),
                          tz * kTileIos + (u >> 6)};
        int oi[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) oi[d] = pos[(int64_t)d * n + p];
        double a[3] = {0.0, 0.0, 0.0};
        for (int dz = -reach; dz <= reach; ++dz)
            for (int dy = -reach; dy <= reach; ++dy)
                for (int dx = -reach; dx <= reach; ++dx) {
                    const uint32_t key = cell_key(wrapn(c[0] + dx, n_ios), wrapn(c[1] + dy, n_ios),
                                                  wrapn(c[2] + dz, n_ios), nt);
                    const uint32_t j0 = cs[key], j1 = cs[key + 1];
                    for (uint32_t j = j0; j < j1; ++j) {
                        // exact separation in units of 2^-15 fine cells (IOS cell = 2^16)
                        const int D[3] = {dx * 65536 + (int)pos[j] - oi[0],
                                          dy * 65536 + (int)pos[(int64_t)n + j] - oi[1],
                                          dz * 65536 + (int)pos[2 * (int64_t)n + j] - oi[2]};
                        const double X = D[0] * 0x1p-15, Y = D[1] * 0x1p-15, Z = D[2] * 0x1p-15;
                        const double r2 = X * X + Y * Y + Z * Z;
                        if (r2 == 0.0) continue;  // the particle itself (or a coincident one)
                        const double r = sqrt(r2);
                        const double t = r * kinv;
                        const int idx = min((int)t, K);
                        const double *q = rows + (int64_t)idx * kPairRow;
                        const double y = q[9] + q[10] * (t - floor(t));
                        double U = q[8];
                        for (int k = 7; k >= 0; --k) U = q[k] + y * U;
                        const double g = U / (r2 * r);
                        a[0] += g * X;
                        a[1] += g * Y;
                        a[2] += g * Z;
                    }
                }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double *dst = acc + (int64_t)d * n + p;
            *dst = accumulate ? *dst + gm * a[d] : gm * a[d];
        }
    }
}

}  // namespace

int launch_fx_to_f64(uint64_t *buf, int64_t m, double unit, hipStream_t s) {
    if (m <= 0) return CUBE2_OK;
    fx_to_f64_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(buf, m, unit);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

int launch_pp64(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n, double *acc,
                int accumulate, hipStream_t s) {
    const double *rows = reinterpret_cast<const double *>(ctx->tables + ctx->pp64_off);
    const int nt = ctx->nt;
    pp64_kernel<<<(unsigned)(nt * nt * nt), kBlock, 0, s>>>(
        pos, cs, (int)n, nt, rows, ctx->pp_K, (double)ctx->pp_K / ctx->cfg.b_fine,
        ctx->cfg.g_newton * ctx->cfg.m_p, acc, accumulate, ctx->pp_halo);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

}  // namespace cube2
