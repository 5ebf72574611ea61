// kick.hip -- leapfrog kick and drift on integer positions (section 2.2.3:
// kick after each force, drift; section 2.3: positions and velocities at
// interlaced times, positions as in-cell integers), the re-sort that keeps
// the IOS order, and the FP64 diagnostics used for time-step control
// (section 3.2: the step follows the maximum acceleration and velocity).
//
// v' = v + kick * a and dq = rint(drift * v' * 2^15) are evaluated in FP64
// with separately rounded operations (FMA contraction is switched off in
// these kernels), so the integer displacement and the stored velocity are
// deterministic functions of the FP32 inputs.  A particle whose v' or
// displacement is not finite (a non-finite acceleration or velocity, or a
// displacement beyond 2^62 units) is not moved, and the status word records
// it (cube2_status then returns CUBE2_ENONFINITE).
#include "common.hpp"

namespace cube2 {
namespace {

__global__ __launch_bounds__(kBlock) void kick_drift_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs,
    const float *__restrict__ vel, const float *__restrict__ acc, int n, int nt, int n_f,
    double kick, double drift, uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
    uint16_t *__restrict__ offs, uint32_t *__restrict__ status) {
#pragma clang fp contract(off)
    __shared__ uint32_t cst[kTileCells + 1];
    int tx, ty, tz;
    tile_of_block(blockIdx.x, nt, tx, ty, tz);
    const int tid = threadIdx.x;
    const uint32_t key0 = (uint32_t)((tz * nt + ty) * nt + tx) * kTileCells;
    stage_cell_starts<kBlock>(cst, cs, key0);
    __syncthreads();
    const int64_t span = (int64_t)n_f << kFracBits;
    const int cbase[3] = {tx * kTileIos, ty * kTileIos, tz * kTileIos};
    bool bad = false;
    for (uint32_t p = cst[0] + tid; p < cst[kTileCells]; p += kBlock) {
        const int u = seg_search_n<kTileCells>(cst, p);
        const int uc[3] = {u & 7, (u >> 3) & 7, u >> 6};
        int c[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int64_t i = (int64_t)d * n + p;
            const double kv = kick * (double)acc[i];
            const double v1 = (double)vel[i] + kv;
            double dq = rint((drift * v1) * 32768.0);
            if (!(fabs(dq) < 0x1p62)) {   // also NaN: the particle stays where it is
                dq = 0.0;
                bad = true;
            }
            int64_t q = ((int64_t)(cbase[d] + uc[d]) << 16) + pos[i];
            q = (q + (int64_t)dq) % span;
            if (q < 0) q += span;
            c[d] = (int)(q >> 16);
            offs[i] = (uint16_t)(q & 0xFFFF);
        }
        keys[p] = cell_key(c[0], c[1], c[2], nt);
        vals[p] = p;
    }
    if (bad) atomicOr(status, kStatusNonFinite);
}

constexpr int kRedBlocks = 1024;

// Per-block partial sums in FP64 over a fixed grid-stride partition, then a
// fixed-order tree: the result does not depend on scheduling.
__global__ __launch_bounds__(kBlock) void reduce_partial(const float *__restrict__ vel,
                                                         const float *__restrict__ acc, int n,
                                                         double *__restrict__ part) {
    __shared__ double sh[8][kBlock];
    double r[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        double v2 = 0.0, a2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double v = vel ? (double)vel[(int64_t)d * n + i] : 0.0;
            const double a = (double)acc[(int64_t)d * n + i];
            r[d] += v;
            r[4 + d] += a;
            v2 += v * v;
            a2 += a * a;
        }
        r[3] += v2;
        r[7] = fmax(r[7], sqrt(a2));
    }
    for (int k = 0; k < 8; ++k) sh[k][threadIdx.x] = r[k];
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int k = 0; k < 8; ++k) {
                const double o = sh[k][threadIdx.x + st];
                sh[k][threadIdx.x] = (k == 7) ? fmax(sh[k][threadIdx.x], o) : sh[k][threadIdx.x] + o;
            }
        __syncthreads();
    }
    if (threadIdx.x < 8) part[(int64_t)blockIdx.x * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void reduce_final(const double *__restrict__ part, int nb, double m,
                             double *__restrict__ out) {
    const int k = threadIdx.x;
    if (k >= 8) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double v = part[(int64_t)b * 8 + k];
        s = (k == 7) ? fmax(s, v) : s + v;
    }
    out[k] = (k == 3) ? 0.5 * m * s : (k == 7 ? s : m * s);
}

__global__ void kd_backward(const int32_t *__restrict__ perm, const float *__restrict__ xbo,
                            const float *__restrict__ vbo, int n, float kick, float drift,
                            float *__restrict__ xbi, float *__restrict__ vbi,
                            float *__restrict__ ab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int p = perm[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t o = (int64_t)d * n;
        const float xb = xbo[o + i];
        const float vb = vbo[o + i] + drift * xb;
        xbi[o + p] = xb;
        vbi[o + p] = vb;
        ab[o + p] = kick * vb;
    }
}

}  // namespace

int launch_kick_drift(cube2_ctx *ctx, const uint16_t *pos_in, const uint32_t *cs_in,
                      const float *vel_in, const float *acc, int64_t n64, double kick,
                      double drift, uint16_t *pos_out, uint32_t *cs_out, float *vel_out,
                      int32_t *perm_out, unsigned char *work, const WorkLayout &L,
                      hipStream_t s) {
    const int n = (int)n64;
    const int nt = ctx->nt;
    uint16_t *offs = reinterpret_cast<uint16_t *>(work + L.offs_tmp);
    if (n > 0) {
        kick_drift_kernel<<<(unsigned)(nt * nt * nt), kBlock, 0, s>>>(
            pos_in, cs_in, vel_in, acc, n, nt, ctx->n_f, kick, drift,
            reinterpret_cast<uint32_t *>(work + L.keys), reinterpret_cast<uint32_t *>(work + L.vals),
            offs, status_word(ctx));
        CUBE2_LAUNCH_CHECK();
    }
    // the re-sort's final gather also forms the kicked velocities
    return launch_sort_by_cell(ctx, n, offs, pos_out, cs_out, perm_out, work, L, s, vel_in, acc,
                               kick, vel_out);
}

int launch_reduce(cube2_ctx *ctx, const float *vel, const float *acc, int64_t n64, double *out8,
                  unsigned char *work, const WorkLayout &L, hipStream_t s) {
    const int n = (int)n64;
    double *part = reinterpret_cast<double *>(work + L.red);
    double *dout = part + (size_t)kRedBlocks * 8;
    if (n > 0) {
        reduce_partial<<<kRedBlocks, kBlock, 0, s>>>(vel, acc, n, part);
        CUBE2_LAUNCH_CHECK();
        reduce_final<<<1, 64, 0, s>>>(part, kRedBlocks, ctx->cfg.m_p, dout);
        CUBE2_LAUNCH_CHECK();
        CUBE2_CHECK_HIP(hipMemcpyAsync(out8, dout, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
        CUBE2_CHECK_HIP(hipStreamSynchronize(s));
    } else {
        for (int k = 0; k < 8; ++k) out8[k] = 0.0;
    }
    return CUBE2_OK;
}

int launch_kick_drift_backward(cube2_ctx *ctx, int64_t n, const int32_t *perm,
                               const float *xbar_out, const float *vbar_out, double kick,
                               double drift, float *xbar_in, float *vbar_in, float *acc_bar,
                               hipStream_t s) {
    (void)ctx;
    kd_backward<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(perm, xbar_out, vbar_out, (int)n,
                                                          (float)kick, (float)drift, xbar_in,
                                                          vbar_in, acc_bar);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

}  // namespace cube2
