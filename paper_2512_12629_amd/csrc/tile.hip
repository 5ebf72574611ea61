// tile.hip -- the tile+buffer mode of section 2.2.3 (PM2 paragraph): the
// finer PM level of a tile is computed on a local periodic box made of the
// tile and a buffer zone around it, from the particles of the tile and of the
// buffer; the truncated finer-level force (eq. 4b) vanishes beyond the
// coarse softening, so a buffer of at least b_coarse + 3 H (the truncation
// plus the assignment and finite-difference reach) leaves the tile's own
// particles with every neighbour that acts on them, and the local box's
// periodic images farther away than the truncation.
//
//   launch_tile_gather: the particles of a box of IOS cells [r0, r0 + R)^3
//     (periodic) in a fixed order (region cells z-major, then the particle
//     order inside a cell), as box-unit positions of the local box of n_local
//     = 2R fine cells ((3, m) SoA at the front of x_local), with their global
//     indices;
//   launch_tile_scatter_add: acc[idx] += acc_local for the gathered particles
//     that lie in the tile proper (local fine-cell coordinates in [lo, hi)).
#include "common.hpp"

namespace cube2 {
namespace {

// region cell r (z-major over R^3) -> global IOS cell key
__device__ __forceinline__ uint32_t region_key(int64_t r, int R, int rx0, int ry0, int rz0,
                                               int n_ios, int nt) {
    const int x = (int)(r % R), y = (int)((r / R) % R), z = (int)(r / ((int64_t)R * R));
    return cell_key(wrapn(rx0 + x, n_ios), wrapn(ry0 + y, n_ios), wrapn(rz0 + z, n_ios), nt);
}

__global__ void region_count_kernel(const uint32_t *__restrict__ cs, int R, int rx0, int ry0,
                                    int rz0, int n_ios, int nt, uint32_t *__restrict__ counts) {
    const int64_t R3 = (int64_t)R * R * R;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > R3) return;
    if (r == R3) {
        counts[r] = 0u;   // the scan turns this entry into the total
        return;
    }
    const uint32_t key = region_key(r, R, rx0, ry0, rz0, n_ios, nt);
    counts[r] = cs[key + 1] - cs[key];
}

// One wave per region cell: its particles go to out[offs[r] ...] with local
// positions (rel cells << 16 | offset) / (n_local 2^15), exact in FP32 for
// n_local <= 512.
__global__ __launch_bounds__(kBlock) void region_write_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs, int n, int R, int rx0,
    int ry0, int rz0, int n_ios, int nt, const uint32_t *__restrict__ offs, float inv_span,
    float *__restrict__ x_local, int32_t *__restrict__ idx, int64_t m_max) {
    const int64_t R3 = (int64_t)R * R * R;
    const int64_t r = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (r >= R3) return;
    const int lane = threadIdx.x & 63;
    const uint32_t key = region_key(r, R, rx0, ry0, rz0, n_ios, nt);
    const uint32_t b = cs[key], e = cs[key + 1], o0 = offs[r];
    const int c[3] = {(int)(r % R), (int)((r / R) % R), (int)(r / ((int64_t)R * R))};
    for (uint32_t p = b + (uint32_t)lane; p < e; p += 64) {
        const int64_t o = (int64_t)o0 + (p - b);
        if (o >= m_max) break;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const uint32_t rel = ((uint32_t)c[d] << 16) | (uint32_t)pos[(int64_t)d * n + p];
            x_local[(int64_t)d * m_max + o] = (float)rel * inv_span;
        }
        idx[o] = (int32_t)p;
    }
}

// acc[d][idx[g]] += acc_local[d][i] for local particle i (local sorted order)
// with g = perm_local[i], when its local position lies in [lo, hi)^3 fine cells
__global__ void scatter_add_kernel(int64_t m, const int32_t *__restrict__ perm_local,
                                   const float *__restrict__ x_local,
                                   const int32_t *__restrict__ idx, float lo, float hi,
                                   float span, const float *__restrict__ acc_local,
                                   float *__restrict__ acc, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int64_t g = perm_local[i];
    bool phys = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float f = x_local[d * m + g] * span;   // fine cells, exact
        phys = phys && f >= lo && f < hi;
    }
    if (!phys) return;
    const int64_t j = idx[g];
#pragma unroll
    for (int d = 0; d < 3; ++d) acc[d * n + j] += acc_local[d * m + i];
}

}  // namespace

int launch_tile_gather(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                       const int (&r0)[3], int R, int n_local, float *x_local, int32_t *idx,
                       int64_t m_max, int64_t *m_out, unsigned char *work, const WorkLayout &L,
                       hipStream_t s) {
    const int64_t R3 = (int64_t)R * R * R;
    // per-cell counts, then offsets, in the fine real mesh area (8 entries per IOS cell)
    uint32_t *offs = reinterpret_cast<uint32_t *>(work + L.real_f);
    uint32_t *tmp = reinterpret_cast<uint32_t *>(work + L.scan_tmp);
    region_count_kernel<<<(unsigned)((R3 + 1 + 255) / 256), 256, 0, s>>>(
        cs, R, r0[0], r0[1], r0[2], ctx->n_ios, ctx->nt, offs);
    CUBE2_LAUNCH_CHECK();
    int rc = launch_exclusive_scan(offs, offs, R3 + 1, tmp, s);
    if (rc) return rc;
    uint32_t total = 0;
    CUBE2_CHECK_HIP(hipMemcpyAsync(&total, offs + R3, 4, hipMemcpyDeviceToHost, s));
    CUBE2_CHECK_HIP(hipStreamSynchronize(s));
    *m_out = total;
    if ((int64_t)total > m_max) return CUBE2_EWORKSPACE;
    if (total == 0) return CUBE2_OK;
    const float inv_span = 1.0f / (float)((int64_t)n_local << kFracBits);
    region_write_kernel<<<(unsigned)((R3 + kBlock / 64 - 1) / (kBlock / 64)), kBlock, 0, s>>>(
        pos, cs, (int)n, R, r0[0], r0[1], r0[2], ctx->n_ios, ctx->nt, offs, inv_span, x_local,
        idx, (int64_t)total);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

int launch_tile_scatter_add(int64_t m, const int32_t *perm_local, const float *x_local,
                            const int32_t *idx, int lo, int hi, int n_local,
                            const float *acc_local, float *acc, int64_t n, hipStream_t s) {
    if (m == 0) return CUBE2_OK;
    scatter_add_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(
        m, perm_local, x_local, idx, (float)lo, (float)hi, (float)n_local, acc_local, acc, n);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

}  // namespace cube2
