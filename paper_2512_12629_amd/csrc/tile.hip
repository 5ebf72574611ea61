// tile.hip -- local boxes of tiles (section 2.2.3): the tile+buffer mode of
// the PM2 paragraph (the finer PM level of a tile computed on a local
// periodic box made of the tile and a buffer zone around it), and the
// subtile boxes of the PM3 level (the same gather, several tiles packed into
// one box).  The truncated level's force vanishes beyond its truncation, so
// a buffer of at least the truncation plus the assignment and
// finite-difference reach (3 mesh cells) leaves the tile's own particles
// with every neighbour that acts on them, and the box's periodic images and
// the other slots' particles beyond the truncation.
//
//   launch_tile_gather: for T tiles (origins in fine cells), the particles of
//     each tile's box of IOS cells [r0_t, r0_t + R)^3 (periodic), in a fixed
//     order (tile by tile; region cells z-major, x fastest; then the particle
//     order inside a cell), placed in slot t of a k^3 grid of slots of 2R
//     fine cells (k the smallest power of two with k^3 >= T), as box-unit
//     positions of the packed box of n_box = 2Rk fine cells ((3, m) SoA at the
//     front of x_local), with their global indices;
//   launch_tile_scatter_add: acc[idx] += scale acc_local for the gathered
//     particles whose slot-relative position lies in [lo, hi)^3 fine cells.
#include "common.hpp"

namespace cube2 {
namespace {

struct Region {
    int R, k, n_ios, nt;
    const int32_t *r0;   // device: 3 T origin IOS cells (x, y, z per tile)
};

// region cell r (tile t = r / R^3, then z-major over R^3) -> global IOS cell
// key, tile-local cell coordinates and the tile index
__device__ __forceinline__ uint32_t region_key(int64_t r, const Region &g, int (&c)[3], int &t) {
    const int64_t R3 = (int64_t)g.R * g.R * g.R;
    t = (int)(r / R3);
    const int64_t l = r - (int64_t)t * R3;
    c[0] = (int)(l % g.R);
    c[1] = (int)((l / g.R) % g.R);
    c[2] = (int)(l / ((int64_t)g.R * g.R));
    const int32_t *o = g.r0 + 3 * t;
    return cell_key(wrapn(o[0] + c[0], g.n_ios), wrapn(o[1] + c[1], g.n_ios),
                    wrapn(o[2] + c[2], g.n_ios), g.nt);
}

__global__ void region_count_kernel(const uint32_t *__restrict__ cs, Region g, int64_t cells,
                                    uint32_t *__restrict__ counts) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > cells) return;
    if (r == cells) {
        counts[r] = 0u;   // the scan turns this entry into the total
        return;
    }
    int c[3], t;
    const uint32_t key = region_key(r, g, c, t);
    counts[r] = cs[key + 1] - cs[key];
}

// One wave per region cell: its particles go to out[offs[r] ...] with the
// positions of their slot, (slot R + cell) << 16 | offset, over n_box 2^15,
// exact in FP32 for n_box <= 512.
__global__ __launch_bounds__(kBlock) void region_write_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs, int n, Region g,
    int64_t cells, const uint32_t *__restrict__ offs, float inv_span, float *__restrict__ x_local,
    int32_t *__restrict__ idx, int64_t m) {
    const int64_t r = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (r >= cells) return;
    const int lane = threadIdx.x & 63;
    int c[3], t;
    const uint32_t key = region_key(r, g, c, t);
    const int sl[3] = {t % g.k, (t / g.k) % g.k, t / (g.k * g.k)};
    const uint32_t b = cs[key], e = cs[key + 1], o0 = offs[r];
    for (uint32_t p = b + (uint32_t)lane; p < e; p += 64) {
        const int64_t o = (int64_t)o0 + (p - b);
        if (o >= m) break;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const uint32_t cell = (uint32_t)(sl[d] * g.R + c[d]);
            const uint32_t rel = (cell << 16) | (uint32_t)pos[(int64_t)d * n + p];
            x_local[(int64_t)d * m + o] = (float)rel * inv_span;
        }
        idx[o] = (int32_t)p;
    }
}

// acc[d][idx[g]] += scale acc_local[d][i] for local particle i (local sorted
// order) with g = perm_local[i], when its position within its slot lies in
// [lo, hi)^3 fine cells
__global__ void scatter_add_kernel(int64_t m, const int32_t *__restrict__ perm_local,
                                   const float *__restrict__ x_local,
                                   const int32_t *__restrict__ idx, float lo, float hi,
                                   float n_box, float n_slot, float scale,
                                   const float *__restrict__ acc_local, float *__restrict__ acc,
                                   int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int64_t gi = perm_local[i];
    bool own = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float f = x_local[d * m + gi] * n_box;            // fine cells, exact
        const float fs = f - floorf(f / n_slot) * n_slot;        // within the slot, exact
        own = own && fs >= lo && fs < hi;
    }
    if (!own) return;
    const int64_t j = idx[gi];
#pragma unroll
    for (int d = 0; d < 3; ++d) acc[d * n + j] += scale * acc_local[d * m + i];
}

}  // namespace

int tile_slots(int T) {
    int k = 1;
    while ((int64_t)k * k * k < T) k <<= 1;
    return k;
}

int launch_tile_gather(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                       const int32_t *r0_host, int T, int R, float *x_local, int32_t *idx,
                       int64_t m_max, int64_t *m_out, unsigned char *work, const WorkLayout &L,
                       hipStream_t s) {
    const int64_t cells = (int64_t)T * R * R * R;
    // per-cell counts, then offsets, in the fine real mesh area; the tile
    // origins in the reduction area
    uint32_t *offs = reinterpret_cast<uint32_t *>(work + L.real_f);
    uint32_t *tmp = reinterpret_cast<uint32_t *>(work + L.scan_tmp);
    int32_t *r0 = reinterpret_cast<int32_t *>(work + L.red);
    CUBE2_CHECK_HIP(hipMemcpyAsync(r0, r0_host, (size_t)T * 3 * sizeof(int32_t),
                                   hipMemcpyHostToDevice, s));
    const int k = tile_slots(T);
    const Region g{R, k, ctx->n_ios, ctx->nt, r0};
    region_count_kernel<<<(unsigned)((cells + 1 + 255) / 256), 256, 0, s>>>(cs, g, cells, offs);
    CUBE2_LAUNCH_CHECK();
    int rc = launch_exclusive_scan(offs, offs, cells + 1, tmp, s);
    if (rc) return rc;
    uint32_t total = 0;
    CUBE2_CHECK_HIP(hipMemcpyAsync(&total, offs + cells, 4, hipMemcpyDeviceToHost, s));
    CUBE2_CHECK_HIP(hipStreamSynchronize(s));
    *m_out = total;
    if ((int64_t)total > m_max) return CUBE2_EWORKSPACE;
    if (total == 0) return CUBE2_OK;
    const int64_t n_box = (int64_t)2 * R * k;
    const float inv_span = 1.0f / (float)(n_box << kFracBits);
    region_write_kernel<<<(unsigned)((cells + kBlock / 64 - 1) / (kBlock / 64)), kBlock, 0, s>>>(
        pos, cs, (int)n, g, cells, offs, inv_span, x_local, idx, (int64_t)total);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

int launch_tile_scatter_add(int64_t m, const int32_t *perm_local, const float *x_local,
                            const int32_t *idx, int T, int lo, int hi, int n_slot, float scale,
                            const float *acc_local, float *acc, int64_t n, hipStream_t s) {
    if (m == 0) return CUBE2_OK;
    const int k = tile_slots(T);
    scatter_add_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(
        m, perm_local, x_local, idx, (float)lo, (float)hi, (float)(n_slot * k), (float)n_slot,
        scale, acc_local, acc, n);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

}  // namespace cube2
