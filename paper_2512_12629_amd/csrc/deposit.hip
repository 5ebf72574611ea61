// deposit.hip -- CIC mass assignment in exact fixed point (section 2.1.2,
// step 1, with the CIC kernel), both PM levels in one particle sweep.
//
// A particle with 15-bit in-cell fraction f (per axis, on the level's mesh)
// gives node j the weight 2^15 - f and node j+1 the weight f; the product of
// three weights (<= 2^45) is added to a uint64 accumulator.  Integer addition
// is associative, so the result is bit-exact and independent of the order of
// the LDS atomics.  The FP32 density is the accumulator rounded to nearest,
// times 2^-45 (particle masses per level cell).
//
// Fine level: one workgroup owns the 16^3 fine nodes of a tile and gathers
// every particle that touches them: its own 8^3 IOS cells plus the layer of
// IOS cells below it on each axis (a particle in fine cell a-1 feeds node a).
// The contributing cells form a 9^3 box of IOS cells, i.e. 729 contiguous
// particle ranges, flattened by a prefix sum and searched per particle.
// Each fine node is then written once, as FP32: no global atomics and no
// 64-bit mesh in HBM.
// Coarse level: only the tile's own particles are assigned; the tile's
// coarse footprint (16/H + 1 nodes per axis) is accumulated in LDS and added
// to a uint64 coarse mesh with global atomics, then converted to FP32.
#include "common.hpp"

namespace cube2 {
namespace {

constexpr int kBox = kTileIos + 1;            // 9 IOS cells per axis
constexpr int kSegs = kBox * kBox * kBox;     // 729
constexpr int kSegPerThread = (kSegs + kBlock - 1) / kBlock;  // 3
constexpr int kCoarseMax = kTileFine / 2 + 1; // 9 coarse nodes per axis (ratio 2)

__global__ void fill_u64(unsigned long long *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Fine CIC weights of one particle of box segment b (IOS cell coordinates in
// the 9^3 box, own cells at 1..8) with in-cell offsets o, added to the
// tile's fine nodes that it reaches.
__device__ __forceinline__ void deposit_fine(const int (&b)[3], const uint32_t (&o)[3],
                                             unsigned long long *acc_f) {
    int j[3];
    uint32_t w[3][2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        j[d] = 2 * (b[d] - 1) + (int)(o[d] >> 15);  // fine cell rel. to the tile
        const uint32_t f = o[d] & 0x7FFFu;
        w[d][0] = 32768u - f;
        w[d][1] = f;
    }
#pragma unroll
    for (int sz = 0; sz < 2; ++sz)
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
            const int nz = j[2] + sz, ny = j[1] + sy;
            if ((unsigned)nz >= (unsigned)kTileFine || (unsigned)ny >= (unsigned)kTileFine)
                continue;
            const uint32_t wyz = w[1][sy] * w[2][sz];  // <= 2^30
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
                const int nx = j[0] + sx;
                if ((unsigned)nx >= (unsigned)kTileFine) continue;
                atomicAdd(&acc_f[(nz * kTileFine + ny) * kTileFine + nx],
                          (unsigned long long)wyz * w[0][sx]);
            }
        }
}

// Coarse CIC weights of the wave's own-tile particles (own = true), added to
// the tile's coarse footprint.  Called by all 64 lanes.  An IOS cell lies in
// one coarse cell, so in a dense cell every lane feeds the same 8 nodes:
// then the 8 weights are summed over the wave first (exact integer sums) and
// one lane adds them, instead of 64 lanes contending for each node.
__device__ __forceinline__ void deposit_coarse_wave(bool own, const int (&b)[3],
                                                    const uint32_t (&o)[3], int hshift, int NC,
                                                    unsigned long long *acc_c) {
    const unsigned long long om = __ballot(own);
    if (om == 0ull) return;
    int j[3];
    uint32_t w[3][2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const uint32_t q = ((uint32_t)(b[d] - 1) << 16) + o[d];  // tile-relative
        j[d] = (int)(q >> (kFracBits + hshift));
        const uint32_t f = (q >> hshift) & 0x7FFFu;
        w[d][0] = own ? 32768u - f : 0u;
        w[d][1] = own ? f : 0u;
    }
    const int key = own ? (j[2] * NC + j[1]) * NC + j[0] : -1;
    const int lead = first_lane(om);
    const int key0 = __shfl(key, lead, 64);
    const bool uniform = __ballot(own && key != key0) == 0ull;
#pragma unroll
    for (int sz = 0; sz < 2; ++sz)
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
            const uint32_t wyz = w[1][sy] * w[2][sz];
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
                const unsigned long long v = (unsigned long long)wyz * w[0][sx];
                const int off = (sz * NC + sy) * NC + sx;
                if (uniform) {
                    const unsigned long long t = wave_sum(v);
                    if ((int)(threadIdx.x & 63) == lead) atomicAdd(&acc_c[key0 + off], t);
                } else if (own) {
                    atomicAdd(&acc_c[key + off], v);
                }
            }
        }
}

template <bool FINE, bool COARSE>
__global__ __launch_bounds__(kBlock) void deposit_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs, int n, int n_f, int nt,
    float *__restrict__ rho_f, unsigned long long *__restrict__ rho_f_fx,
    unsigned long long *__restrict__ coarse_acc, int n_c, int hshift, uint32_t *status,
    const uint32_t *__restrict__ order, uint32_t *__restrict__ queue) {
    __shared__ uint32_t seg_pre[kSegs + 1];
    __shared__ uint32_t seg_src[kSegs];
    __shared__ unsigned long long acc_f[FINE ? kTileFine * kTileFine * kTileFine : 1];
    __shared__ unsigned long long acc_c[COARSE ? kCoarseMax * kCoarseMax * kCoarseMax : 1];
    __shared__ uint32_t scan_sh[kBlock / 64 + 1];
    __shared__ int tile_sh;

    const int tid = threadIdx.x;
    const int n_ios = nt * kTileIos;
    const int NC = (kTileFine >> hshift) + 1;  // coarse nodes per axis touched by the tile
    int round = 0, tx, ty, tz;
    while (claim_tile(order, queue, nt * nt * nt, nt, round, &tile_sh, tx, ty, tz)) {
        const int c0x = tx * kTileIos, c0y = ty * kTileIos, c0z = tz * kTileIos;

        if (FINE)
            for (int i = tid; i < kTileFine * kTileFine * kTileFine; i += kBlock) acc_f[i] = 0ull;
        if (COARSE)
            for (int i = tid; i < NC * NC * NC; i += kBlock) acc_c[i] = 0ull;

        // particle ranges of the 9^3 box of IOS cells [c0-1, c0+8)
        uint32_t cnt[kSegPerThread], src[kSegPerThread], sum = 0;
#pragma unroll
        for (int k = 0; k < kSegPerThread; ++k) {
            const int s = tid * kSegPerThread + k;
            cnt[k] = 0;
            src[k] = 0;
            if (s < kSegs) {
                const int bx = s % kBox, by = (s / kBox) % kBox, bz = s / (kBox * kBox);
                const bool own = bx > 0 && by > 0 && bz > 0;
                if (FINE || own) {
                    const uint32_t key = cell_key(wrapn(c0x + bx - 1, n_ios), wrapn(c0y + by - 1, n_ios),
                                                  wrapn(c0z + bz - 1, n_ios), nt);
                    src[k] = cs[key];
                    cnt[k] = cs[key + 1] - src[k];
                }
            }
            sum += cnt[k];
        }
        uint32_t total;
        uint32_t pre = block_exclusive_scan(sum, scan_sh, total);
#pragma unroll
        for (int k = 0; k < kSegPerThread; ++k) {
            const int s = tid * kSegPerThread + k;
            if (s < kSegs) {
                seg_pre[s] = pre;
                seg_src[s] = src[k];
            }
            pre += cnt[k];
        }
        if (tid == 0) {
            seg_pre[kSegs] = total;
            // Overflow guard: a fine node sums at most `total` weights of 2^45
            // each; a coarse node sums the own particles of at most 8 tiles.
            const uint32_t key0 = (uint32_t)((tz * nt + ty) * nt + tx) * kTileCells;
            const uint32_t own = cs[key0 + kTileCells] - cs[key0];
            if ((FINE && total >= (1u << 19)) || (COARSE && own >= (1u << 16))) atomicOr(status, 1u);
        }
        __syncthreads();

        // The loop runs wave-uniformly (every lane of a wave takes the same
        // trips) so that the coarse weights can be summed over the wave; each
        // trip takes kBatch particles per lane, whose segment searches and
        // position loads are all issued before the first deposit.
        constexpr int kBatch = 4;
        const int lane = tid & 63;
        for (uint32_t w0 = (uint32_t)(tid - lane); w0 < total; w0 += kBlock * kBatch) {
            int sg[kBatch];
            uint32_t o[kBatch][3];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const uint32_t v = w0 + k * kBlock + lane;
                sg[k] = v < total ? seg_search(seg_pre, kSegs, v) : -1;
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                o[k][0] = o[k][1] = o[k][2] = 0u;
                if (sg[k] < 0) continue;
                const uint32_t p = seg_src[sg[k]] + (w0 + k * kBlock + lane - seg_pre[sg[k]]);
#pragma unroll
                for (int d = 0; d < 3; ++d) o[k][d] = pos[(int64_t)d * n + p];
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const bool valid = sg[k] >= 0;
                const int s = valid ? sg[k] : 0;
                const int b[3] = {s % kBox, (s / kBox) % kBox, s / (kBox * kBox)};
                if (FINE && valid) deposit_fine(b, o[k], acc_f);
                if (COARSE)
                    deposit_coarse_wave(valid && b[0] > 0 && b[1] > 0 && b[2] > 0, b, o[k], hshift, NC,
                                        acc_c);
            }
        }
        __syncthreads();

        if (FINE) {
            const int a0x = tx * kTileFine, a0y = ty * kTileFine, a0z = tz * kTileFine;
            for (int i = tid; i < kTileFine * kTileFine * kTileFine; i += kBlock) {
                const int lx = i % kTileFine, ly = (i / kTileFine) % kTileFine,
                          lz = i / (kTileFine * kTileFine);
                const int64_t g = ((int64_t)(a0z + lz) * n_f + (a0y + ly)) * n_f + (a0x + lx);
                const unsigned long long v = acc_f[i];
                rho_f[g] = (float)v * 0x1p-45f;
                if (rho_f_fx) rho_f_fx[g] = v;
            }
        }
        if (COARSE) {
            const int A0x = (tx * kTileFine) >> hshift, A0y = (ty * kTileFine) >> hshift,
                      A0z = (tz * kTileFine) >> hshift;
            for (int i = tid; i < NC * NC * NC; i += kBlock) {
                const unsigned long long v = acc_c[i];
                if (!v) continue;
                const int lx = i % NC, ly = (i / NC) % NC, lz = i / (NC * NC);
                const int64_t g = ((int64_t)wrapn(A0z + lz, n_c) * n_c + wrapn(A0y + ly, n_c)) * n_c +
                                  wrapn(A0x + lx, n_c);
                atomicAdd(&coarse_acc[g], v);
            }
        }
    }  // tiles
}

__global__ void coarse_finalize(const unsigned long long *__restrict__ accum, int64_t m,
                                float *__restrict__ rho, unsigned long long *__restrict__ fx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const unsigned long long v = accum[i];
    rho[i] = (float)v * 0x1p-45f;
    if (fx) fx[i] = v;
}

}  // namespace

int launch_deposit(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                   float *rho_f, uint64_t *rho_f_fx, float *rho_c, uint64_t *rho_c_fx,
                   unsigned char *work, const WorkLayout &L, hipStream_t s) {
    const int nt = ctx->nt;
    const unsigned blocks = (unsigned)(nt * nt * nt);
    uint32_t *status = status_word(ctx);
    const bool coarse = rho_c != nullptr && ctx->n_levels > 1;
    const bool fine = rho_f != nullptr;
    auto *cacc = reinterpret_cast<unsigned long long *>(work + L.coarse_acc);
    const int n_c = coarse ? ctx->lv[1].n : 1;
    const int hshift = coarse ? ctx->lv[1].hshift : 0;
    const int64_t mc = (int64_t)n_c * n_c * n_c;
    if (coarse) {
        fill_u64<<<(unsigned)((mc + 255) / 256), 256, 0, s>>>(cacc, mc);
        CUBE2_LAUNCH_CHECK();
    }
    auto *ffx = reinterpret_cast<unsigned long long *>(rho_f_fx);
    if (!fine && !coarse) return CUBE2_EINVAL;
    // persistent workgroups over the tiles, heaviest first
    int r = launch_order_tiles(ctx, cs, work, L, s);
    if (r) return r;
    const uint32_t *order = tile_order_ptr(work, L);
    uint32_t *queue = tile_queue_ptr(ctx, work, L);
    const int ntiles = (int)blocks;
    if (fine && coarse)
        deposit_kernel<true, true><<<persistent_grid(deposit_kernel<true, true>, kBlock, ntiles),
                                     kBlock, 0, s>>>(pos, cs, (int)n, ctx->n_f, nt, rho_f, ffx, cacc,
                                                     n_c, hshift, status, order, queue);
    else if (fine)
        deposit_kernel<true, false><<<persistent_grid(deposit_kernel<true, false>, kBlock, ntiles),
                                      kBlock, 0, s>>>(pos, cs, (int)n, ctx->n_f, nt, rho_f, ffx,
                                                      cacc, n_c, hshift, status, order, queue);
    else
        deposit_kernel<false, true><<<persistent_grid(deposit_kernel<false, true>, kBlock, ntiles),
                                      kBlock, 0, s>>>(pos, cs, (int)n, ctx->n_f, nt, nullptr,
                                                      nullptr, cacc, n_c, hshift, status, order,
                                                      queue);
    CUBE2_LAUNCH_CHECK();
    if (coarse) {
        coarse_finalize<<<(unsigned)((mc + 255) / 256), 256, 0, s>>>(
            cacc, mc, rho_c, reinterpret_cast<unsigned long long *>(rho_c_fx));
        CUBE2_LAUNCH_CHECK();
    }
    return CUBE2_OK;
}

}  // namespace cube2
