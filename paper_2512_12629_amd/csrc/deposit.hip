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
//
// TSC (eq. 5, context flag CUBE2_ASSIGN_TSC): a particle with in-cell
// fraction f has nearest node n0 = j + [f >= 1/2] and offset m = f - [f >=
// 1/2] (units 2^-15, m in [-2^14, 2^14)); nodes n0-1, n0, n0+1 get the
// 16-bit weights W- = round((2^14 - m)^2 / 2^15), W+ = round((2^14 + m)^2 /
// 2^15) and W0 = 2^16 - W- - W+ (eq. 5 to 2^-16, summing exactly to one
// particle).  Products are below 2^47, the density is the accumulator times
// 2^-48.  A fine node then also receives particles of the next IOS cell up,
// so the gathered box is 10^3 IOS cells; the coarse footprint has 16/H + 3
// nodes per axis.
#include "common.hpp"

namespace cube2 {
namespace {

// Gathered box of IOS cells per axis: [c0-1, c0+8) for CIC, [c0-1, c0+9) for TSC.
// CR: the smallest coarse ratio the LDS coarse footprint is sized for (2, or
// 4 for ratios 4 and 8, which keeps the block within 40 KB of LDS: four
// workgroups per CU).
template <int P, int CR = 4> struct DepGeo {
    static constexpr int BOX = kTileIos + (P == 3 ? 2 : 1);
    static constexpr int SEGS = BOX * BOX * BOX;              // 729 or 1000
    static constexpr int SEG_PER_THREAD = (SEGS + kBlock - 1) / kBlock;
    static constexpr int CMAX = kTileFine / CR + (P == 3 ? 3 : 1);  // coarse nodes per axis
};

// TSC weights of offset m (units 2^-15, m in [-2^14, 2^14)) in units of 2^-16.
__device__ __forceinline__ void tsc_weights(int m, uint32_t (&w)[3]) {
    const uint32_t a = (uint32_t)(16384 - m), b = (uint32_t)(16384 + m);
    w[0] = (a * a + 16384u) >> 15;
    w[2] = (b * b + 16384u) >> 15;
    w[1] = 65536u - w[0] - w[2];
}

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

// Fine TSC weights of one particle of box segment b, added to the tile's
// fine nodes that it reaches (nodes n0-1 .. n0+1 per axis).
__device__ __forceinline__ void deposit_fine_tsc(const int (&b)[3], const uint32_t (&o)[3],
                                                 unsigned long long *acc_f) {
    int j[3];
    uint32_t w[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int f = (int)(o[d] & 0x7FFFu);
        const int hi = f >= 16384 ? 1 : 0;
        j[d] = 2 * (b[d] - 1) + (int)(o[d] >> 15) + hi - 1;  // node n0 - 1, rel. to the tile
        tsc_weights(f - (hi << 15), w[d]);
    }
#pragma unroll
    for (int sz = 0; sz < 3; ++sz)
#pragma unroll
        for (int sy = 0; sy < 3; ++sy) {
            const int nz = j[2] + sz, ny = j[1] + sy;
            if ((unsigned)nz >= (unsigned)kTileFine || (unsigned)ny >= (unsigned)kTileFine)
                continue;
            const uint32_t wyz = w[1][sy] * w[2][sz];  // < 2^32
#pragma unroll
            for (int sx = 0; sx < 3; ++sx) {
                const int nx = j[0] + sx;
                if ((unsigned)nx >= (unsigned)kTileFine) continue;
                atomicAdd(&acc_f[(nz * kTileFine + ny) * kTileFine + nx],
                          (unsigned long long)wyz * w[0][sx]);
            }
        }
}

// Coarse TSC weights of the wave's own-tile particles, added to the tile's
// coarse footprint (LDS index = coarse node - tile origin + 1), wave-summed
// when every own lane shares its nearest node.
__device__ __forceinline__ void deposit_coarse_wave_tsc(bool own, const int (&b)[3],
                                                        const uint32_t (&o)[3], int hshift, int NC,
                                                        unsigned long long *acc_c) {
    const unsigned long long om = __ballot(own);
    if (om == 0ull) return;
    int j[3];
    uint32_t w[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const uint32_t q = ((uint32_t)(b[d] - 1) << 16) + o[d];  // tile-relative
        const uint32_t y = q >> hshift;                           // 2^-15 coarse cells
        const int f = (int)(y & 0x7FFFu);
        const int hi = f >= 16384 ? 1 : 0;
        j[d] = (int)(y >> kFracBits) + hi;                        // n0, LDS index of n0 - 1
        tsc_weights(f - (hi << 15), w[d]);
        if (!own) w[d][0] = w[d][1] = w[d][2] = 0u;
    }
    const int key = own ? (j[2] * NC + j[1]) * NC + j[0] : -1;
    const int lead = first_lane(om);
    const int key0 = __builtin_amdgcn_readlane(key, lead);
    const bool uniform = __ballot(own && key != key0) == 0ull;
#pragma unroll
    for (int sz = 0; sz < 3; ++sz)
#pragma unroll
        for (int sy = 0; sy < 3; ++sy) {
            const uint32_t wyz = w[1][sy] * w[2][sz];
#pragma unroll
            for (int sx = 0; sx < 3; ++sx) {
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
    const int key0 = __builtin_amdgcn_readlane(key, lead);
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

template <bool FINE, bool COARSE, int P, int CR>
__global__ __launch_bounds__(kBlock) void deposit_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs, int n, int n_f, int nt,
    float *__restrict__ rho_f, unsigned long long *__restrict__ rho_f_fx,
    unsigned long long *__restrict__ coarse_acc, int n_c, int hshift, uint32_t *status,
    const uint32_t *__restrict__ order, uint32_t *__restrict__ queue) {
    using Geo = DepGeo<P, CR>;
    constexpr int kBox = Geo::BOX, kSegs = Geo::SEGS;
    constexpr int kSegPerThread = Geo::SEG_PER_THREAD, kCoarseMax = Geo::CMAX;
    __shared__ uint32_t seg_pre[kSegs + 1];
    __shared__ uint32_t seg_src[kSegs];
    __shared__ unsigned long long acc_f[FINE ? kTileFine * kTileFine * kTileFine : 1];
    __shared__ unsigned long long acc_c[COARSE ? kCoarseMax * kCoarseMax * kCoarseMax : 1];
    __shared__ uint32_t scan_sh[kBlock / 64 + 1];
    __shared__ int next_sh;

    const int tid = threadIdx.x;
    const int n_ios = nt * kTileIos;
    const int NC = (kTileFine >> hshift) + (P == 3 ? 3 : 1);  // coarse nodes per axis touched
    const int ntiles = nt * nt * nt;

    // Particle ranges (start, count) of this thread's segments of the box of
    // IOS cells [c0-1, c0+kBox-1) around tile t.
    uint32_t cnt[kSegPerThread], src[kSegPerThread];
    auto load_segments = [&](int t) {
        const int c0x = (t % nt) * kTileIos, c0y = ((t / nt) % nt) * kTileIos,
                  c0z = (t / (nt * nt)) * kTileIos;
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
                    cnt[k] = cs[key + 1];  // end; the count is formed where it is used
                }
            }
        }
    };

    // Persistent workgroups over the heaviest-first tile order.  The loop is
    // software-pipelined: the claim of the next tile is in flight while the
    // current one deposits, and the next tile's segment ranges are loaded
    // while the current one writes its nodes.
    if (tid == 0) {
        const int slot = claim_slot(queue, ntiles);
        next_sh = slot < ntiles ? (int)order[slot] : -1;
    }
    __syncthreads();
    int t = next_sh;
    if (t >= 0) load_segments(t);
    while (t >= 0) {
        const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
        int slot = ntiles;
        if (tid == 0) slot = claim_slot(queue, ntiles);

        if (FINE)
            for (int i = tid; i < kTileFine * kTileFine * kTileFine; i += kBlock) acc_f[i] = 0ull;
        if (COARSE)
            for (int i = tid; i < NC * NC * NC; i += kBlock) acc_c[i] = 0ull;

        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kSegPerThread; ++k) {
            cnt[k] -= src[k];
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
        if (tid == 0) seg_pre[kSegs] = total;
        __syncthreads();
        if (tid == 0) {
            // Overflow guard: a fine node sums at most `total` weights of 2^45
            // (CIC) or 2^47 (TSC) each; a coarse node sums the own particles
            // of at most 8 tiles.  The own cells' particles are one contiguous
            // range, from the first own segment to the end of the last.
            const int s_first = (1 * kBox + 1) * kBox + 1;
            const int s_last = (kTileIos * kBox + kTileIos) * kBox + kTileIos;
            const uint32_t own =
                seg_src[s_last] + (seg_pre[s_last + 1] - seg_pre[s_last]) - seg_src[s_first];
            const uint32_t fine_max = P == 3 ? (1u << 17) : (1u << 19);
            const uint32_t own_max = P == 3 ? (1u << 14) : (1u << 16);
            if ((FINE && total >= fine_max) || (COARSE && own >= own_max)) atomicOr(status, kStatusOverflow);
        }

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
                // searched for every lane (a lane past the end searches for the
                // last particle, total >= 1 here), so that the kBatch searches
                // interleave their LDS reads outside any branch
                const uint32_t v = w0 + k * kBlock + lane;
                const int u = seg_search_n<kSegs>(seg_pre, v < total ? v : total - 1);
                sg[k] = v < total ? u : -1;
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
                const bool own = valid && b[0] > 0 && b[1] > 0 && b[2] > 0 && b[0] <= kTileIos &&
                                 b[1] <= kTileIos && b[2] <= kTileIos;
                if (P == 3) {
                    if (FINE && valid) deposit_fine_tsc(b, o[k], acc_f);
                    if (COARSE) deposit_coarse_wave_tsc(own, b, o[k], hshift, NC, acc_c);
                } else {
                    if (FINE && valid) deposit_fine(b, o[k], acc_f);
                    if (COARSE) deposit_coarse_wave(own, b, o[k], hshift, NC, acc_c);
                }
            }
        }
        // the next tile (the claim made at the top of this one has returned)
        if (tid == 0) next_sh = slot < ntiles ? (int)order[slot] : -1;
        __syncthreads();
        const int t_next = next_sh;
        if (t_next >= 0) load_segments(t_next);

        if (FINE) {
            const int a0x = tx * kTileFine, a0y = ty * kTileFine, a0z = tz * kTileFine;
            for (int i = tid; i < kTileFine * kTileFine * kTileFine; i += kBlock) {
                const int lx = i % kTileFine, ly = (i / kTileFine) % kTileFine,
                          lz = i / (kTileFine * kTileFine);
                const int64_t g = ((int64_t)(a0z + lz) * n_f + (a0y + ly)) * n_f + (a0x + lx);
                const unsigned long long v = acc_f[i];
                // streaming store: a tile row is half a cache line, and the
                // mesh is read back only by the next kernel
                __builtin_nontemporal_store((float)v * (P == 3 ? 0x1p-48f : 0x1p-45f), &rho_f[g]);
                if (rho_f_fx) rho_f_fx[g] = v;
            }
        }
        if (COARSE) {
            const int lo = P == 3 ? 1 : 0;  // footprint starts one node below (TSC)
            const int A0x = ((tx * kTileFine) >> hshift) - lo, A0y = ((ty * kTileFine) >> hshift) - lo,
                      A0z = ((tz * kTileFine) >> hshift) - lo;
            for (int i = tid; i < NC * NC * NC; i += kBlock) {
                const unsigned long long v = acc_c[i];
                if (!v) continue;
                const int lx = i % NC, ly = (i / NC) % NC, lz = i / (NC * NC);
                const int64_t g = ((int64_t)wrapn(A0z + lz, n_c) * n_c + wrapn(A0y + ly, n_c)) * n_c +
                                  wrapn(A0x + lx, n_c);
                atomicAdd(&coarse_acc[g], v);
            }
        }
        t = t_next;
        __syncthreads();  // this tile is done with the LDS arrays
    }  // tiles
}

__global__ void coarse_finalize(const unsigned long long *__restrict__ accum, int64_t m,
                                float *__restrict__ rho, unsigned long long *__restrict__ fx,
                                float unit) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const unsigned long long v = accum[i];
    rho[i] = (float)v * unit;
    if (fx) fx[i] = v;
}

template <bool FINE, bool COARSE, int P, int CR>
void launch_one_deposit(const uint16_t *pos, const uint32_t *cs, int64_t n, int n_f, int nt,
                        float *rho_f, unsigned long long *ffx, unsigned long long *cacc, int n_c,
                        int hshift, uint32_t *status, const uint32_t *order, uint32_t *queue,
                        int ntiles, hipStream_t s) {
    auto k = deposit_kernel<FINE, COARSE, P, CR>;
    k<<<persistent_grid(k, kBlock, ntiles), kBlock, 0, s>>>(pos, cs, (int)n, n_f, nt, rho_f, ffx, cacc,
                                                          n_c, hshift, status, order, queue);
}

template <int P>
int launch_deposit_kernels(bool fine, bool coarse, const uint16_t *pos, const uint32_t *cs, int64_t n,
                           int n_f, int nt, float *rho_f, unsigned long long *ffx,
                           unsigned long long *cacc, int n_c, int hshift, uint32_t *status,
                           const uint32_t *order, uint32_t *queue, int ntiles, hipStream_t s) {
    if (coarse && (kTileFine >> hshift) + (P == 3 ? 3 : 1) > DepGeo<P, 2>::CMAX) return CUBE2_EINVAL;
    const bool r2 = hshift < 2;  // coarse ratio 2: the wider footprint
    if (fine && coarse) {
        if (r2)
            launch_one_deposit<true, true, P, 2>(pos, cs, n, n_f, nt, rho_f, ffx, cacc, n_c, hshift,
                                                 status, order, queue, ntiles, s);
        else
            launch_one_deposit<true, true, P, 4>(pos, cs, n, n_f, nt, rho_f, ffx, cacc, n_c, hshift,
                                                 status, order, queue, ntiles, s);
    } else if (fine) {
        launch_one_deposit<true, false, P, 4>(pos, cs, n, n_f, nt, rho_f, ffx, cacc, n_c, hshift,
                                              status, order, queue, ntiles, s);
    } else {
        if (r2)
            launch_one_deposit<false, true, P, 2>(pos, cs, n, n_f, nt, nullptr, nullptr, cacc, n_c,
                                                  hshift, status, order, queue, ntiles, s);
        else
            launch_one_deposit<false, true, P, 4>(pos, cs, n, n_f, nt, nullptr, nullptr, cacc, n_c,
                                                  hshift, status, order, queue, ntiles, s);
    }
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
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
    if (ctx->tsc)
        r = launch_deposit_kernels<3>(fine, coarse, pos, cs, n, ctx->n_f, nt, rho_f, ffx, cacc, n_c,
                                      hshift, status, order, queue, ntiles, s);
    else
        r = launch_deposit_kernels<2>(fine, coarse, pos, cs, n, ctx->n_f, nt, rho_f, ffx, cacc, n_c,
                                      hshift, status, order, queue, ntiles, s);
    if (r) return r;
    if (coarse) {
        coarse_finalize<<<(unsigned)((mc + 255) / 256), 256, 0, s>>>(
            cacc, mc, rho_c, reinterpret_cast<unsigned long long *>(rho_c_fx),
            ctx->tsc ? 0x1p-48f : 0x1p-45f);
        CUBE2_LAUNCH_CHECK();
    }
    return CUBE2_OK;
}

}  // namespace cube2
