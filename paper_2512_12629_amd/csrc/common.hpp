// common.hpp -- shared definitions of the gfx950 CUBE2 force library.
//
// Geometry used by every kernel:
//   * fine mesh: n_f cells per side, positions q in units of 2^-15 fine cells;
//   * IOS cells of 2x2x2 fine cells (n_ios = n_f/2 per side), the unit of the
//     particle order; tiles of 8^3 IOS cells (16^3 fine cells) group them;
//   * key of IOS cell c = tile index * 512 + cell-in-tile index, both x fastest.
// Every particle-side kernel runs one workgroup per tile: the tile's particles
// are the contiguous range cell_start[key0] .. cell_start[key0 + 512].
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/cube2.h"

namespace cube2 {

constexpr int kFracBits = 15;     // in-cell fraction of a fine cell
constexpr int kTileIos = 8;       // IOS cells per tile side
constexpr int kTileFine = 16;     // fine cells per tile side
constexpr int kTileCells = 512;   // IOS cells per tile
constexpr int kBlock = 256;       // threads of the particle-side kernels

struct Level {
    int n = 0;          // cells per side
    int H = 1;          // spacing in fine cells
    int hshift = 0;     // log2(H)
    int pitch = 0;      // complex row pitch of the half spectrum
    double b_a = 0;     // softening of the level (fine cells)
    double b_prev = 0;  // truncation (fine cells); <= 0 means infinity
    size_t tw_off = 0;  // byte offset of the twiddle table in `tables`
    size_t g_off = 0;   // byte offset of the octant Green's table
    size_t gz_off = 0;  // the same values in the z pass's order (FP32, see fft.hip)
    size_t tw64_off = 0, g64_off = 0;  // FP64 copies (CUBE2_FP64_FORM only)
};

}  // namespace cube2

namespace cube2 {
// Pair-law table of the PP kernels (built on the host, see pp.hip).
constexpr int kPairKMax = 128;     // grid intervals of [0, b_f)
constexpr int kPairRow = 12;       // floats per interval: 9 coefficients, y map, pad
// FP32 forward pair law, indexed by s = r^2: one row of 4 cubic coefficients
// per 1/16 of an octave, for s in [2^-31, 2^7).  The row of s is its float
// bit pattern shifted right by 19 (exponent and top 4 mantissa bits) minus
// kSRow0.
constexpr int kSMantBits = 4;
constexpr int kSRow0 = (127 - 31) << kSMantBits;
constexpr int kSRows = (7 + 31) << kSMantBits;  // 608
}  // namespace cube2

struct cube2_ctx {
    cube2_config cfg;
    int pp_K = 0;                      // intervals of the pair-law grid
    float pp_kinv = 0.f;               // K / b_f
    float pp_negc = 0.f;               // -1/b_f^2, rounded away from zero (FP32 pair law)
    int pp_halo = 1;                   // PP neighbour reach in IOS cells: 1 (b_f <= 2), 2 (b_f <= 4)
    std::vector<float> pp_srows;       // kSRows * 4 floats: the FP32 forward pair law by s = r^2
    size_t pp_soff = 0;                // byte offset of pp_srows in `tables`
    std::vector<double> pp_rows64;     // the same rows in FP64
    size_t pp64_off = 0;               // FP64 rows (CUBE2_FP64_FORM only)
    bool fp64 = false;                 // CUBE2_FP64_FORM
    bool tsc = false;                  // CUBE2_ASSIGN_TSC: TSC instead of CIC on every PM level
    bool isolated = false;             // CUBE2_ISOLATED: isolated boundaries (appendix A)
    int n_f = 0, n_ios = 0, nt = 0;   // fine cells, IOS cells, tiles per side
    int64_t n_cells = 0;               // IOS cells
    int n_levels = 1;                  // 1 or 2; level 0 = fine, 1 = coarse
    cube2::Level lv[2];
    size_t table_bytes = 0;
    unsigned char *tables = nullptr;   // device; set by cube2_init_tables
    hipStream_t side = nullptr;        // cube2_force's PP stream (default priority), made by cube2_init_tables
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // the PM adjoint's second stream (default priority) and its fork/join
    // events: the cotangent scatter beside the recomputed forward potentials
    hipStream_t side2 = nullptr;
    hipEvent_t ev_fork2 = nullptr, ev_join2 = nullptr;
};

namespace cube2 {

// Byte layout of the work buffer for n particles.
struct WorkLayout {
    size_t real_f, real_c, bar_f, bar_c, spec, coarse_acc;
    size_t real64_f, real64_c, spec64;  // FP64 form (zero-sized without it)
    size_t keys, vals, keys2, vals2, hist, scan_tmp, offs_tmp, red;
    size_t pp_order, pp_hist, pp_scan, acc_pp;  // cube2_force's concurrent PP: own tile queue, output
    size_t tile_order;  // 4 x (tiles) + 64 uint32: PP tile order, its sort buffers, work counter
    size_t vel_tmax;    // velocity codec: one FP32 maximum per tile
    size_t total;
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

WorkLayout work_layout(const cube2_ctx *ctx, int64_t n);

// bits of the device status word
constexpr uint32_t kStatusOverflow = 1u;    // a deposit or codec accumulator could overflow
constexpr uint32_t kStatusNonFinite = 2u;   // a kick-drift met a non-finite velocity or step

inline uint32_t *status_word(const cube2_ctx *ctx) {
    return reinterpret_cast<uint32_t *>(ctx->tables);
}

// ---- device helpers ------------------------------------------------------

__device__ __forceinline__ uint32_t cell_key(int cx, int cy, int cz, int nt) {
    int tx = cx >> 3, ty = cy >> 3, tz = cz >> 3;
    int ux = cx & 7, uy = cy & 7, uz = cz & 7;
    return (uint32_t)(((tz * nt + ty) * nt + tx) * kTileCells + (uz * 8 + uy) * 8 + ux);
}

// Tile coordinates of workgroup b.  Blocks are dealt to the 8 XCDs round
// robin; this mapping gives each XCD a contiguous slab of tiles so that the
// halos shared between neighbouring tiles stay in one L2.
__device__ __forceinline__ void tile_of_block(int b, int nt, int &tx, int &ty, int &tz) {
    int ntiles = nt * nt * nt;
    int t = b;
    if ((ntiles & 7) == 0) t = (b & 7) * (ntiles >> 3) + (b >> 3);
    tx = t % nt;
    ty = (t / nt) % nt;
    tz = t / (nt * nt);
}

// TSC weights (eq. 5, 16-bit fixed point as the deposit) of the 15-bit
// fraction f of one axis: nearest-node shift hi and the three weights.
template <typename T>
__device__ __forceinline__ int tsc_axis(int f, T (&w)[3]) {
    const int hi = f >= 16384 ? 1 : 0;
    const int m = f - (hi << 15);
    const uint32_t a = (uint32_t)(16384 - m), b = (uint32_t)(16384 + m);
    const uint32_t w0 = (a * a + 16384u) >> 15, w2 = (b * b + 16384u) >> 15;
    const T inv = T(1.0 / 65536.0);
    w[0] = (T)w0 * inv;
    w[2] = (T)w2 * inv;
    w[1] = (T)(65536u - w0 - w2) * inv;
    return hi;
}

// The same weights with their derivatives in the particle coordinate (level
// units): d = m 2^-15 is the offset from the nearest node, and the slopes of
// eq. 5 at the three nodes are -(1/2 - d), -2d and 1/2 + d.
template <typename T>
__device__ __forceinline__ int tsc_axis_grad(int f, T (&w)[3], T (&dw)[3]) {
    const int hi = tsc_axis<T>(f, w);
    const T d = (T)(f - (hi << 15)) * T(1.0 / 32768.0);
    dw[0] = -(T(0.5) - d);
    dw[1] = T(-2) * d;
    dw[2] = T(0.5) + d;
    return hi;
}

__device__ __forceinline__ int wrapn(int i, int n) {  // n is a power of two
    return i & (n - 1);
}

// Largest s in [0, cnt) with pre[s] <= v (pre nondecreasing, pre[0] <= v).
__device__ __forceinline__ int seg_search(const uint32_t *pre, int cnt, uint32_t v) {
    int lo = 0, hi = cnt;  // invariant: pre[lo] <= v, answer in [lo, hi)
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// The same index for a count known at compile time: the last u in [0, CNT)
// with pre[u] <= v, found bit by bit from the highest power of two below
// CNT (pre non-decreasing, so pre[u] <= v holds exactly up to the answer).
// Unrolled and branch-free: no loop control, and the LDS reads of
// independent searches in one thread interleave.  When CNT is not a power
// of two, pre must hold CNT + 1 entries with pre[CNT] > v (the end of the
// last segment): a candidate at or beyond CNT reads pre[CNT] instead, which
// fails the test, so no step needs a branch.
template <int CNT>
__device__ __forceinline__ int seg_search_n(const uint32_t *pre, uint32_t v) {
    static_assert(CNT >= 1, "empty range");
    constexpr int TOP = [] {
        int t = 1;
        while (2 * t < CNT) t *= 2;
        return CNT > 1 ? t : 0;
    }();
    int lo = 0;
#pragma unroll
    for (int step = TOP; step > 0; step >>= 1) {
        const int c = lo + step;
        if (2 * TOP - step < CNT) {   // c < CNT whatever steps were taken (folds once unrolled)
            if (pre[c] <= v) lo = c;
        } else {
            if (pre[c < CNT ? c : CNT] <= v) lo = c;
        }
    }
    return lo;
}

// Block-wide exclusive scan of one uint32 per thread (blockDim == BLOCK).
template <int BLOCK = kBlock>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh /*BLOCK/64+1*/,
                                                         uint32_t &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) {
        uint32_t s = sh[w];
        if (w < wid) off += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

// Tile scheduling of the per-tile kernels.  With a work queue (queue != 0)
// the workgroups are persistent: each takes the next tile of the
// heaviest-first order (launch_order_tiles) from one global counter until the
// order is exhausted.  Without a queue, workgroup b takes the tile
// tile_of_block(b) once.  claim_tile is called by all threads of the
// workgroup and returns false when the workgroup is done (a block-uniform
// result).

// One claim on the work counter (a single thread calls it): the position in
// `order` of the next tile, or a value >= ntiles when all are taken.
__device__ __forceinline__ int claim_slot(uint32_t *queue, int ntiles) {
    const uint32_t v = atomicAdd(queue, 1u);
    return v < (uint32_t)ntiles ? (int)v : ntiles;
}

__device__ __forceinline__ bool claim_tile(const uint32_t *order, uint32_t *queue, int ntiles,
                                          int nt, int &round, int *tile_sh, int &tx, int &ty,
                                          int &tz) {
    if (queue) {
        __syncthreads();  // the previous tile is done with the LDS arrays
        if (threadIdx.x == 0) *tile_sh = claim_slot(queue, ntiles);
        __syncthreads();
        const int ti = *tile_sh;
        if (ti >= ntiles) return false;
        const int t = (int)order[ti];
        tx = t % nt;
        ty = (t / nt) % nt;
        tz = t / (nt * nt);
    } else {
        if (round > 0) return false;
        tile_of_block(blockIdx.x, nt, tx, ty, tz);
    }
    ++round;
    return true;
}

// Sums over the 64 lanes of a wave (butterfly; every lane must be active).
// The order of the additions is fixed, so float sums are deterministic.
// One DPP lane permutation within rows of 16 lanes, applied to both halves
// of a 64-bit value.
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((unsigned long long)hi << 32) | lo;
}

// Sum of a 64-bit integer over the 64 lanes of a wave (every lane active),
// returned to every lane.  Within each row of 16 lanes, DPP butterflies
// (quad_perm [1,0,3,2] and [2,3,0,1], then the half-row and row mirrors)
// leave the row's sum in all its lanes; the four row sums are then read from
// lanes 0, 16, 32 and 48.  No LDS traffic; the integer sum is exact, so its
// order does not matter.
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    v += dpp_u64<0xB1>(v);
    v += dpp_u64<0x4E>(v);
    v += dpp_u64<0x141>(v);
    v += dpp_u64<0x140>(v);
    const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    unsigned long long s = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        s += ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)hi, 16 * r) << 32) |
             (uint32_t)__builtin_amdgcn_readlane((int)lo, 16 * r);
    return s;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Lane of the first set bit of a nonzero wave mask.
__device__ __forceinline__ int first_lane(unsigned long long mask) {
    return __ffsll((long long)mask) - 1;
}

// The kTileCells + 1 particle starts of one tile (cs[key0 .. key0 + 512])
// into LDS, every load of a thread issued before its LDS stores.
template <int BLOCK>
__device__ __forceinline__ void stage_cell_starts(uint32_t *__restrict__ dst,
                                                  const uint32_t *__restrict__ cs, uint32_t key0) {
    constexpr int PER = (kTileCells + 1 + BLOCK - 1) / BLOCK;
    uint32_t v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {  // unconditional loads (clamped index)
        const int i = (int)threadIdx.x + k * BLOCK;
        v[k] = cs[key0 + (i <= kTileCells ? i : kTileCells)];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = (int)threadIdx.x + k * BLOCK;
        if (i <= kTileCells) dst[i] = v[k];
    }
}


// Copy the periodic S^3 block of an n^3 mesh starting at node (x0, y0, z0)
// (wrapped) into LDS, x fastest.  Each wave copies 64/S whole x-rows per pass
// (lane -> (row, x) fixed for the whole copy, so a row is one contiguous
// read), the row's (y, z) is advanced incrementally, and the loads of one
// thread are issued in batches (all in flight before the LDS stores).  A
// block that does not wrap (most of them) is read through one base address
// and a 32-bit offset advanced by constants; a wrapping one through the
// wrapped node indices.
template <int S, int BLOCK, typename T, int MAXB = 20>
__device__ __forceinline__ void stage_block(T *__restrict__ dst, const T *__restrict__ mesh, int n,
                                            int x0, int y0, int z0) {
    static_assert(S <= 64 && BLOCK % 64 == 0, "rows must fit a wave");
    constexpr int RPW = 64 / S;          // rows per wave and pass
    constexpr int RPP = RPW * (BLOCK / 64);
    constexpr int ROWS = S * S;
    constexpr int PASSES = (ROWS + RPP - 1) / RPP;
    constexpr int BATCH = PASSES < MAXB ? PASSES : MAXB;
    constexpr int DY = RPP % S, DZ = RPP / S;
    // every lane loads in every pass, also lanes whose value is not stored
    // (rr == RPW, rows past ROWS): the rows it visits are r0 + j RPP <=
    // PASSES RPP, so their z stays at most LZMAX
    constexpr int LZMAX = (PASSES * RPP) / S;
    const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
    const int rr = lane / S, lx = lane - rr * S;
    const bool act = rr < RPW;
    const int r0 = w * RPW + rr;
    const int m = n - 1;
    const int gx = (x0 + lx) & m;
    int ly = r0 % S, lz = r0 / S;       // (y, z) of this thread's current row
    const bool inside = x0 >= 0 && y0 >= 0 && z0 >= 0 && x0 + S <= n && y0 + S <= n &&
                        z0 + LZMAX < n;   // block-uniform
    const T *__restrict__ base = mesh + ((size_t)(inside ? z0 : 0) * n + (inside ? y0 : 0)) * n +
                                 (inside ? x0 : 0);
    const uint32_t nn = (uint32_t)n * (uint32_t)n;
    uint32_t off = (uint32_t)lz * nn + (uint32_t)ly * (uint32_t)n + (uint32_t)lx;
    const uint32_t dstep = (uint32_t)DY * (uint32_t)n + (uint32_t)DZ * nn;
    const uint32_t dwrap = nn - (uint32_t)S * (uint32_t)n;   // ly passed S: one z up
#pragma unroll
    for (int p0 = 0; p0 < PASSES; p0 += BATCH) {
        T v[BATCH];
        if (inside) {
#pragma unroll
            for (int k = 0; k < BATCH; ++k) {
                v[k] = base[off];
                ly += DY;
                off += dstep;
                if (ly >= S) {
                    ly -= S;
                    off += dwrap;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < BATCH; ++k) {
                // the wrapped (y, z, x) is a node of the mesh for every lane
                const uint32_t row =
                    (uint32_t)((z0 + lz) & m) * (uint32_t)n + (uint32_t)((y0 + ly) & m);
                v[k] = mesh[row * (uint32_t)n + (uint32_t)gx];
                ly += DY;
                lz += DZ;
                if (ly >= S) {
                    ly -= S;
                    ++lz;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < BATCH; ++k) {
            const int r = r0 + (p0 + k) * RPP;
            if (act && p0 + k < PASSES && r < ROWS) dst[r * S + lx] = v[k];
        }
    }
}

// ---- launch helpers (host) -------------------------------------------------

#define CUBE2_CHECK_HIP(expr)                                  \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return CUBE2_EHIP;               \
    } while (0)

#define CUBE2_LAUNCH_CHECK() CUBE2_CHECK_HIP(hipGetLastError())

// Host entry points of the kernel files (return CUBE2_* codes).
int launch_pack(cube2_ctx *ctx, const float *x, int64_t n, uint16_t *pos, uint32_t *cell_start,
                int32_t *perm, unsigned char *work, const WorkLayout &L, hipStream_t s);
// The stable sort by IOS cell of keys/vals (work) with the offsets of the
// unsorted particles; with vel != NULL the final gather also forms the kicked
// velocities vel_out[i] = vel[p] + kick acc[p] (FP64, separately rounded) of
// the sorted particles, p = perm[i].
int launch_sort_by_cell(cube2_ctx *ctx, int64_t n, const uint16_t *offs_in_unsorted,
                        uint16_t *pos, uint32_t *cell_start, int32_t *perm,
                        unsigned char *work, const WorkLayout &L, hipStream_t s,
                        const float *vel = nullptr, const float *acc = nullptr, double kick = 0.0,
                        float *vel_out = nullptr);
int launch_deposit(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                   float *rho_f, uint64_t *rho_f_fx, float *rho_c, uint64_t *rho_c_fx,
                   unsigned char *work, const WorkLayout &L, hipStream_t s);
int launch_green(cube2_ctx *ctx, hipStream_t s);
int launch_fft_r2c(cube2_ctx *ctx, int level, const float *mesh, float2 *spec, hipStream_t s);
int launch_potential(cube2_ctx *ctx, int level, const float *rho, float *phi, float2 *spec,
                     hipStream_t s);
int launch_potential64(cube2_ctx *ctx, int level, const double *rho, double *phi, double2 *spec,
                       hipStream_t s);
int launch_interp64(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                    const double *phi_f, const double *phi_c, double *acc, int accumulate,
                    hipStream_t s);
int launch_pp64(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n, double *acc,
                int accumulate, hipStream_t s);
int launch_fx_to_f64(uint64_t *buf, int64_t m, double unit, hipStream_t s);
int launch_interp(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                  const float *phi_f, const float *phi_c, float *acc, int accumulate,
                  hipStream_t s);
int launch_order_tiles(cube2_ctx *ctx, const uint32_t *cs, unsigned char *work,
                       const WorkLayout &L, hipStream_t s);
int launch_reset_tile_queue(cube2_ctx *ctx, unsigned char *work, const WorkLayout &L,
                            hipStream_t s);
// Device-wide exclusive scan of m uint32 (in may equal out); tmp: the
// scan_tmp work region.
int launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t m, uint32_t *tmp,
                          hipStream_t s);
int launch_interp_levels(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                         const float *phi_f, const float *phi_c, float *acc, int accumulate,
                         int levels, hipStream_t s);
int launch_tile_gather(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                       const int32_t *r0_host, int T, int R, float *x_local, int32_t *idx,
                       int64_t m_max, int64_t *m_out, unsigned char *work, const WorkLayout &L,
                       hipStream_t s);
// side k of the k^3 grid of slots that holds T tiles (a power of two)
int tile_slots(int T);
int launch_tile_scatter_add(int64_t m, const int32_t *perm_local, const float *x_local,
                            const int32_t *idx, int T, int lo, int hi, int n_slot, float scale,
                            const float *acc_local, float *acc, int64_t n, hipStream_t s);

// The tile order and work counter written by launch_order_tiles.
inline const uint32_t *tile_order_ptr(unsigned char *work, const WorkLayout &L) {
    return reinterpret_cast<const uint32_t *>(work + L.tile_order);
}
inline uint32_t *tile_queue_ptr(const cube2_ctx *ctx, unsigned char *work, const WorkLayout &L) {
    return reinterpret_cast<uint32_t *>(work + L.tile_order) + 4 * (size_t)ctx->nt * ctx->nt * ctx->nt;
}

// Workgroups of `kernel` (block threads, no dynamic LDS) that fit on the
// device at once, at most `ntiles`: the grid of a persistent launch.
template <typename K>
inline unsigned persistent_grid(K kernel, int block, int ntiles) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess)
        return (unsigned)ntiles;
    const long g = (long)(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
    return (unsigned)(g < ntiles ? g : ntiles);
}
int vel_bulk_side(const cube2_ctx *ctx);
int vel_layout_check(const cube2_ctx *ctx, const WorkLayout &L);
int launch_vel_encode(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                      const float *vel, int16_t *vq, float *v_bulk, float *v_scale,
                      unsigned char *work, const WorkLayout &L, hipStream_t s);
int launch_vel_decode(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                      const int16_t *vq, const float *v_bulk, const float *v_scale, float *vel,
                      hipStream_t s);
int launch_pp_concurrent(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                         const float *abar, float *acc_pp, unsigned char *work, const WorkLayout &L,
                         hipStream_t s);
int launch_add3(float *acc, const float *acc_pp, int64_t m, hipStream_t s);
// skip (device, one byte per tile, index (tz nt + ty) nt + tx, may be NULL):
// tiles whose own particles the kernel leaves alone
int launch_pp(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n, float *acc,
              int accumulate, unsigned char *work, const WorkLayout &L, hipStream_t s,
              const uint8_t *skip = nullptr);
// Address of the no-allocation entry point's scratch array on the current
// device (taken once per device); out may be NULL.
int noalloc_setup(unsigned char **out);
int build_pair_table(cube2_ctx *ctx);
int launch_kick_drift(cube2_ctx *ctx, const uint16_t *pos_in, const uint32_t *cs_in,
                      const float *vel_in, const float *acc, int64_t n, double kick,
                      double drift, uint16_t *pos_out, uint32_t *cs_out, float *vel_out,
                      int32_t *perm_out, unsigned char *work, const WorkLayout &L,
                      hipStream_t s);
int launch_reduce(cube2_ctx *ctx, const float *vel, const float *acc, int64_t n, double *out8,
                  unsigned char *work, const WorkLayout &L, hipStream_t s);
int launch_deposit_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                            int level, const float *rho_bar, float *x_bar, int accumulate,
                            hipStream_t s);
int launch_pm_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                       const float *acc_bar, float *x_bar, int accumulate, unsigned char *work,
                       const WorkLayout &L, hipStream_t s);
int launch_pp_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                       const float *acc_bar, float *x_bar, int accumulate, unsigned char *work,
                       const WorkLayout &L, hipStream_t s);
int launch_kick_drift_backward(cube2_ctx *ctx, int64_t n, const int32_t *perm,
                               const float *xbar_out, const float *vbar_out, double kick,
                               double drift, float *xbar_in, float *vbar_in, float *acc_bar,
                               hipStream_t s);

}  // namespace cube2
