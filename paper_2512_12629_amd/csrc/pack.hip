// pack.hip -- IOS particle order (section 2.3): quantise positions to integer
// in-cell offsets and sort particles stably by IOS cell, so that the particle
// order encodes cell membership and a prefix count per cell (cell_start)
// replaces per-particle cell indices.
//
// The sort is a stable least-significant-digit radix sort on the cell key
// (8-bit digits), written for 64-wide wavefronts: per 4096-key block a digit
// histogram, one device-wide scan of the digit-major histogram, then a
// scatter in which each key's rank among equal digits of its block comes
// from wave ballots (a 64-lane match on the digit) plus per-wave counts in
// LDS; the block's keys are staged in LDS in digit order and written out in
// runs.  Ties keep their input order, so the result equals a stable argsort.
// cell_start is read off the sorted keys (no per-cell atomics).
#include "common.hpp"

namespace cube2 {
namespace {

constexpr int kSortItems = 16;                   // keys per thread per block
constexpr int kSortTile = kBlock * kSortItems;   // 4096 keys per block
constexpr int kScanItems = 4;                    // items per thread in the scan
constexpr int kScanTile = kBlock * kScanItems;   // 1024

__global__ void fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// q = floor(x * n_f * 2^15) mod (n_f * 2^15); key of the IOS cell; offsets.
__global__ void quantize_kernel(const float *__restrict__ x, int n, int n_f, int nt,
                                uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                uint16_t *__restrict__ offs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double span = (double)n_f * 32768.0;
    const int64_t mask = (int64_t)n_f * 32768 - 1;
    int c[3];
    for (int d = 0; d < 3; ++d) {
        const int64_t q = (int64_t)floor((double)x[(int64_t)d * n + i] * span) & mask;
        c[d] = (int)(q >> 16);
        offs[(int64_t)d * n + i] = (uint16_t)(q & 0xFFFF);
    }
    keys[i] = cell_key(c[0], c[1], c[2], nt);
    vals[i] = (uint32_t)i;
}

// Exclusive scan, phase 1: scan each 1024-element tile, record tile sums.
__global__ void scan_tiles(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                           int64_t m, uint32_t *__restrict__ sums) {
    __shared__ uint32_t sh[kBlock / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems], s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < m) ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t pre = block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) out[base + k] = pre;
        pre += v[k];
    }
    if (threadIdx.x == 0 && sums) sums[blockIdx.x] = total;
}

__global__ void scan_add(uint32_t *__restrict__ out, int64_t m, const uint32_t *__restrict__ offs) {
    const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
    const uint32_t o = offs[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t j = i + (int64_t)k * kBlock;
        if (j < m) out[j] += o;
    }
}

// Device-wide exclusive scan of m entries (in may equal out); tmp holds
// the per-level tile sums.
int exclusive_scan(const uint32_t *in, uint32_t *out, int64_t m, uint32_t *tmp, hipStream_t s) {
    const int64_t tiles = (m + kScanTile - 1) / kScanTile;
    if (tiles <= 1) {
        scan_tiles<<<1, kBlock, 0, s>>>(in, out, m, nullptr);
        CUBE2_LAUNCH_CHECK();
        return CUBE2_OK;
    }
    uint32_t *sums = tmp;
    scan_tiles<<<(unsigned)tiles, kBlock, 0, s>>>(in, out, m, sums);
    CUBE2_LAUNCH_CHECK();
    int r = exclusive_scan(sums, sums, tiles, tmp + align_up((size_t)tiles, 64), s);
    if (r) return r;
    scan_add<<<(unsigned)tiles, kBlock, 0, s>>>(out, m, sums);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

__global__ void radix_count(const uint32_t *__restrict__ keys, int n, int shift, int nblk,
                            uint32_t *__restrict__ ghist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    ghist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Scatter of one 4096-key block.  The scanned digit-major histogram goff
// gives each (digit, block) its global start; the difference of consecutive
// entries is the block's own count of that digit.  Keys are first placed in
// LDS in digit order (rank among equal digits from wave ballots plus per-wave
// counts, so ties keep their input order), then written out in LDS order, so
// that consecutive threads write consecutive addresses of one digit's run.
__global__ void radix_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                              uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, int n,
                              int shift, int nblk, const uint32_t *__restrict__ goff) {
    __shared__ uint32_t gbase[256];  // global start of each digit of this block
    __shared__ uint32_t lpre[256];   // block-local start of each digit
    __shared__ uint32_t run[256];    // next free block-local slot of each digit
    __shared__ uint32_t wcnt[kBlock / 64][256];
    __shared__ uint32_t scan_sh[kBlock / 64 + 1];
    __shared__ uint32_t sk[kSortTile], sv[kSortTile];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    {
        const int64_t e = (int64_t)tid * nblk + blockIdx.x;
        const uint32_t g = goff[e];
        const uint32_t next = (e + 1 < (int64_t)nblk * 256) ? goff[e + 1] : (uint32_t)n;
        uint32_t total;
        const uint32_t lp = block_exclusive_scan(next - g, scan_sh, total);
        gbase[tid] = g;
        lpre[tid] = lp;
        run[tid] = lp;
    }
    for (int k = 0; k < kBlock / 64; ++k) wcnt[k][tid] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t blk0 = (int64_t)blockIdx.x * kSortTile;
    const int cnt = (int)min((int64_t)kSortTile, (int64_t)n - blk0);
    for (int r = 0; r < kSortItems; ++r) {
        const int li = r * kBlock + tid;
        const bool valid = li < cnt;
        uint32_t key = 0, val = 0, dig = 0;
        if (valid) {
            key = kin[blk0 + li];
            val = vin[blk0 + li];
            dig = (key >> shift) & 255u;
        }
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][dig] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t o = run[dig] + rank;
            for (int k = 0; k < w; ++k) o += wcnt[k][dig];
            sk[o] = key;
            sv[o] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int k = 0; k < kBlock / 64; ++k) {
            add += wcnt[k][tid];
            wcnt[k][tid] = 0;
        }
        run[tid] += add;
        __syncthreads();
    }
    for (int j = tid; j < cnt; j += kBlock) {
        const uint32_t key = sk[j];
        const uint32_t dig = (key >> shift) & 255u;
        const uint32_t o = gbase[dig] + ((uint32_t)j - lpre[dig]);
        kout[o] = key;
        vout[o] = sv[j];
    }
}

// cell_start from the sorted keys: entry c is the first index whose key is
// >= c, so index i (0..n) writes the entries (key[i-1], key[i]] (with key[-1]
// = -1 and key[n] = n_cells).  Every entry has exactly one writer.  A run of
// more than 64 entries (a stretch of empty cells) is written by the whole
// wave, so that sparse inputs do not leave one lane writing most of the mesh.
__global__ void cell_starts_kernel(const uint32_t *__restrict__ keys, int n, int64_t n_cells,
                                   uint32_t *__restrict__ cell_start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int64_t lo = 0, hi = -1;
    if (i <= n) {
        lo = i == 0 ? 0 : (int64_t)keys[i - 1] + 1;
        hi = i == n ? n_cells : (int64_t)keys[i];
    }
    const bool wide = hi - lo >= 64;
    if (!wide)
        for (int64_t c = lo; c <= hi; ++c) cell_start[c] = (uint32_t)i;
    uint64_t m = __ballot(wide);
    while (m) {
        const int l = __ffsll((long long)m) - 1;
        m &= m - 1;
        const long long a = __shfl((long long)lo, l, 64), b = __shfl((long long)hi, l, 64);
        const uint32_t v = (uint32_t)__shfl((int)i, l, 64);
        for (long long c = a + lane; c <= b; c += 64) cell_start[c] = v;
    }
}

__global__ void gather_offsets(const uint32_t *__restrict__ perm, const uint16_t *__restrict__ offs,
                               int n, uint16_t *__restrict__ pos, int32_t *__restrict__ perm_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = perm[i];
    pos[i] = offs[p];
    pos[(int64_t)n + i] = offs[(int64_t)n + p];
    pos[2 * (int64_t)n + i] = offs[2 * (int64_t)n + p];
    if (perm_out) perm_out[i] = (int32_t)p;
}

// gather_offsets and the kick of the velocities in one pass over the
// permutation: vout[i] = vel[p] + kick acc[p] in FP64 with separately rounded
// operations (the value the kick-drift kernel drifted with), p = perm[i].
__global__ void gather_offsets_kick(const uint32_t *__restrict__ perm,
                                    const uint16_t *__restrict__ offs, int n,
                                    uint16_t *__restrict__ pos, int32_t *__restrict__ perm_out,
                                    const float *__restrict__ vel, const float *__restrict__ acc,
                                    double kick, float *__restrict__ vout) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t p = perm[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t o = (int64_t)d * n;
        pos[o + i] = offs[o + p];
        const double kv = kick * (double)acc[o + p];
        vout[o + i] = (float)((double)vel[o + p] + kv);
    }
    perm_out[i] = (int32_t)p;
}

// Tiles in dispatch order b (the XCD-slab order of tile_of_block), keyed by
// how many thousand particles they own, largest first.
__global__ void tile_keys_kernel(const uint32_t *__restrict__ cs, int nt, uint32_t *__restrict__ keys,
                                 uint32_t *__restrict__ vals) {
    const int ntiles = nt * nt * nt;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= ntiles) return;
    int tx, ty, tz;
    tile_of_block(b, nt, tx, ty, tz);
    const uint32_t t = (uint32_t)((tz * nt + ty) * nt + tx);
    const uint32_t cnt = cs[(t + 1) * kTileCells] - cs[t * kTileCells];
    keys[b] = 255u - min(cnt >> 10, 255u);
    vals[b] = t;
}

}  // namespace

int launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t m, uint32_t *tmp,
                          hipStream_t s) {
    return exclusive_scan(in, out, m, tmp, s);
}

// Work order of the persistent per-tile kernels: the tiles sorted (stably,
// one 8-bit radix pass) by their particle count in units of 1024, descending,
// so that the heaviest tiles start first and the light ones keep the
// XCD-slab order.  The tile indices land in the first ntiles words of the
// tile_order region; the work counter (tile_queue_ptr) is reset to zero.
int launch_order_tiles(cube2_ctx *ctx, const uint32_t *cs, unsigned char *work,
                       const WorkLayout &L, hipStream_t s) {
    const int nt = ctx->nt;
    const int ntiles = nt * nt * nt;
    uint32_t *base = reinterpret_cast<uint32_t *>(work + L.tile_order);
    uint32_t *order = base, *vin = base + ntiles, *kin = base + 2 * ntiles, *kout = base + 3 * ntiles;
    uint32_t *tmp = reinterpret_cast<uint32_t *>(work + L.scan_tmp);
    uint32_t *ghist = reinterpret_cast<uint32_t *>(work + L.hist);
    tile_keys_kernel<<<(ntiles + 255) / 256, 256, 0, s>>>(cs, nt, kin, vin);
    CUBE2_LAUNCH_CHECK();
    const int nblk = (ntiles + kSortTile - 1) / kSortTile;
    radix_count<<<nblk, kBlock, 0, s>>>(kin, ntiles, 0, nblk, ghist);
    CUBE2_LAUNCH_CHECK();
    int r = exclusive_scan(ghist, ghist, (int64_t)nblk * 256, tmp, s);
    if (r) return r;
    radix_scatter<<<nblk, kBlock, 0, s>>>(kin, vin, kout, order, ntiles, 0, nblk, ghist);
    CUBE2_LAUNCH_CHECK();
    return launch_reset_tile_queue(ctx, work, L, s);
}

int launch_reset_tile_queue(cube2_ctx *ctx, unsigned char *work, const WorkLayout &L,
                            hipStream_t s) {
    fill_u32<<<1, 64, 0, s>>>(tile_queue_ptr(ctx, work, L), 0u, 1);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

// keys/vals (work) and offs_tmp (work) hold the unsorted particles.
int launch_sort_by_cell(cube2_ctx *ctx, int64_t n64, const uint16_t *offs, uint16_t *pos,
                        uint32_t *cell_start, int32_t *perm, unsigned char *work,
                        const WorkLayout &L, hipStream_t s, const float *vel, const float *acc,
                        double kick, float *vel_out) {
    const int n = (int)n64;
    uint32_t *tmp = reinterpret_cast<uint32_t *>(work + L.scan_tmp);
    uint32_t *k0 = reinterpret_cast<uint32_t *>(work + L.keys);
    uint32_t *v0 = reinterpret_cast<uint32_t *>(work + L.vals);
    uint32_t *k1 = reinterpret_cast<uint32_t *>(work + L.keys2);
    uint32_t *v1 = reinterpret_cast<uint32_t *>(work + L.vals2);
    uint32_t *ghist = reinterpret_cast<uint32_t *>(work + L.hist);
    int r = CUBE2_OK;
    if (n == 0) {
        cell_starts_kernel<<<1, 64, 0, s>>>(k0, 0, ctx->n_cells, cell_start);
        CUBE2_LAUNCH_CHECK();
        return CUBE2_OK;
    }

    int bits = 0;
    while (((int64_t)1 << bits) < ctx->n_cells) ++bits;
    const int nblk = (n + kSortTile - 1) / kSortTile;
    for (int shift = 0; shift < bits; shift += 8) {
        radix_count<<<nblk, kBlock, 0, s>>>(k0, n, shift, nblk, ghist);
        CUBE2_LAUNCH_CHECK();
        r = exclusive_scan(ghist, ghist, (int64_t)nblk * 256, tmp, s);
        if (r) return r;
        radix_scatter<<<nblk, kBlock, 0, s>>>(k0, v0, k1, v1, n, shift, nblk, ghist);
        CUBE2_LAUNCH_CHECK();
        uint32_t *t = k0; k0 = k1; k1 = t;
        t = v0; v0 = v1; v1 = t;
    }
    // cell_start (n_cells + 1 entries, the last = n) from the sorted keys
    cell_starts_kernel<<<(unsigned)((n + 1 + 255) / 256), 256, 0, s>>>(k0, n, ctx->n_cells, cell_start);
    CUBE2_LAUNCH_CHECK();
    if (vel)
        gather_offsets_kick<<<(n + 255) / 256, 256, 0, s>>>(v0, offs, n, pos, perm, vel, acc, kick,
                                                           vel_out);
    else
        gather_offsets<<<(n + 255) / 256, 256, 0, s>>>(v0, offs, n, pos, perm);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

int launch_pack(cube2_ctx *ctx, const float *x, int64_t n64, uint16_t *pos, uint32_t *cell_start,
                int32_t *perm, unsigned char *work, const WorkLayout &L, hipStream_t s) {
    const int n = (int)n64;
    uint16_t *offs = reinterpret_cast<uint16_t *>(work + L.offs_tmp);
    if (n > 0) {
        quantize_kernel<<<(n + 255) / 256, 256, 0, s>>>(
            x, n, ctx->n_f, ctx->nt, reinterpret_cast<uint32_t *>(work + L.keys),
            reinterpret_cast<uint32_t *>(work + L.vals), offs);
        CUBE2_LAUNCH_CHECK();
    }
    return launch_sort_by_cell(ctx, n, offs, pos, cell_start, perm, work, L, s);
}

}  // namespace cube2
