// pp.hip -- the short-range particle-particle force (eq. 4d): for every pair
// closer than the fine softening b_f (the cutoff of the finest PM level),
//   a_i += G m [R(r, b_pp) - R(r, b_f)] (x_j - x_i) / r,
// with R of eq. (2).  An IOS cell is 2 fine cells, so for b_f <= 2 every
// pair lies in the same or in adjacent IOS cells (27 neighbour cells), and
// for 2 < b_f <= 4 within two cells (125); the cell-sorted particle order is
// the linked list of the paper (section 2.3).
//
// One workgroup per tile.  The particles of the tile and of its halo of H
// cells (a (8 + 2H)^3 box of IOS cells) are staged in LDS as FP32 positions
// relative to the tile origin in fine cells.  Offsets are multiples of 2^-15
// below 2^5, so these floats and their differences are exact: the pair
// separation is the exact integer one.  Each thread takes one particle of the
// tile and loops over its neighbour cells, which in the staged box are
// (2H + 1)^2 contiguous ranges (x-rows of 2H + 1 cells); neighbours in a
// dense cell are read by all lanes of a wave at the same LDS address (a
// broadcast).  Per range the pair sum is accumulated in FP32 and then added
// to the total with Kahan compensation.  Boxes too large for LDS read the
// same data from HBM.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.hpp"

namespace cube2 {
namespace {

// H: the neighbour reach in IOS cells, 1 for b_f <= 2 fine cells (27
// neighbour cells) and 2 for b_f <= 4 (125).  The staged box has
// 8 + 2H IOS cells per axis.
template <int H> struct PPBox {
    static constexpr int PB = kTileIos + 2 * H;   // 10 or 12 IOS cells per axis
    static constexpr int SEGS = PB * PB * PB;      // 1000 or 1728
    static constexpr int W = 2 * H + 1;            // neighbour cells per axis
};
// Forward: 512 threads, 3840 staged particles (60 KB; 3456 with the wider
// box): 2 blocks (4 waves per SIMD) per CU.  Adjoint: the cotangent is staged
// too, so it runs 1024-thread blocks with 4096 staged particles (128 KB):
// 1 block (4 waves per SIMD).
template <bool ADJ, int H> struct PPGeo {
    static constexpr int BLOCK = ADJ ? 1024 : 512;
    static constexpr int CAP = ADJ ? 4096 : (H == 1 ? 3840 : 3456);
    static constexpr int SEG_PER_THREAD = (PPBox<H>::SEGS + BLOCK - 1) / BLOCK;
};

}  // namespace

// The pair law g(r) = [R(r,b_pp) - R(r,b_f)] / r (eqs. 2 and 4d) as
// g = U(r) / r^3 with U = r^3 g.  On each of the intervals delimited by the
// breakpoints of eq. (2) -- b_pp/2, b_pp (PP softening), b_f/2 (fine
// softening) -- and the cutoff b_f, U is an exact polynomial of degree 8 in r:
//   r^3 b^-3 F_in(r/b)  = sum_k a_k b^(-3-k) r^(k+3),
//   r^3 b^-3 F_out(r/b) = 3/35 - 32/5 (r/b)^2 + sum_k c_k b^(-3-k) r^(k+3),
//   r^3 r^-3 = 1 (Newtonian beyond b_pp),
// with F_in, F_out the two polynomial branches of R(r,b)/r in t = r/b.
// [0, b_f) is cut into K equal intervals with every breakpoint on an
// interval edge, and each interval stores its polynomial re-expanded (FP64,
// on the host) in a local variable y in [0, 1]:  y = fract(r K / b_f) (left
// edge, keeps U ~ r^3 accurate at r -> 0) or y = 1 - fract(.) (right edge)
// on the intervals where 1/r^2 - R(r, b_f) vanishes like (1 - r/b_f)^5 at the
// cutoff, which use the exact factorisation r^3 g = s^5 Q(1 - s),
// s = 1 - r/b_f, Q(t) = 32/35 + 32/7 t + 704/35 t^2 + 64/5 t^3.  The row of
// r >= b_f is zero.  This exact table, in FP64, serves the plain FP64 form.
//
// The FP32 forward kernel evaluates g as a function of s = r^2 instead, which
// needs neither a square root nor r^-3.  Since g vanishes like (b_f - r)^5 at
// the cutoff, and sparse particles often have all their neighbours close to
// it, the table does not hold g itself: with h = g / (b_f^2 - s)^5, smooth and
// nonzero up to and beyond the cutoff (there the factorised form gives h =
// Q(1 - r/b_f) / (r^3 (b_f (b_f + r))^5), continued analytically past b_f),
// it holds H = h b_f^10 w = g / w^4 with w = 1 - s/b_f^2, still smooth (one
// simple zero at the cutoff, continued linearly past it), and the kernel
// forms g = H w^4 with w clamped to [0, 1]: exact zero beyond the cutoff.
// Near the cutoff the fit of H errs like 1/w relative (7e-7 at w = 1/32 on
// the row s in [3.75, 3.875) for b_f = 2), as the FP32 rounding of s does
// anyway (b_f^2 - s turns it into 6e-8 / w per power of w); with more powers
// of w in the table the cubic would have to follow a multiple zero.  s is cut
// at its float exponent and top 4 mantissa bits (1/16 of an octave, s in
// [2^-31, 2^7)); on each piece H is the cubic through its values at the 4 Chebyshev nodes (fitted in FP64
// on the host from eq. (2) evaluated in extended precision).  For exact s the
// table's g is within 8e-7 of the true g, relative; FP32 rounding of s adds
// its own part near the cutoff, as rounding of r does in any evaluation.  The
// row index is the bit pattern of s shifted right, the local variable the
// remaining 19 mantissa bits read as a float in [0, 1/16).  Every pair
// separation in the staged box is below 2(H + 1) fine cells per axis (4 or
// 6), so s < 108 < 2^7 and the row exists; the 2^-31 added to s (below the smallest nonzero
// separation squared, 2^-30) keeps a coincident pair on row 0, where g is
// finite and g D = 0.

namespace {

// The pair-law table in LDS, declared at namespace scope so that every
// access is a 32-bit LDS address, indexed by s = r^2 (the forward and the
// adjoint kernel both read it).
__shared__ float4 pair_srows[kSRows];

__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// g(r) * D accumulated into (fx, fy, fz) from the s-indexed table (LDS).
// The table holds H = g / w^4, and w = 1 - s/b_f^2 is formed as one FMA with
// the result clamped to [0, 1] (negc = -1/b_f^2 rounded away from zero, so
// that w = 0 for every s >= b_f^2).
__device__ __forceinline__ float unit_clamp(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }

__device__ __forceinline__ void pair_accumulate(float dx, float dy, float dz, float negc, float &fx,
                                                float &fy, float &fz) {
    const float s = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, 0x1p-31f)));
    const uint32_t b = __float_as_uint(s);
    const float4 c = pair_srows[(b >> (23 - kSMantBits)) - kSRow0];
    const float z = __uint_as_float((b & ((1u << (23 - kSMantBits)) - 1u)) | 0x3F800000u) - 1.0f;
    const float h = fmaf(fmaf(fmaf(c.w, z, c.z), z, c.y), z, c.x);
    const float w = unit_clamp(fmaf(s, negc, 1.0f));
    const float w2 = w * w;
    const float g = h * (w2 * w2);
    fx = fmaf(g, dx, fx);
    fy = fmaf(g, dy, fy);
    fz = fmaf(g, dz, fz);
}

// Adjoint of one pair for the cotangents: out += J(D) u with u = abar_j -
// abar_i and J = d(g D)/dD = g I + 2 g_s D D^T, g_s = dg/ds.  It reads the
// forward's table: H = g / w^4, w = 1 - s/b_f^2, and, by synthetic
// division of the same cubic, dH/dz, with z the local variable of the row
// (s = 2^e (1 + z)), so H_s = (dH/dz) 2^-e; one 16-byte table read per pair
// (the LDS reads, not the arithmetic, limit this kernel).  With w clamped to
// [0, 1] as in pair_accumulate: g = H w^4 and 2 g_s = w^3 (2 H_s w + 8 negc
// H), negc = -1/b_f^2.  Every term enters the accumulators through an FMA.
__device__ __forceinline__ void pair_adjoint(float dx, float dy, float dz, float ux, float uy,
                                             float uz, float negc, float &ox, float &oy,
                                             float &oz) {
    const float s = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, 0x1p-31f)));
    const uint32_t b = __float_as_uint(s);
    const float4 c = pair_srows[(b >> (23 - kSMantBits)) - kSRow0];
    const float z = __uint_as_float((b & ((1u << (23 - kSMantBits)) - 1u)) | 0x3F800000u) - 1.0f;
    const float inv2e2 = __uint_as_float(0x7F800000u - (b & 0x7F800000u));  // 2^(1-e)
    float h = fmaf(c.w, z, c.z);
    float hz = fmaf(c.w, z, h);
    h = fmaf(h, z, c.y);
    hz = fmaf(hz, z, h);
    h = fmaf(h, z, c.x);
    const float w = unit_clamp(fmaf(s, negc, 1.0f));
    const float w2 = w * w;
    const float g = h * (w2 * w2);
    const float gs2 = (w2 * w) * fmaf(hz * inv2e2, w, (8.0f * negc) * h);  // 2 g_s
    const float du = fmaf(dz, uz, fmaf(dy, uy, dx * ux)) * gs2;
    ox = fmaf(du, dx, fmaf(g, ux, ox));
    oy = fmaf(du, dy, fmaf(g, uy, oy));
    oz = fmaf(du, dz, fmaf(g, uz, oz));
}

// Heavy tiles are done in z-chunks: own cells are ordered z-major, so the own
// cells of z-layers [z0, z1) are a contiguous particle range and the box cells
// they need are the contiguous box layers [z0, z1 + 2H), a contiguous slice of
// the staged list.

// The heaviest tiles are split: the first kSplitTiles entries of the
// heaviest-first order are offered as kSplitParts work items each; a tile
// with `own` particles uses min(kSplitParts, ceil(own / block)) of them,
// each part staging the tile's box and taking every nparts-th block of its
// own particles, and the other items end at once.  A tile where Plummer
// spheres overlap holds several times the pairs of one sphere, and when a
// workload has few tiles per workgroup such a tile would end the kernel
// alone; each particle's sum is still formed by one thread in the same
// order.  (Splitting four tiles per workgroup was slower: every part
// stages the box again.)
// The two-cell reach (b_f > 2) keeps whole tiles: it has ~5x the pairs per
// tile, so its tiles are not few per workgroup, and the split's bookkeeping
// would take it past 128 VGPRs (one workgroup per CU instead of two).
constexpr int kSplitParts = 8, kSplitTiles = 128;
template <int H> constexpr int split_parts() { return H == 1 ? kSplitParts : 1; }

// ADJ = false: acc = G m sum_j g D (forward).  ADJ = true: out = G m sum_j
// J(D) (abar_j - abar_i) for the cotangent abar (the adjoint), which stages
// abar_j beside x_j and so holds half as many particles per chunk.
template <bool ADJ, int H>
__global__ __launch_bounds__((PPGeo<ADJ, H>::BLOCK)) void pp_kernel(const uint16_t *__restrict__ pos,
                                                     const uint32_t *__restrict__ cs, int n,
                                                     int nt, const float4 *__restrict__ table,
                                                     float negc, float gm,
                                                     const float *__restrict__ abar,
                                                     float *__restrict__ acc, int accumulate,
                                                     const uint32_t *__restrict__ order,
                                                     uint32_t *__restrict__ queue, int ntiles,
                                                     int nsplit,
                                                     const uint8_t *__restrict__ skip) {
    constexpr int CAP = PPGeo<ADJ, H>::CAP;
    constexpr int kPPBlock = PPGeo<ADJ, H>::BLOCK;
    constexpr int kPSegPerThread = PPGeo<ADJ, H>::SEG_PER_THREAD;
    constexpr int kPB = PPBox<H>::PB, kPSegs = PPBox<H>::SEGS, kW = PPBox<H>::W;
    __shared__ uint32_t seg_pre[kPSegs + 1];
    __shared__ uint32_t seg_src[kPSegs];
    // staged particles; the adjoint interleaves each position with its
    // cotangent (xs[2 v], xs[2 v + 1]), so that both reads of a pair share one
    // address register
    constexpr int XS = ADJ ? 2 : 1;
    __shared__ float4 xs[XS * CAP];
    __shared__ uint32_t cst[kTileCells + 1];     // own cells: particle starts (tile-relative)
    __shared__ uint32_t scan_sh[kPPBlock / 64 + 1];
    __shared__ int chunk_sh, tile_sh;
    __shared__ uint32_t maxcnt_sh;

    const int tid = threadIdx.x;
    const int n_ios = nt * kTileIos;
    const float inv = 1.0f / 32768.0f;
    for (int i = tid; i < kSRows; i += kPPBlock) pair_srows[i] = table[i];

    // Persistent workgroups: each takes the next work item of the
    // heaviest-first order (claim_slot) until all are taken (the exit test
    // is block-uniform).  Thread 0 claims the next item while the current
    // one is processed.  Items [0, nsplit kSplitParts) are the parts of the
    // nsplit heaviest tiles, the rest one whole tile each.
    constexpr int kParts = split_parts<H>();
    const int nitems = ntiles + nsplit * (kParts - 1);
    const int split_items = nsplit * kParts;
    int next = 0;
    if (tid == 0) next = claim_slot(queue, nitems);
    for (;;) {
        if (tid == 0) {
            tile_sh = next;
            maxcnt_sh = 0u;
        }
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(tile_sh);   // block-uniform
        if (item >= nitems) break;
        if (tid == 0) next = claim_slot(queue, nitems);
        const bool split = kParts > 1 && item < split_items;
        const int ti = split ? item / kParts : item - split_items + nsplit;
        const int part = split ? item % kParts : 0;
        const int t = (int)order[ti];
        int nparts = 1;
        if (split) {
            const uint32_t own = cs[(uint32_t)(t + 1) * kTileCells] - cs[(uint32_t)t * kTileCells];
            nparts = (int)min((own + kPPBlock - 1) / kPPBlock, (uint32_t)kParts);
            nparts = __builtin_amdgcn_readfirstlane(max(nparts, 1));
        }
        if ((skip && skip[t]) || part >= nparts) {   // another level's tile, or a spare part
            __syncthreads();     // every thread has read tile_sh
            continue;
        }
        const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
        const int c0x = tx * kTileIos, c0y = ty * kTileIos, c0z = tz * kTileIos;

        // particle ranges of the 10^3 box of IOS cells [c0-1, c0+9)
        uint32_t cnt[kPSegPerThread], src[kPSegPerThread], pre_k[kPSegPerThread];
        uint32_t sum = 0, mx = 0;
#pragma unroll
        for (int k = 0; k < kPSegPerThread; ++k) {
            const int s = tid * kPSegPerThread + k;
            cnt[k] = 0;
            src[k] = 0;
            if (s < kPSegs) {
                const int bx = s % kPB, by = (s / kPB) % kPB, bz = s / (kPB * kPB);
                const uint32_t key = cell_key(wrapn(c0x + bx - H, n_ios), wrapn(c0y + by - H, n_ios),
                                              wrapn(c0z + bz - H, n_ios), nt);
                src[k] = cs[key];
                cnt[k] = cs[key + 1] - src[k];
            }
            sum += cnt[k];
            mx = max(mx, cnt[k]);
        }
        atomicMax(&maxcnt_sh, mx);
        uint32_t total;
        uint32_t pre = block_exclusive_scan<kPPBlock>(sum, scan_sh, total);
#pragma unroll
        for (int k = 0; k < kPSegPerThread; ++k) {
            const int s = tid * kPSegPerThread + k;
            if (s < kPSegs) {
                seg_pre[s] = pre;
                seg_src[s] = src[k];
            }
            pre_k[k] = pre;
            pre += cnt[k];
        }
        if (tid == 0) seg_pre[kPSegs] = total;
        __syncthreads();
        // own cells (box segments with coordinates 1..8): their particle
        // starts relative to the tile's first particle, from the box ranges
        // (the own cells' particles are one contiguous range)
        const uint32_t p0 = seg_src[(H * kPB + H) * kPB + H];
        for (int i = tid; i <= kTileCells; i += kPPBlock) {
            if (i < kTileCells) {
                const int s = (((i >> 6) + H) * kPB + ((i >> 3) & 7) + H) * kPB + (i & 7) + H;
                cst[i] = seg_src[s] - p0;
            } else {
                const int s = ((7 + H) * kPB + 7 + H) * kPB + 7 + H;  // last own cell
                cst[i] = seg_src[s] + (seg_pre[s + 1] - seg_pre[s]) - p0;
            }
        }
        if (tid == 0) {
            // z-chunks: the smallest power-of-two count whose staged slices fit
            int C = 1;
            for (; C < 8; C <<= 1) {
                bool fits = true;
                for (int c = 0; c < C; ++c) {
                    const int z0 = c * 8 / C, z1 = (c + 1) * 8 / C;
                    if (seg_pre[(z1 + 2 * H) * kPB * kPB] - seg_pre[z0 * kPB * kPB] > (uint32_t)CAP)
                        fits = false;
                }
                if (fits) break;
            }
            chunk_sh = C;
        }
        __syncthreads();
        const int C = chunk_sh;
        const uint32_t maxcnt = maxcnt_sh;

        for (int c = 0; c < C; ++c) {
            const int z0 = c * 8 / C, z1 = (c + 1) * 8 / C;
            const uint32_t vb = seg_pre[z0 * kPB * kPB], ve = seg_pre[(z1 + 2 * H) * kPB * kPB];
            const bool staged = ve - vb <= (uint32_t)CAP;
            if (c > 0) __syncthreads();  // previous chunk done with xs
            if (!ADJ && staged && C == 1 && maxcnt <= 4) {
                // sparse box: every thread copies the particles of its own
                // segments (at most 4 each), no search needed; one segment at
                // a time keeps the register footprint of the staging small
#pragma unroll 1
                for (int k = 0; k < kPSegPerThread; ++k) {
                    const int s = tid * kPSegPerThread + k;
                    const int bx = s % kPB, by = (s / kPB) % kPB, bz = s / (kPB * kPB);
                    uint32_t o[4][3];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if ((uint32_t)i >= cnt[k]) continue;
                        const uint32_t p = src[k] + i;
                        o[i][0] = pos[p];
                        o[i][1] = pos[(int64_t)n + p];
                        o[i][2] = pos[2 * (int64_t)n + p];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if ((uint32_t)i >= cnt[k]) continue;
                        float4 q;
                        q.x = (float)(2 * (bx - H)) + (float)o[i][0] * inv;
                        q.y = (float)(2 * (by - H)) + (float)o[i][1] * inv;
                        q.z = (float)(2 * (bz - H)) + (float)o[i][2] * inv;
                        q.w = 0.0f;
                        xs[XS * (pre_k[k] + i)] = q;
                        if (ADJ) {
                            const uint32_t p = src[k] + i;
                            xs[XS * (pre_k[k] + i) + 1] = make_float4(abar[p], abar[(int64_t)n + p],
                                                                      abar[2 * (int64_t)n + p], 0.f);
                        }
                    }
                }
            } else if (staged) {
                // kStage particles per thread at a time: the segment searches and
                // the loads of a batch are issued before the LDS stores
                constexpr int kStage = 4;
                for (uint32_t v0 = vb + tid; v0 < ve; v0 += kPPBlock * kStage) {
                    int sg[kStage];
                    uint32_t pj[kStage];
#pragma unroll
                    for (int k = 0; k < kStage; ++k) {
                        const uint32_t v = v0 + k * kPPBlock;
                        sg[k] = v < ve ? seg_search(seg_pre, kPSegs, v) : -1;
                        pj[k] = sg[k] < 0 ? 0u : seg_src[sg[k]] + (v - seg_pre[sg[k]]);
                    }
                    uint32_t o[kStage][3];
                    float4 ab[kStage];
#pragma unroll
                    for (int k = 0; k < kStage; ++k) {
                        if (sg[k] < 0) continue;
                        const uint32_t p = pj[k];
                        o[k][0] = pos[p];
                        o[k][1] = pos[(int64_t)n + p];
                        o[k][2] = pos[2 * (int64_t)n + p];
                        if (ADJ)
                            ab[k] = make_float4(abar[p], abar[(int64_t)n + p],
                                                abar[2 * (int64_t)n + p], 0.f);
                    }
#pragma unroll
                    for (int k = 0; k < kStage; ++k) {
                        if (sg[k] < 0) continue;
                        const int s = sg[k];
                        const int bx = s % kPB, by = (s / kPB) % kPB, bz = s / (kPB * kPB);
                        float4 q;
                        q.x = (float)(2 * (bx - H)) + (float)o[k][0] * inv;
                        q.y = (float)(2 * (by - H)) + (float)o[k][1] * inv;
                        q.z = (float)(2 * (bz - H)) + (float)o[k][2] * inv;
                        q.w = 0.0f;
                        const uint32_t v = v0 + k * kPPBlock;
                        xs[XS * (v - vb)] = q;
                        if (ADJ) xs[XS * (v - vb) + 1] = ab[k];
                    }
                }
            }
            __syncthreads();
            // own particles of the cells [z0*64, z1*64): a contiguous range;
            // part p of a split tile takes its blocks p, p + nparts, ...
            const uint32_t q0 = cst[z0 * 64], q1 = cst[z1 * 64];
            for (uint32_t lp = q0 + (uint32_t)(part * kPPBlock + tid); lp < q1;
                 lp += (uint32_t)(kPPBlock * nparts)) {
                const int u = seg_search_n<kTileCells>(cst, lp);
                const uint32_t p = p0 + lp;
                const int bx = (u & 7) + H, by = ((u >> 3) & 7) + H, bz = (u >> 6) + H;
                float xi, yi, zi;
                if (staged) {
                    // the particle itself is staged: same exact floats, no HBM read
                    const int su = (bz * kPB + by) * kPB + bx;
                    const float4 qi = xs[XS * (seg_pre[su] + (lp - cst[u]) - vb)];
                    xi = qi.x;
                    yi = qi.y;
                    zi = qi.z;
                } else {
                    xi = (float)(2 * (bx - H)) + (float)pos[p] * inv;
                    yi = (float)(2 * (by - H)) + (float)pos[(int64_t)n + p] * inv;
                    zi = (float)(2 * (bz - H)) + (float)pos[2 * (int64_t)n + p] * inv;
                }
                float aix = 0.f, aiy = 0.f, aiz = 0.f;
                if (ADJ) {
                    aix = abar[p];
                    aiy = abar[(int64_t)n + p];
                    aiz = abar[2 * (int64_t)n + p];
                }
                float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
                if (staged) {
                    // the three x-neighbours of a cell are consecutive box segments,
                    // so the 27 neighbour cells are 9 contiguous ranges of xs
                    for (int row = 0; row < kW * kW; ++row) {
                        const int oy = row % kW - H, oz = row / kW - H;
                        const int sm = ((bz + oz) * kPB + (by + oy)) * kPB + bx;
                        const uint32_t v0 = seg_pre[sm - H] - vb, v1 = seg_pre[sm + H + 1] - vb;
                        float fx = 0.f, fy = 0.f, fz = 0.f;
                        if (ADJ) {
                            // four pairs per iteration: the loop control and the LDS
                            // latency spread over more work.  The loops run on the
                            // LDS address against precomputed bounds, never below xs
                            // (LDS addresses compare unsigned).
                            const float4 *q = xs + 2 * v0;
                            const float4 *const qe = xs + 2 * v1;
                            const float4 *const qe4 = xs + 2 * (v1 >= v0 + 3 ? v1 - 3 : v0);
                            for (; q < qe4; q += 8) {
                                float4 x[4], a[4];
#pragma unroll
                                for (int t = 0; t < 4; ++t) {
                                    x[t] = q[2 * t];
                                    a[t] = q[2 * t + 1];
                                }
#pragma unroll
                                for (int t = 0; t < 4; ++t)
                                    pair_adjoint(x[t].x - xi, x[t].y - yi, x[t].z - zi, a[t].x - aix,
                                                 a[t].y - aiy, a[t].z - aiz, negc, fx, fy, fz);
                            }
                            for (; q < qe; q += 2) {
                                const float4 qa = q[0], aa = q[1];
                                pair_adjoint(qa.x - xi, qa.y - yi, qa.z - zi, aa.x - aix, aa.y - aiy,
                                             aa.z - aiz, negc, fx, fy, fz);
                            }
                        } else {
                            // two pairs per iteration.  The loop runs on the LDS
                            // address against a precomputed bound, never below xs
                            // (one add and one compare per trip).
                            const float4 *q = xs + v0;
                            const float4 *const qend = xs + v1;
                            const float4 *const qe = xs + (v1 > v0 ? v1 - 1 : v0);
                            for (; q < qe; q += 2) {
                                const float4 qa = q[0], qb = q[1];
                                pair_accumulate(qa.x - xi, qa.y - yi, qa.z - zi, negc, fx, fy, fz);
                                pair_accumulate(qb.x - xi, qb.y - yi, qb.z - zi, negc, fx, fy, fz);
                            }
                            if (q < qend) {
                                const float4 qa = q[0];
                                pair_accumulate(qa.x - xi, qa.y - yi, qa.z - zi, negc, fx, fy, fz);
                            }
                        }
                        kahan_add(sx, cx, fx);
                        kahan_add(sy, cy, fy);
                        kahan_add(sz, cz, fz);
                    }
                } else {
                    for (int nb = 0; nb < kW * kW * kW; ++nb) {
                        const int ox = nb % kW - H, oy = (nb / kW) % kW - H, oz = nb / (kW * kW) - H;
                        const int s = ((bz + oz) * kPB + (by + oy)) * kPB + (bx + ox);
                        const uint32_t v0 = seg_pre[s], v1 = seg_pre[s + 1];
                        const float bxo = (float)(2 * (bx + ox - H)), byo = (float)(2 * (by + oy - H)),
                                    bzo = (float)(2 * (bz + oz - H));
                        float fx = 0.f, fy = 0.f, fz = 0.f;
                        for (uint32_t v = v0; v < v1; ++v) {
                            const uint32_t pj = seg_src[s] + (v - v0);
                            const float xj = bxo + (float)pos[pj] * inv;
                            const float yj = byo + (float)pos[(int64_t)n + pj] * inv;
                            const float zj = bzo + (float)pos[2 * (int64_t)n + pj] * inv;
                            if (ADJ)
                                pair_adjoint(xj - xi, yj - yi, zj - zi, abar[pj] - aix,
                                             abar[(int64_t)n + pj] - aiy, abar[2 * (int64_t)n + pj] - aiz,
                                             negc, fx, fy, fz);
                            else
                                pair_accumulate(xj - xi, yj - yi, zj - zi, negc, fx, fy, fz);
                        }
                        kahan_add(sx, cx, fx);
                        kahan_add(sy, cy, fy);
                        kahan_add(sz, cz, fz);
                    }
                }
                const float a[3] = {gm * sx, gm * sy, gm * sz};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    float *dst = acc + (int64_t)d * n + p;
                    *dst = accumulate ? *dst + a[d] : a[d];
                }
            }
        }
        __syncthreads();  // this tile is done with the LDS arrays
    }
}

}  // namespace

namespace {

// Q(y) = P(alpha + beta y) for a degree-8 polynomial (coefficients low to high).
void compose(const double P[9], double alpha, double beta, double Q[9]) {
    double q[9] = {P[8], 0, 0, 0, 0, 0, 0, 0, 0};
    for (int m = 7; m >= 0; --m) {
        double t[9];
        for (int j = 0; j < 9; ++j) t[j] = alpha * q[j] + (j > 0 ? beta * q[j - 1] : 0.0);
        t[0] += P[m];
        for (int j = 0; j < 9; ++j) q[j] = t[j];
    }
    for (int j = 0; j < 9; ++j) Q[j] = q[j];
}

}  // namespace

namespace {

// h = g / (b_f^2 - r^2)^5 for the pair law g(r) of eqs. (2) and (4d), in
// extended precision: where 1/r^2 - R(r, b_f) would cancel (r >= b_pp and
// r >= b_f/2) through its factorised form (which also continues h past the
// cutoff), elsewhere from the branches of R(r, b).
long double pair_h_direct(double b_pp, double b_f, double rd) {
    using X = long double;
    const X r = rd, bf = b_f;
    auto r_over_r = [&](X b) -> X {  // R(r, b) / r
        const X t = r / b;
        if (t >= 1) return 1 / (r * r * r);
        if (2 * t < 1)
            return (X(64) / 5 + t * t * (X(-256) / 5 + t * (32 + t * (X(1536) / 35 + t * (X(-192) / 5))))) /
                   (b * b * b);
        const X p = X(3) / 35 / (t * t) - X(32) / 5 +
                    t * (X(256) / 5 + t * (-96 + t * (X(256) / 5 + t * (32 + t * (X(-1536) / 35 + t * (X(64) / 5))))));
        return p / (b * b * r);
    };
    if (r >= b_pp && 2 * r >= bf) {
        // r^3 g = q^5 Q(q), q = 1 - r/b_f, and b_f^2 - r^2 = q b_f (b_f + r)
        const X q = 1 - r / bf;
        const X Q = X(1344) / 35 + q * (X(-2912) / 35 + q * (X(2048) / 35 + q * (X(-64) / 5)));
        const X u = bf * (bf + r);
        return Q / (r * r * r * u * u * u * u * u);
    }
    const X w = bf * bf - r * r;
    return (r_over_r(b_pp) - r_over_r(bf)) / (w * w * w * w * w);
}

// A table of H = g / w^4 = h b_f^10 w, w = 1 - s/b_f^2, by s = r^2 (see the
// comments above pair_accumulate and pair_adjoint): row t covers s in
// [2^e (1 + i/2^mb), 2^e (1 + (i+1)/2^mb)) with (e + 127) 2^mb + i = t + row0,
// and holds the polynomial of degree D-1 in z in [0, 2^-mb) through H at the
// D Chebyshev nodes, solved in FP64 in the variable y = 2^mb z and rescaled.  Built from
// eq. (2) directly (extended precision), independent of the r grid; rows
// beyond the cutoff are zero.
void fit_h_rows(const cube2_ctx *ctx, int mb, int D, int row0, int nrows, int row_floats,
                std::vector<float> &out) {
    const double pi = 3.14159265358979323846, bf = ctx->cfg.b_fine;
    const long double bf10 = std::pow((long double)bf, 10);  // rows hold H = h b_f^10 w
    std::vector<double> yn(D);
    for (int j = 0; j < D; ++j) yn[j] = 0.5 + 0.5 * std::cos(pi * (j + 0.5) / D);
    out.assign((size_t)nrows * row_floats, 0.0f);
    for (int t = 0; t < nrows; ++t) {
        const int e = ((t + row0) >> mb) - 127, i = (t + row0) & ((1 << mb) - 1);
        const double scale = std::ldexp(1.0, e), inv = 1.0 / (1 << mb);
        if (scale * (1.0 + i * inv) >= bf * bf) continue;  // beyond the cutoff: h = 0
        double A[8][9];
        for (int j = 0; j < D; ++j) {
            const double sv = scale * (1.0 + (i + yn[j]) * inv);
            double p = 1.0;
            for (int k = 0; k < D; ++k, p *= yn[j]) A[j][k] = p;
            const long double w = 1.0L - (long double)sv / ((long double)bf * bf);
            A[j][D] = (double)(pair_h_direct(ctx->cfg.b_pp, bf, std::sqrt(sv)) * bf10 * w);
        }
        for (int c = 0; c < D; ++c) {  // Gauss-Jordan, partial pivoting
            int pv = c;
            for (int r = c + 1; r < D; ++r)
                if (std::fabs(A[r][c]) > std::fabs(A[pv][c])) pv = r;
            for (int k = 0; k <= D; ++k) std::swap(A[c][k], A[pv][k]);
            for (int r = 0; r < D; ++r) {
                if (r == c) continue;
                const double f = A[r][c] / A[c][c];
                for (int k = c; k <= D; ++k) A[r][k] -= f * A[c][k];
            }
        }
        double p = 1.0;
        for (int k = 0; k < D; ++k, p *= (1 << mb))
            out[(size_t)t * row_floats + k] = (float)(A[k][D] / A[k][k] * p);
    }
}

}  // namespace

// The pair-law tables (see the comment above pair_accumulate).  Returns
// nonzero when no K <= kPairKMax puts b_pp/2, b_pp and b_f/2 on interval
// edges (the pieces would then straddle a breakpoint of eq. 2).
int build_pair_table(cube2_ctx *ctx) {
    static const double a[6] = {64.0 / 5, 0.0, -256.0 / 5, 32.0, 1536.0 / 35, -192.0 / 5};
    static const double c[6] = {256.0 / 5, -96.0, 256.0 / 5, 32.0, -1536.0 / 35, 64.0 / 5};
    const double bpp = ctx->cfg.b_pp, bf = ctx->cfg.b_fine;
    // smallest K with b_pp/2, b_pp and b_f/2 on interval edges
    int K = 0;
    for (int k = 1; k <= kPairKMax; ++k) {
        const double w = bf / k;
        bool ok = true;
        for (double b : {bpp / 2, bpp, bf / 2}) {
            const double q = b / w;
            if (std::fabs(q - std::nearbyint(q)) > 1e-9 * std::max(1.0, q)) ok = false;
        }
        if (ok) { K = k; break; }
    }
    if (K == 0) return 1;
    const double w = bf / K;
    ctx->pp_K = K;
    ctx->pp_kinv = (float)(K / bf);
    // -1/b_f^2 rounded away from zero: s * (-negc) >= 1 whenever s >= b_f^2
    float cinv = (float)(1.0 / (bf * bf));
    if ((double)cinv < 1.0 / (bf * bf)) cinv = std::nextafter(cinv, 2.0f * cinv);
    ctx->pp_negc = -cinv;
    ctx->pp_rows64.assign((size_t)(K + 1) * kPairRow, 0.0);
    for (int k = 0; k < K; ++k) {
        const double mid = (k + 0.5) * w, rl = k * w, rr = (k + 1) * w;
        const int pb = mid < bpp / 2 ? 0 : (mid < bpp ? 1 : 2);  // in, out, Newtonian
        const int fb = mid < bf / 2 ? 0 : 1;                      // in, out
        double P[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Q[9];
        double ya, yb;
        if (pb == 2 && fb == 1) {
            // r^3 g = s^5 Q(1-s) = s^5 (1344/35 - 2912/35 s + 2048/35 s^2 - 64/5 s^3),
            // s = (b_f - r)/b_f = (b_f - rr)/b_f + (w/b_f) y, y = 1 - fract
            P[5] = 1344.0 / 35;
            P[6] = -2912.0 / 35;
            P[7] = 2048.0 / 35;
            P[8] = -64.0 / 5;
            compose(P, (bf - rr) / bf, w / bf, Q);
            ya = 1.0;
            yb = -1.0;
        } else {
            auto add = [&](int br, double b, double sg) {
                if (br == 0) {
                    for (int i = 0; i < 6; ++i) P[i + 3] += sg * a[i] * std::pow(b, -3 - i);
                } else if (br == 1) {
                    P[0] += sg * 3.0 / 35;
                    P[2] += sg * (-32.0 / 5) / (b * b);
                    for (int i = 0; i < 6; ++i) P[i + 3] += sg * c[i] * std::pow(b, -3 - i);
                } else {
                    P[0] += sg;
                }
            };
            add(pb, bpp, 1.0);
            add(fb, bf, -1.0);
            compose(P, rl, w, Q);  // r = rl + w y, y = fract
            ya = 0.0;
            yb = 1.0;
        }
        double *row64 = &ctx->pp_rows64[(size_t)k * kPairRow];
        for (int j = 0; j < 9; ++j) row64[j] = Q[j];
        row64[9] = ya;
        row64[10] = yb;
    }
    fit_h_rows(ctx, kSMantBits, 4, kSRow0, kSRows, 4, ctx->pp_srows);
    return 0;
}

namespace {

template <bool ADJ, int H>
int launch_pp_kernel_h(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                     const float *abar, float *out, int accumulate, unsigned char *work,
                     const WorkLayout &L, hipStream_t s, float grid_frac,
                     const uint8_t *skip) {
    const float4 *table = reinterpret_cast<const float4 *>(ctx->tables + ctx->pp_soff);
    const int nt = ctx->nt;
    const int ntiles = nt * nt * nt;
    int r = launch_order_tiles(ctx, cs, work, L, s);
    if (r) return r;
    const uint32_t *order = tile_order_ptr(work, L);
    uint32_t *queue = tile_queue_ptr(ctx, work, L);
    auto k = pp_kernel<ADJ, H>;
    const int nsplit = split_parts<H>() > 1 ? std::min(kSplitTiles, ntiles) : 0;
    const int nitems = ntiles + nsplit * (split_parts<H>() - 1);
    const unsigned grid = std::max(
        1u, (unsigned)((float)persistent_grid(k, PPGeo<ADJ, H>::BLOCK, nitems) * grid_frac));
    k<<<grid, PPGeo<ADJ, H>::BLOCK, 0, s>>>(
        pos, cs, (int)n, nt, table, ctx->pp_negc,
        (float)(ctx->cfg.g_newton * ctx->cfg.m_p), abar, out, accumulate, order, queue, ntiles,
        nsplit, skip);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

template <bool ADJ>
int launch_pp_kernel(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                     const float *abar, float *out, int accumulate, unsigned char *work,
                     const WorkLayout &L, hipStream_t s, float grid_frac = 1.0f,
                     const uint8_t *skip = nullptr) {
    if (ctx->pp_halo == 1)
        return launch_pp_kernel_h<ADJ, 1>(ctx, pos, cs, n, abar, out, accumulate, work, L, s,
                                          grid_frac, skip);
    return launch_pp_kernel_h<ADJ, 2>(ctx, pos, cs, n, abar, out, accumulate, work, L, s,
                                      grid_frac, skip);
}

__global__ void add3_kernel(float *__restrict__ acc, const float *__restrict__ b, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) acc[i] = acc[i] + b[i];
}

// The same sum four floats at a time (both arrays 16-byte aligned, m4 = m / 4).
__global__ void add3_kernel4(float4 *__restrict__ acc, const float4 *__restrict__ b, int64_t m4) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m4) {
        const float4 x = acc[i], y = b[i];
        acc[i] = make_float4(x.x + y.x, x.y + y.y, x.z + y.z, x.w + y.w);
    }
}

// Share of the persistent PP grid when the PM force runs beside it: the PM
// kernels take the freed workgroup slots, and the memory-bound PM and the
// VALU-bound PP then overlap on the same CUs.
constexpr float kPPConcurrentFrac = 0.75f;
// ... on meshes of fewer than 64^3 tiles (256^3 particles on a 512^3 mesh),
// where the PM part is a smaller share of the step and the PP has fewer
// tiles per workgroup, the whole grid (measured: 7.08 ms, against 7.19 at
// 7/8 and 7.46 at 3/4).
constexpr int kPPConcurrentFullBelowNt = 64;
// With the two-cell reach (b_f > 2) the PP has ~5x the pairs and the PM part
// fits in what the PP leaves: the full grid (measured at b_f = 3.5 on 512^3
// particles: 89.9 ms, against 91.9 at 7/8, 104.7 at 3/4 and 98.4 with PM and
// PP one after the other).
constexpr float kPPConcurrentFracH2 = 1.0f;
// The same for the PP adjoint beside the PM adjoint (1024-thread workgroups,
// one per CU): measured on 512^3 particles, 5/8 of the CUs gave the shortest
// force adjoint (106.0 ms; 3/4 107.6, 7/8 106.7, all 110.5, 9/16 110.6).
constexpr float kPPAdjConcurrentFrac = 0.625f;
// ... and on meshes of fewer than 64^3 tiles, 7/8 (measured on 256^3
// particles: force adjoint 14.2 ms, against 14.3 with the whole grid and
// 17.6 at 5/8).
constexpr float kPPAdjConcurrentFracSmall = 0.875f;
// ... and with the two-cell reach, 7/8 (measured at b_f = 3.5 on 512^3
// particles: 212.5 ms, against 214.9 with the full grid, 280.0 at 5/8 and
// 226.7 with PM and PP adjoints one after the other).
constexpr float kPPAdjConcurrentFracH2 = 0.875f;

}  // namespace

// PP force (abar == nullptr) or its adjoint for the cotangents abar into
// acc_pp (not accumulated) with its own tile order and work counter (the
// pp_order / pp_hist / pp_scan regions), so that it can run on another stream
// while the PM part uses the shared ones.
int launch_pp_concurrent(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                         const float *abar, float *acc_pp, unsigned char *work, const WorkLayout &L,
                         hipStream_t s) {
    WorkLayout Lpp = L;
    Lpp.tile_order = L.pp_order;
    Lpp.hist = L.pp_hist;
    Lpp.scan_tmp = L.pp_scan;
    const bool small = ctx->nt < kPPConcurrentFullBelowNt;
    if (abar)
        return launch_pp_kernel<true>(ctx, pos, cs, n, abar, acc_pp, 0, work, Lpp, s,
                                      ctx->pp_halo != 1 ? kPPAdjConcurrentFracH2
                                      : small           ? kPPAdjConcurrentFracSmall
                                                        : kPPAdjConcurrentFrac);
    const float frac = ctx->pp_halo != 1 ? kPPConcurrentFracH2
                       : small           ? 1.0f
                                         : kPPConcurrentFrac;
    return launch_pp_kernel<false>(ctx, pos, cs, n, nullptr, acc_pp, 0, work, Lpp, s, frac);
}

int launch_add3(float *acc, const float *acc_pp, int64_t m, hipStream_t s) {
    if (m <= 0) return CUBE2_OK;
    int64_t done = 0;
    if ((((uintptr_t)acc | (uintptr_t)acc_pp) & 15u) == 0 && m >= 4) {
        const int64_t m4 = m / 4;
        add3_kernel4<<<(unsigned)((m4 + 255) / 256), 256, 0, s>>>(
            reinterpret_cast<float4 *>(acc), reinterpret_cast<const float4 *>(acc_pp), m4);
        done = 4 * m4;
    }
    if (m > done)
        add3_kernel<<<(unsigned)((m - done + 255) / 256), 256, 0, s>>>(acc + done, acc_pp + done,
                                                                       m - done);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

int launch_pp(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n, float *acc,
              int accumulate, unsigned char *work, const WorkLayout &L, hipStream_t s,
              const uint8_t *skip) {
    return launch_pp_kernel<false>(ctx, pos, cs, n, nullptr, acc, accumulate, work, L, s, 1.0f,
                                   skip);
}

int launch_pp_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                       const float *acc_bar, float *x_bar, int accumulate, unsigned char *work,
                       const WorkLayout &L, hipStream_t s) {
    return launch_pp_kernel<true>(ctx, pos, cs, n, acc_bar, x_bar, accumulate, work, L, s);
}

}  // namespace cube2

extern "C" int cube2_pair_law_f32(const cube2_ctx *ctx, const float *d, float *g, int64_t n) {
    using namespace cube2;
    if (!ctx || n < 0 || (n > 0 && (!d || !g))) return CUBE2_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        const float dx = d[i], dy = d[n + i], dz = d[2 * n + i];
        // the staged box's reach: below 2 (halo + 1) fine cells per axis
        const float lim = 2.0f * (float)(ctx->pp_halo + 1);
        if (!(std::fabs(dx) < lim && std::fabs(dy) < lim && std::fabs(dz) < lim))
            return CUBE2_EINVAL;
        // the operations of pair_accumulate, in the same order
        const float s = std::fmaf(dz, dz, std::fmaf(dy, dy, std::fmaf(dx, dx, 0x1p-31f)));
        uint32_t b;
        std::memcpy(&b, &s, 4);
        const float *c = &ctx->pp_srows[(size_t)((b >> (23 - kSMantBits)) - kSRow0) * 4];
        const uint32_t zb = (b & ((1u << (23 - kSMantBits)) - 1u)) | 0x3F800000u;
        float z;
        std::memcpy(&z, &zb, 4);
        z -= 1.0f;
        const float h = std::fmaf(std::fmaf(std::fmaf(c[3], z, c[2]), z, c[1]), z, c[0]);
        const float w = std::fmin(std::fmax(std::fmaf(s, ctx->pp_negc, 1.0f), 0.0f), 1.0f);
        const float w2 = w * w;
        g[i] = h * (w2 * w2);
    }
    return CUBE2_OK;
}

extern "C" int cube2_pair_jacobian_f32(const cube2_ctx *ctx, const float *d, float *g, float *gs,
                                       int64_t n) {
    using namespace cube2;
    if (!ctx || n < 0 || (n > 0 && (!d || !g || !gs))) return CUBE2_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        const float dx = d[i], dy = d[n + i], dz = d[2 * n + i];
        // the staged box's reach: below 2 (halo + 1) fine cells per axis
        const float lim = 2.0f * (float)(ctx->pp_halo + 1);
        if (!(std::fabs(dx) < lim && std::fabs(dy) < lim && std::fabs(dz) < lim))
            return CUBE2_EINVAL;
        // the operations of pair_adjoint, in the same order
        const float s = std::fmaf(dz, dz, std::fmaf(dy, dy, std::fmaf(dx, dx, 0x1p-31f)));
        uint32_t b;
        std::memcpy(&b, &s, 4);
        const float *c = &ctx->pp_srows[(size_t)((b >> (23 - kSMantBits)) - kSRow0) * 4];
        const uint32_t zb = (b & ((1u << (23 - kSMantBits)) - 1u)) | 0x3F800000u;
        const uint32_t eb = 0x7F800000u - (b & 0x7F800000u);
        float z, inv2e2;
        std::memcpy(&z, &zb, 4);
        std::memcpy(&inv2e2, &eb, 4);
        z -= 1.0f;
        float h = std::fmaf(c[3], z, c[2]);
        float hz = std::fmaf(c[3], z, h);
        h = std::fmaf(h, z, c[1]);
        hz = std::fmaf(hz, z, h);
        h = std::fmaf(h, z, c[0]);
        const float w = std::fmin(std::fmax(std::fmaf(s, ctx->pp_negc, 1.0f), 0.0f), 1.0f);
        const float w2 = w * w;
        g[i] = h * (w2 * w2);
        gs[i] = 0.5f * ((w2 * w) * std::fmaf(hz * inv2e2, w, (8.0f * ctx->pp_negc) * h));
    }
    return CUBE2_OK;
}
