// pp.hip -- the short-range particle-particle force (eq. 4d): for every pair
// closer than the fine softening b_f (the cutoff of the finest PM level),
//   a_i += G m [R(r, b_pp) - R(r, b_f)] (x_j - x_i) / r,
// with R of eq. (2).  Because b_f <= 2 fine cells = one IOS cell, every pair
// lies in the same or in adjacent IOS cells, so the cell-sorted particle
// order is the linked list of the paper (section 2.3).
//
// One workgroup per tile.  The particles of the tile and of its one-cell halo
// (a 10^3 box of IOS cells) are staged in LDS as FP32 positions relative to
// the tile origin in fine cells.  Offsets are multiples of 2^-15 below 2^5,
// so these floats and their differences are exact: the pair separation is
// the exact integer one.  Each thread takes one particle of the tile and
// loops over its 27 neighbour cells; neighbours in a dense cell are read by
// all lanes of a wave at the same LDS address (a broadcast).  Per neighbour
// cell the pair sum is accumulated in FP32 and then added to the total with
// Kahan compensation.  Boxes too large for LDS read the same data from HBM.
#include "common.hpp"

namespace cube2 {
namespace {

constexpr int kPB = kTileIos + 2;          // 10 IOS cells per axis
constexpr int kPSegs = kPB * kPB * kPB;    // 1000
constexpr int kPSegPerThread = (kPSegs + kBlock - 1) / kBlock;  // 4
constexpr int kCap = 3072;                 // staged particles (48 KB)

struct PairLaw {
    // R(r,b)/r in terms of t = r/b:  b^-3 F(t) with
    //   F_in(t)  = 64/5 - 256/5 t^2 + 32 t^3 + 1536/35 t^4 - 192/5 t^5        (t < 1/2)
    //   F_out(t) = 3/(35 t^3) - 32/(5 t) + 256/5 - 96 t + 256/5 t^2 + 32 t^3
    //              - 1536/35 t^4 + 64/5 t^5                                   (1/2 <= t < 1)
    //   F(t)     = t^-3                                                       (t >= 1)
    float bpp, ibpp, ibpp3;  // b_pp, 1/b_pp, 1/b_pp^3
    float bf, ibf, ibf3, bf2;
};

__device__ __forceinline__ float f_in(float t) {
    const float t2 = t * t;
    return 64.0f / 5.0f + t2 * (-256.0f / 5.0f + t * (32.0f + t * (1536.0f / 35.0f + t * (-192.0f / 5.0f))));
}
__device__ __forceinline__ float f_out(float t, float tinv) {
    const float poly = 256.0f / 5.0f + t * (-96.0f + t * (256.0f / 5.0f + t * (32.0f + t * (-1536.0f / 35.0f + t * (64.0f / 5.0f)))));
    return poly + tinv * (-32.0f / 5.0f + tinv * tinv * (3.0f / 35.0f));
}

// On b_f/2 <= r < b_f with r >= b_pp, g = [1/r^2 - R(r, b_f)] / r vanishes
// like (1 - t)^5 at the cutoff and the difference cancels in FP32.  Dividing
// out the root gives the exact factored form
//   g = b_f^-3 (1 - t)^5 (32/35 + 32/7 t + 704/35 t^2 + 64/5 t^3) / t^3.
__device__ __forceinline__ float tail_poly(float t) {
    return 32.0f / 35.0f + t * (32.0f / 7.0f + t * (704.0f / 35.0f + t * (64.0f / 5.0f)));
}

// g(r) = [R(r,b_pp) - R(r,b_f)] / r for 0 < r < b_f (caller checks the range).
__device__ __forceinline__ float pair_g(float r2, const PairLaw &L) {
    const float rinv = __frsqrt_rn(r2);
    const float r = r2 * rinv;
    const float tf = r * L.ibf;  // < 1
    if (r >= L.bpp) {
        if (tf >= 0.5f) {
            const float s = 1.0f - tf, s2 = s * s, tinv = L.bf * rinv;
            return L.ibf3 * (s2 * s2 * s) * tail_poly(tf) * (tinv * tinv * tinv);
        }
        return rinv * rinv * rinv - f_in(tf) * L.ibf3;
    }
    const float gf = (tf < 0.5f ? f_in(tf) : f_out(tf, L.bf * rinv)) * L.ibf3;
    const float tp = r * L.ibpp;
    const float gp = (tp < 0.5f ? f_in(tp) : f_out(tp, L.bpp * rinv)) * L.ibpp3;
    return gp - gf;
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

__global__ __launch_bounds__(kBlock) void pp_kernel(const uint16_t *__restrict__ pos,
                                                    const uint32_t *__restrict__ cs, int n, int nt,
                                                    PairLaw law, float gm,
                                                    float *__restrict__ acc, int accumulate) {
    __shared__ uint32_t seg_pre[kPSegs + 1];
    __shared__ uint32_t seg_src[kPSegs];
    __shared__ float4 xs[kCap];
    __shared__ uint32_t scan_sh[kBlock / 64 + 1];

    int tx, ty, tz;
    tile_of_block(blockIdx.x, nt, tx, ty, tz);
    const int tid = threadIdx.x;
    const int n_ios = nt * kTileIos;
    const int c0x = tx * kTileIos, c0y = ty * kTileIos, c0z = tz * kTileIos;

    uint32_t cnt[kPSegPerThread], src[kPSegPerThread], sum = 0;
#pragma unroll
    for (int k = 0; k < kPSegPerThread; ++k) {
        const int s = tid * kPSegPerThread + k;
        cnt[k] = 0;
        src[k] = 0;
        if (s < kPSegs) {
            const int bx = s % kPB, by = (s / kPB) % kPB, bz = s / (kPB * kPB);
            const uint32_t key = cell_key(wrapn(c0x + bx - 1, n_ios), wrapn(c0y + by - 1, n_ios),
                                          wrapn(c0z + bz - 1, n_ios), nt);
            src[k] = cs[key];
            cnt[k] = cs[key + 1] - src[k];
        }
        sum += cnt[k];
    }
    uint32_t total;
    uint32_t pre = block_exclusive_scan(sum, scan_sh, total);
#pragma unroll
    for (int k = 0; k < kPSegPerThread; ++k) {
        const int s = tid * kPSegPerThread + k;
        if (s < kPSegs) {
            seg_pre[s] = pre;
            seg_src[s] = src[k];
        }
        pre += cnt[k];
    }
    if (tid == 0) seg_pre[kPSegs] = total;
    __syncthreads();
    const bool staged = total <= (uint32_t)kCap;
    const float inv = 1.0f / 32768.0f;
    if (staged) {
        for (uint32_t v = tid; v < total; v += kBlock) {
            const int s = seg_search(seg_pre, kPSegs, v);
            const uint32_t p = seg_src[s] + (v - seg_pre[s]);
            const int bx = s % kPB, by = (s / kPB) % kPB, bz = s / (kPB * kPB);
            float4 q;
            q.x = (float)(2 * (bx - 1)) + (float)pos[p] * inv;
            q.y = (float)(2 * (by - 1)) + (float)pos[(int64_t)n + p] * inv;
            q.z = (float)(2 * (bz - 1)) + (float)pos[2 * (int64_t)n + p] * inv;
            q.w = 0.0f;
            xs[v] = q;
        }
    }
    __syncthreads();

    // own particles: box cells with b in [1, 9)
    const uint32_t key0 = (uint32_t)((tz * nt + ty) * nt + tx) * kTileCells;
    const uint32_t p0 = cs[key0], p1 = cs[key0 + kTileCells];
    for (uint32_t p = p0 + tid; p < p1; p += kBlock) {
        // the own cell of p: search the own cells' segments (row by row is
        // not contiguous in the box), using the tile's cell_start directly
        int lo = 0, hi = kTileCells;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cs[key0 + mid] <= p) lo = mid; else hi = mid;
        }
        const int bx = (lo & 7) + 1, by = ((lo >> 3) & 7) + 1, bz = (lo >> 6) + 1;
        const float xi = (float)(2 * (bx - 1)) + (float)pos[p] * inv;
        const float yi = (float)(2 * (by - 1)) + (float)pos[(int64_t)n + p] * inv;
        const float zi = (float)(2 * (bz - 1)) + (float)pos[2 * (int64_t)n + p] * inv;
        float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
        for (int nb = 0; nb < 27; ++nb) {
            const int ox = nb % 3 - 1, oy = (nb / 3) % 3 - 1, oz = nb / 9 - 1;
            const int s = ((bz + oz) * kPB + (by + oy)) * kPB + (bx + ox);
            const uint32_t v0 = seg_pre[s], v1 = seg_pre[s + 1];
            float fx = 0.f, fy = 0.f, fz = 0.f;
            for (uint32_t v = v0; v < v1; ++v) {
                float xj, yj, zj;
                if (staged) {
                    const float4 q = xs[v];
                    xj = q.x;
                    yj = q.y;
                    zj = q.z;
                } else {
                    const uint32_t pj = seg_src[s] + (v - v0);
                    xj = (float)(2 * (bx + ox - 1)) + (float)pos[pj] * inv;
                    yj = (float)(2 * (by + oy - 1)) + (float)pos[(int64_t)n + pj] * inv;
                    zj = (float)(2 * (bz + oz - 1)) + (float)pos[2 * (int64_t)n + pj] * inv;
                }
                const float dx = xj - xi, dy = yj - yi, dz = zj - zi;
                const float r2 = dx * dx + dy * dy + dz * dz;
                if (r2 > 0.0f && r2 < law.bf2) {
                    const float g = pair_g(r2, law);
                    fx += g * dx;
                    fy += g * dy;
                    fz += g * dz;
                }
            }
            kahan_add(sx, cx, fx);
            kahan_add(sy, cy, fy);
            kahan_add(sz, cz, fz);
        }
        const float a[3] = {gm * sx, gm * sy, gm * sz};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float *dst = acc + (int64_t)d * n + p;
            *dst = accumulate ? *dst + a[d] : a[d];
        }
    }
}

}  // namespace

int launch_pp(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n, float *acc,
              int accumulate, hipStream_t s) {
    const double bpp = ctx->cfg.b_pp, bf = ctx->cfg.b_fine;
    PairLaw law;
    law.bpp = (float)bpp;
    law.ibpp = (float)(1.0 / bpp);
    law.ibpp3 = (float)(1.0 / (bpp * bpp * bpp));
    law.bf = (float)bf;
    law.ibf = (float)(1.0 / bf);
    law.ibf3 = (float)(1.0 / (bf * bf * bf));
    law.bf2 = (float)(bf * bf);
    const int nt = ctx->nt;
    pp_kernel<<<(unsigned)(nt * nt * nt), kBlock, 0, s>>>(
        pos, cs, (int)n, nt, law, (float)(ctx->cfg.g_newton * ctx->cfg.m_p), acc, accumulate);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

}  // namespace cube2
