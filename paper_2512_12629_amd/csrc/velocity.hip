// velocity.hip -- IOS velocities (section 2.3): each velocity component is
// stored as a 16-bit integer relative to a bulk velocity field on a mesh.
// The paper defers the conversion to an earlier paper; the codec here is a
// plain linear one:
//   v_bulk(c) = mean velocity of the particles in bulk cell c (FP32),
//   s         = max_i |v_i - v_bulk(c_i)| / 32767 (one global scale, FP32),
//   q_i       = rint((v_i - v_bulk(c_i)) / s)          (int16),
//   decode    : v_i = v_bulk(c_i) + s q_i              (two FP32 roundings),
// so that |decode - v| <= s/2 plus FP32 rounding.  The bulk mesh is the
// coarse PM mesh (cells of coarse_ratio fine cells), or cells of 4 fine cells
// with one level; a bulk cell lies inside one tile, so every tile computes
// the means of its own cells.  The cell sums are exact 64-bit fixed point (a
// scale S = 2^(41 - e) with max|v| < 2^e), so the means are deterministic.
#include <algorithm>

#include "common.hpp"

namespace cube2 {
namespace {

// max |x| over m floats as the bit pattern of a non-negative float; *out
// must be zero on entry
__global__ void vabsmax_kernel(const float *__restrict__ x, int64_t m, unsigned int *out) {
    float v = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        v = fmaxf(v, fabsf(x[i]));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(v));
}

__global__ void vset2_kernel(unsigned int *p) {
    p[0] = 0u;
    p[1] = 0u;
}

// fixed-point scale S = 2^(41 - e) with max|v| < 2^e (1 when max is 0)
__device__ __forceinline__ float vel_scale(unsigned int amax_bits) {
    const float m = __uint_as_float(amax_bits);
    if (!(m > 0.0f) || !(m < 3.0e38f)) return 1.0f;
    int e;
    (void)frexpf(m, &e);
    return ldexpf(1.0f, min(41 - e, 100));
}

// bulk cell of a particle inside its tile: IOS cell u (0..511), offsets o
__host__ __device__ __forceinline__ int bulk_cell(int u, const uint32_t (&o)[3], int shift, int ct) {
    const int fx = 2 * (u & 7) + (int)(o[0] >> 15), fy = 2 * ((u >> 3) & 7) + (int)(o[1] >> 15),
              fz = 2 * (u >> 6) + (int)(o[2] >> 15);
    return ((fz >> shift) * ct + (fy >> shift)) * ct + (fx >> shift);
}

__host__ __device__ __forceinline__ int64_t bulk_index(int tx, int ty, int tz, int lc, int ct, int nb) {
    const int cx = tx * ct + lc % ct, cy = ty * ct + (lc / ct) % ct, cz = tz * ct + lc / (ct * ct);
    return ((int64_t)cz * nb + cy) * nb + cx;
}

// Per tile: cell counts and fixed-point velocity sums of its bulk cells, the
// means written to v_bulk, and max |v - v_bulk| of its particles written to
// tmax[tile] (one global atomic per wave on a single address would
// serialise; the tile maxima are reduced by a second pass).
__global__ __launch_bounds__(kBlock) void vel_bulk_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs, const float *__restrict__ vel,
    int n, int nt, int shift, int nb, const unsigned int *__restrict__ amax,
    float *__restrict__ v_bulk, float *__restrict__ tmax, uint32_t *status) {
    __shared__ float wmax[kBlock / 64];
    __shared__ uint32_t cnt[kTileCells];
    __shared__ unsigned long long sum[3][kTileCells];
    __shared__ float vb[3][kTileCells];
    __shared__ uint32_t cst[kTileCells + 1];
    int tx, ty, tz;
    tile_of_block(blockIdx.x, nt, tx, ty, tz);
    const int tid = threadIdx.x;
    const int ct = kTileFine >> shift;       // bulk cells per tile axis
    const int ncell = ct * ct * ct;
    for (int i = tid; i < ncell; i += kBlock) {
        cnt[i] = 0u;
        sum[0][i] = sum[1][i] = sum[2][i] = 0ull;
    }
    const uint32_t key0 = (uint32_t)((tz * nt + ty) * nt + tx) * kTileCells;
    stage_cell_starts<kBlock>(cst, cs, key0);
    __syncthreads();
    const float S = vel_scale(amax[0]), invS = 1.0f / S;
    const uint32_t p0 = cst[0], p1 = cst[kTileCells];
    // Particles are sorted by IOS cell, so equal bulk cells come in runs of
    // consecutive lanes.  A segmented inclusive scan (exact integer sums)
    // leaves each run's count and sums in its last lane, which adds them:
    // one LDS atomic per run instead of one per particle on a few addresses.
    const int lane = tid & 63;
    for (uint32_t w0 = p0 + (uint32_t)(tid - lane); w0 < p1; w0 += kBlock) {
        const uint32_t p = w0 + (uint32_t)lane;
        const bool valid = p < p1;
        int lc = -1;
        uint32_t c = 0u;
        unsigned long long f[3] = {0ull, 0ull, 0ull};
        if (valid) {
            const int u = seg_search_n<kTileCells>(cst, p);
            uint32_t o[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) o[d] = pos[(int64_t)d * n + p];
            lc = bulk_cell(u, o, shift, ct);
            c = 1u;
#pragma unroll
            for (int d = 0; d < 3; ++d)
                f[d] = (unsigned long long)__float2ll_rn(vel[(int64_t)d * n + p] * S);
        }
        const int lc_up = __shfl_up(lc, 1, 64), lc_dn = __shfl_down(lc, 1, 64);
        int head = (lane == 0 || lc != lc_up) ? 1 : 0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t c_up = __shfl_up(c, off, 64);
            const unsigned long long f0 = __shfl_up(f[0], off, 64), f1 = __shfl_up(f[1], off, 64),
                                     f2 = __shfl_up(f[2], off, 64);
            const int h_up = __shfl_up(head, off, 64);
            if (lane >= off) {
                if (!head) {
                    c += c_up;
                    f[0] += f0;
                    f[1] += f1;
                    f[2] += f2;
                }
                head |= h_up;
            }
        }
        if (valid && (lane == 63 || lc_dn != lc)) {
            atomicAdd(&cnt[lc], c);
#pragma unroll
            for (int d = 0; d < 3; ++d) atomicAdd(&sum[d][lc], f[d]);
        }
    }
    __syncthreads();
    for (int i = tid; i < ncell; i += kBlock) {
        const uint32_t c = cnt[i];
        // 2^22 values below 2^41 each keep the sum within 63 bits
        if (c >= (1u << 22)) atomicOr(status, kStatusOverflow);
        const int64_t g = bulk_index(tx, ty, tz, i, ct, nb);
        const int64_t m3 = (int64_t)nb * nb * nb;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float mean =
                c ? __fdiv_rn(__fmul_rn((float)(long long)sum[d][i], invS), (float)c) : 0.0f;
            vb[d][i] = mean;
            v_bulk[d * m3 + g] = mean;
        }
    }
    __syncthreads();
    float dmax = 0.0f;
    for (uint32_t p = p0 + tid; p < p1; p += kBlock) {
        const int u = seg_search_n<kTileCells>(cst, p);
        uint32_t o[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) o[d] = pos[(int64_t)d * n + p];
        const int lc = bulk_cell(u, o, shift, ct);
#pragma unroll
        for (int d = 0; d < 3; ++d)
            dmax = fmaxf(dmax, fabsf(__fsub_rn(vel[(int64_t)d * n + p], vb[d][lc])));
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, m, 64));
    if ((tid & 63) == 0) wmax[tid >> 6] = dmax;
    __syncthreads();
    if (tid == 0) {
        float b = 0.0f;
        for (int w = 0; w < kBlock / 64; ++w) b = fmaxf(b, wmax[w]);
        tmax[blockIdx.x] = b;
    }
}

// the global scale s = max |v - v_bulk| / 32767 (1 when every deviation is 0)
__device__ __forceinline__ float vel_step(unsigned int dmax_bits) {
    const float m = __uint_as_float(dmax_bits);
    return m > 0.0f ? __fdiv_rn(m, 32767.0f) : 1.0f;
}

// Per tile: q = rint((v - v_bulk) / s) (ENCODE: reads vel_in and amax,
// writes vq_out and v_scale_out) or v = v_bulk + s q (decode: reads vq_in and
// v_scale, writes vel_out).
template <bool ENCODE>
__global__ __launch_bounds__(kBlock) void vel_code_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs, int n, int nt, int shift,
    int nb, const float *__restrict__ v_bulk, const unsigned int *__restrict__ amax,
    const float *__restrict__ vel_in, int16_t *__restrict__ vq_out, float *__restrict__ v_scale_out,
    const float *__restrict__ v_scale, const int16_t *__restrict__ vq_in,
    float *__restrict__ vel_out) {
    __shared__ uint32_t cst[kTileCells + 1];
    int tx, ty, tz;
    tile_of_block(blockIdx.x, nt, tx, ty, tz);
    const int tid = threadIdx.x;
    const int ct = kTileFine >> shift;
    const uint32_t key0 = (uint32_t)((tz * nt + ty) * nt + tx) * kTileCells;
    stage_cell_starts<kBlock>(cst, cs, key0);
    __syncthreads();
    const float s = ENCODE ? vel_step(amax[1]) : v_scale[0];
    if (ENCODE && blockIdx.x == 0 && tid == 0) v_scale_out[0] = s;
    const int64_t m3 = (int64_t)nb * nb * nb;
    for (uint32_t p = cst[0] + tid; p < cst[kTileCells]; p += kBlock) {
        const int u = seg_search_n<kTileCells>(cst, p);
        uint32_t o[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) o[d] = pos[(int64_t)d * n + p];
        const int64_t g = bulk_index(tx, ty, tz, bulk_cell(u, o, shift, ct), ct, nb);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float b = v_bulk[d * m3 + g];
            if (ENCODE) {
                const float r = rintf(__fdiv_rn(__fsub_rn(vel_in[(int64_t)d * n + p], b), s));
                vq_out[(int64_t)d * n + p] = (int16_t)fminf(fmaxf(r, -32767.0f), 32767.0f);
            } else {
                // two roundings, as documented: no contraction into an FMA
#pragma clang fp contract(off)
                const float sq = s * (float)vq_in[(int64_t)d * n + p];
                vel_out[(int64_t)d * n + p] = b + sq;
            }
        }
    }
}

// bulk cells: the coarse mesh's cells, or 4 fine cells with one level
int bulk_shift(const cube2_ctx *ctx) { return ctx->n_levels > 1 ? ctx->lv[1].hshift : 2; }

}  // namespace

int vel_bulk_side(const cube2_ctx *ctx) { return ctx->n_f >> bulk_shift(ctx); }

// The codec's index arithmetic for this context, run on the host with the
// kernels' own functions: every particle position of every IOS cell of a tile
// (offsets at both ends of both fine cells) lands in one of the tile's
// ct^3 <= 512 bulk cells (the LDS arrays), every bulk cell of every tile in
// [0, nb^3) (v_bulk), and the tile maxima fit their work area.
int vel_layout_check(const cube2_ctx *ctx, const WorkLayout &L) {
    const int shift = bulk_shift(ctx), nb = ctx->n_f >> shift, nt = ctx->nt;
    const int ct = kTileFine >> shift;
    if (ct < 1 || ct * ct * ct > kTileCells || (int64_t)nt * ct != nb) return CUBE2_EUNSUPPORTED;
    static const uint32_t offs[4] = {0u, 0x7FFFu, 0x8000u, 0xFFFFu};
    for (int u = 0; u < kTileCells; ++u)
        for (int a = 0; a < 64; ++a) {
            const uint32_t o[3] = {offs[a & 3], offs[(a >> 2) & 3], offs[a >> 4]};
            const int lc = bulk_cell(u, o, shift, ct);
            if (lc < 0 || lc >= ct * ct * ct) return CUBE2_EUNSUPPORTED;
        }
    const int64_t nb3 = (int64_t)nb * nb * nb;
    for (int tz = 0; tz < nt; ++tz)
        for (int ty = 0; ty < nt; ++ty)
            for (int tx = 0; tx < nt; ++tx)
                for (int lc = 0; lc < ct * ct * ct; ++lc) {
                    const int64_t g = bulk_index(tx, ty, tz, lc, ct, nb);
                    if (g < 0 || g >= nb3) return CUBE2_EUNSUPPORTED;
                }
    const size_t ntiles = (size_t)nt * nt * nt;
    if (L.vel_tmax + ntiles * sizeof(float) > L.total) return CUBE2_EWORKSPACE;
    return CUBE2_OK;
}

int launch_vel_encode(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                      const float *vel, int16_t *vq, float *v_bulk, float *v_scale,
                      unsigned char *work, const WorkLayout &L, hipStream_t s) {
    const int nt = ctx->nt;
    const unsigned blocks = (unsigned)(nt * nt * nt);
    const int shift = bulk_shift(ctx), nb = ctx->n_f >> shift;
    unsigned int *amax = reinterpret_cast<unsigned int *>(work + L.red);
    vset2_kernel<<<1, 1, 0, s>>>(amax);
    CUBE2_LAUNCH_CHECK();
    if (n > 0) {
        const int64_t m3 = 3 * n;
        const unsigned gb = (unsigned)std::min<int64_t>(4096, (m3 + 255) / 256);
        vabsmax_kernel<<<gb, 256, 0, s>>>(vel, m3, amax);
        CUBE2_LAUNCH_CHECK();
    }
    // per-tile maxima in their own work area (one float per tile)
    float *tmax = reinterpret_cast<float *>(work + L.vel_tmax);
    vel_bulk_kernel<<<blocks, kBlock, 0, s>>>(pos, cs, vel, (int)n, nt, shift, nb, amax, v_bulk, tmax,
                                              status_word(ctx));
    CUBE2_LAUNCH_CHECK();
    vabsmax_kernel<<<(unsigned)std::min<int64_t>(1024, ((int64_t)blocks + 255) / 256), 256, 0, s>>>(
        tmax, (int64_t)blocks, amax + 1);
    CUBE2_LAUNCH_CHECK();
    vel_code_kernel<true><<<blocks, kBlock, 0, s>>>(pos, cs, (int)n, nt, shift, nb, v_bulk, amax,
                                                    vel, vq, v_scale, nullptr, nullptr, nullptr);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

int launch_vel_decode(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                      const int16_t *vq, const float *v_bulk, const float *v_scale, float *vel,
                      hipStream_t s) {
    if (n == 0) return CUBE2_OK;
    const int nt = ctx->nt;
    const unsigned blocks = (unsigned)(nt * nt * nt);
    const int shift = bulk_shift(ctx), nb = ctx->n_f >> shift;
    vel_code_kernel<false><<<blocks, kBlock, 0, s>>>(pos, cs, (int)n, nt, shift, nb, v_bulk, nullptr,
                                                     nullptr, nullptr, nullptr, v_scale, vq, vel);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

}  // namespace cube2
