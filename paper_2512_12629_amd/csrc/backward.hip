// backward.hip -- adjoints (vector-Jacobian products) of the deposit, the PM
// force and the PP force.  The paper has no adjoint; these follow from the
// forward definitions:
//
// PM, one level of spacing H, c = G m / H^2, unit-mass density rho:
//   a_i = c sum_n W(y_i - n) E(n),  E = -D phi,  phi = K rho,  rho = sum_j W
//   Abar_d(n)  = c sum_i W(y_i - n) abar_{i,d}
//   phibar     = +D . Abar   (the 4-point stencil is antisymmetric: D^T = -D)
//   rhobar     = K phibar    (G real and even: K symmetric; same FFT pipeline)
//   xbar_i    += sum_n grad W(y_i - n) [c abar_i . E(n) + rhobar(n)]
// grad W of the CIC weights is piecewise constant: (1/H) (+-1) times the two
// other weights (left-continuous at cell faces).  With TSC assignment (eq. 5,
// context flag CUBE2_ASSIGN_TSC) the weights are the forward's 16-bit ones
// and their slopes those of eq. 5 at the offset d from the nearest node:
// -(1/2 - d), -2d, 1/2 + d (1/H), the rounding taken as the identity.
//
// The scatters of c*abar onto the meshes accumulate in LDS in 64-bit fixed
// point (integer LDS atomics are an order of magnitude faster than FP32 ones
// on gfx950, and integer sums are exact and order independent): a
// contribution v becomes rint(v S) with S = 2^(41 - e), 2^e > c max|abar|, so
// a node can take 2^21 contributions before its sum could leave 63 bits.
//
// The PP adjoint lives with the PP kernel (pp.hip).
#include <algorithm>

#include "common.hpp"

namespace cube2 {
namespace {

// max |x| over m floats as the bit pattern of a non-negative float (which
// orders like the float); *out must be zero on entry
__global__ void absmax_kernel(const float *__restrict__ x, int64_t m, unsigned int *out) {
    float v = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        v = fmaxf(v, fabsf(x[i]));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(v));
}

__global__ void set_u32(unsigned int *p, unsigned int v) { *p = v; }

// fixed-point scale S = 2^(41 - e) with c * max|abar| < 2^e
__device__ __forceinline__ float fixed_scale(const unsigned int *amax_bits, float c) {
    const float m = __uint_as_float(*amax_bits) * fabsf(c);
    if (!(m > 0.0f) || !(m < 3.0e38f)) return 1.0f;
    int e;
    (void)frexpf(m, &e);
    return ldexpf(1.0f, min(41 - e, 100));
}

// rint(v) as a 64-bit two's-complement integer (half to even), |v| < 2^51:
// v is exact in FP64, adding 1.5 * 2^52 rounds it to an integer and leaves
// that integer in the low mantissa bits, and the exponent bits cancel in the
// difference of the two bit patterns.  Four instructions instead of the
// eleven of a float-to-int64 conversion; the same integer.
__device__ __forceinline__ unsigned long long to_fixed(float v) {
    const double m = 6755399441055744.0;   // 1.5 * 2^52
    const double t = (double)v + m;
    return (unsigned long long)(__double_as_longlong(t) - __double_as_longlong(m));
}

// A fixed-point difference to FP32 through FP64: 5 instructions instead of
// the 12 of a direct int64-to-float conversion, and the same float while
// |d| < 2^53 (the FP64 step is then exact; node sums stay far below that).
__device__ __forceinline__ float fixed_to_float(long long d) { return (float)(double)d; }

// ---------------------------------------------------------------------------
// fine level: phibar on a 16^3 node tile.  For each component d in turn, the
// workgroup scatters c*abar_d with the CIC weights onto the nodes of the
// tile plus a 2-node halo (20^3 nodes, fixed point in LDS), from every
// particle whose CIC footprint reaches that region (an 11^3 box of IOS cells:
// a particle in fine cell j feeds nodes j and j+1), then adds the d term of
// the stencil transpose phibar = D . Abar on the 16^3 interior.
// ---------------------------------------------------------------------------

constexpr int kAN = kTileFine + 4;           // 20 nodes per axis: [a0-2, a0+18)
constexpr int kAN3 = kAN * kAN * kAN;
constexpr int kPhiBlock = 512;
// IOS cells per axis whose particles reach the 20^3 nodes: [c0-2, c0+9) for
// CIC, [c0-2, c0+10) for TSC (a particle in fine cell j feeds j-1 .. j+2)
// LUT: staged particles whose box cell is looked up once per tile (not in
// each of the three passes), as many as fit beside the rest at two
// workgroups per CU
template <int P> struct PhiGeo {
    static constexpr int AB = kTileIos + (P == 3 ? 4 : 3);   // 11 or 12
    static constexpr int SEGS = AB * AB * AB;
    static constexpr int SEG_PER_THREAD = (SEGS + kPhiBlock - 1) / kPhiBlock;
    static constexpr int LUT = P == 3 ? 1984 : 3584;
};

template <int P>
__global__ __launch_bounds__(kPhiBlock) void fine_phibar_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs,
    const float *__restrict__ abar, int n, int n_f, int nt, float c,
    const unsigned int *__restrict__ amax_bits, float *__restrict__ phibar) {
    constexpr int kAB = PhiGeo<P>::AB, kASegs = PhiGeo<P>::SEGS;
    constexpr int kASegPerThread = PhiGeo<P>::SEG_PER_THREAD;
    __shared__ uint32_t seg_pre[kASegs + 1];
    __shared__ uint32_t seg_src[kASegs];
    __shared__ unsigned long long A[kAN3];   // one component at a time, fixed point
    __shared__ uint32_t scan_sh[kPhiBlock / 64 + 1];
    __shared__ uint16_t lut[PhiGeo<P>::LUT];   // box cell of each staged particle
    int tx, ty, tz;
    tile_of_block(blockIdx.x, nt, tx, ty, tz);
    const int tid = threadIdx.x;
    const int n_ios = nt * kTileIos;
    const int c0x = tx * kTileIos, c0y = ty * kTileIos, c0z = tz * kTileIos;
    uint32_t cnt[kASegPerThread], src[kASegPerThread], sum = 0;
#pragma unroll
    for (int k = 0; k < kASegPerThread; ++k) {
        const int s = tid * kASegPerThread + k;
        cnt[k] = 0;
        src[k] = 0;
        if (s < kASegs) {
            const int bx = s % kAB, by = (s / kAB) % kAB, bz = s / (kAB * kAB);
            const uint32_t key = cell_key(wrapn(c0x + bx - 2, n_ios), wrapn(c0y + by - 2, n_ios),
                                          wrapn(c0z + bz - 2, n_ios), nt);
            src[k] = cs[key];
            cnt[k] = cs[key + 1] - src[k];
        }
        sum += cnt[k];
    }
    uint32_t total;
    uint32_t pre = block_exclusive_scan<kPhiBlock>(sum, scan_sh, total);
#pragma unroll
    for (int k = 0; k < kASegPerThread; ++k) {
        const int s = tid * kASegPerThread + k;
        if (s < kASegs) {
            seg_pre[s] = pre;
            seg_src[s] = src[k];
        }
        pre += cnt[k];
    }
    if (tid == 0) seg_pre[kASegs] = total;
    // the box cell of every staged particle, searched once for the three passes
    const bool use_lut = total <= (uint32_t)PhiGeo<P>::LUT;   // block-uniform
    __syncthreads();
    if (use_lut)
        for (uint32_t v = tid; v < total; v += kPhiBlock) lut[v] = (uint16_t)seg_search_n<kASegs>(seg_pre, v);
    const float S = fixed_scale(amax_bits, c), invS = 1.0f / S;
    const float cS = c * S;
    const float inv = 1.0f / 32768.0f;
    constexpr int T = kTileFine;
    constexpr int NPT = T * T * T / kPhiBlock;   // interior nodes per thread
    float out[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) out[k] = 0.0f;
    // phibar(m) = sum_d (2/3)(A_d(m+e_d) - A_d(m-e_d)) - (1/12)(A_d(m+2e_d) - A_d(m-2e_d)),
    // one component d per pass
    for (int d = 0; d < 3; ++d) {
        for (int i = tid; i < kAN3; i += kPhiBlock) A[i] = 0ull;
        __syncthreads();
        constexpr int kBatch = 2;
        for (uint32_t v0 = tid; v0 < total; v0 += kPhiBlock * kBatch) {
            int sg[kBatch];
            uint32_t o[kBatch][3];
            float ab[kBatch];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                // looked up for every lane (past the end: the last particle,
                // total >= 1 here) so that the lookups of the batch interleave
                const uint32_t v = v0 + k * kPhiBlock, vv = v < total ? v : total - 1;
                const int u = use_lut ? (int)lut[vv] : seg_search_n<kASegs>(seg_pre, vv);
                sg[k] = v < total ? u : -1;
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                if (sg[k] < 0) continue;
                const uint32_t p = seg_src[sg[k]] + (v0 + k * kPhiBlock - seg_pre[sg[k]]);
#pragma unroll
                for (int e = 0; e < 3; ++e) o[k][e] = pos[(int64_t)e * n + p];
                ab[k] = cS * abar[(int64_t)d * n + p];
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                if (sg[k] < 0) continue;
                const int s = sg[k];
                const int b[3] = {s % kAB, (s / kAB) % kAB, s / (kAB * kAB)};
                int j[3];          // first node of the footprint in the 20^3 box
                float w[3][P];
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    j[e] = 2 * (b[e] - 2) + (int)(o[k][e] >> 15) + 2;  // fine cell's node
                    const int f = (int)(o[k][e] & 0x7FFFu);
                    if constexpr (P == 3) {
                        j[e] += tsc_axis<float>(f, w[e]) - 1;
                    } else {
                        w[e][1] = (float)f * inv;
                        w[e][0] = (float)(32768 - f) * inv;
                    }
                }
#pragma unroll
                for (int sz = 0; sz < P; ++sz)
#pragma unroll
                    for (int sy = 0; sy < P; ++sy) {
                        const int nz = j[2] + sz, ny = j[1] + sy;
                        if ((unsigned)nz >= (unsigned)kAN || (unsigned)ny >= (unsigned)kAN) continue;
                        const float wyz = w[1][sy] * w[2][sz] * ab[k];
                        // row of the node line, as two small products (24-bit
                        // multiplies; a product of the sum is a 32-bit one)
                        const int row = nz * (kAN * kAN) + ny * kAN;
#pragma unroll
                        for (int sx = 0; sx < P; ++sx) {
                            const int nx = j[0] + sx;
                            if ((unsigned)nx >= (unsigned)kAN) continue;
                            atomicAdd(&A[row + nx], to_fixed(wyz * w[0][sx]));
                        }
                    }
            }
        }
        __syncthreads();
        const int st = d == 0 ? 1 : (d == 1 ? kAN : kAN * kAN);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int i = tid + k * kPhiBlock;
            const int lx = i % T, ly = (i / T) % T, lz = i / (T * T);
            const int m = ((lz + 2) * kAN + ly + 2) * kAN + lx + 2;
            const long long d1 = (long long)(A[m + st] - A[m - st]);
            const long long d2 = (long long)(A[m + 2 * st] - A[m - 2 * st]);
            out[k] += invS * ((2.0f / 3.0f) * fixed_to_float(d1) - (1.0f / 12.0f) * fixed_to_float(d2));
        }
        __syncthreads();  // the next pass clears A
    }
    // node i = tid + k kPhiBlock: the same (x, y) for every k, z advancing by
    // kPhiBlock / T^2 layers per k
    static_assert(kPhiBlock % (T * T) == 0, "whole z-layers per step");
    const int a0x = tx * T, a0y = ty * T, a0z = tz * T;
    const int lx = tid % T, ly = (tid / T) % T, lz = tid / (T * T);
    float *dst = phibar + ((int64_t)(a0z + lz) * n_f + (a0y + ly)) * n_f + (a0x + lx);
    const int64_t zstep = (int64_t)(kPhiBlock / (T * T)) * n_f * n_f;
#pragma unroll
    for (int k = 0; k < NPT; ++k) dst[k * zstep] = out[k];
}

// ---------------------------------------------------------------------------
// coarse level: CIC scatter of c*abar (3 components) per tile in LDS, added
// in the same fixed point to a 3-component coarse mesh of 64-bit integers
// (exact, so the sum does not depend on the order of the tiles), then the
// stencil transpose on that mesh with one conversion to FP32 per node
// ---------------------------------------------------------------------------

// coarse nodes per axis of a tile's footprint at ratio 2: 9 (CIC), 11 (TSC,
// one more on each side)
template <int P> constexpr int coarse_nodes_max() { return kTileFine / 2 + (P == 3 ? 3 : 1); }

template <int P>
__global__ __launch_bounds__(kBlock) void coarse_abar_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs,
    const float *__restrict__ abar, int n, int nt, int n_c, int hshift, float c,
    const unsigned int *__restrict__ amax_bits, unsigned long long *__restrict__ Amesh) {
    constexpr int kCN = coarse_nodes_max<P>();
    __shared__ unsigned long long A[3][kCN * kCN * kCN];   // fixed point
    __shared__ uint32_t cst[kTileCells + 1];
    int tx, ty, tz;
    tile_of_block(blockIdx.x, nt, tx, ty, tz);
    const int tid = threadIdx.x;
    const int lo = P == 3 ? 1 : 0;                          // footprint starts lo nodes below
    const int NC = (kTileFine >> hshift) + 1 + 2 * lo;
    for (int i = tid; i < 3 * kCN * kCN * kCN; i += kBlock) (&A[0][0])[i] = 0ull;
    const float S = fixed_scale(amax_bits, c);
    const uint32_t key0 = (uint32_t)((tz * nt + ty) * nt + tx) * kTileCells;
    stage_cell_starts<kBlock>(cst, cs, key0);
    __syncthreads();
    const float inv = 1.0f / 32768.0f;
    // Wave-uniform loop over the tile's particles.  An IOS cell lies in one
    // coarse cell, so in a dense cell all lanes feed the same 8 nodes: the 24
    // weighted values are then summed over the wave (fixed order) and one
    // lane adds them, instead of 64 lanes contending for each address.
    const int lane = tid & 63;
    const uint32_t pbeg = cst[0], pend = cst[kTileCells];
    for (uint32_t w0 = pbeg + (uint32_t)(tid - lane); w0 < pend; w0 += kBlock) {
        const uint32_t p = w0 + lane;
        const bool valid = p < pend;
        int j[3] = {0, 0, 0};   // first footprint node, tile-footprint coordinates
        float w[3][P] = {}, ab[3] = {0.f, 0.f, 0.f};
        if (valid) {
            const int u = seg_search_n<kTileCells>(cst, p);
            const int uc[3] = {u & 7, (u >> 3) & 7, u >> 6};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const uint32_t q = ((uint32_t)uc[d] << 16) + pos[(int64_t)d * n + p];
                j[d] = (int)(q >> (kFracBits + hshift));
                const int f = (int)((q >> hshift) & 0x7FFFu);
                if constexpr (P == 3) {
                    j[d] += tsc_axis<float>(f, w[d]);   // n0 - 1 + lo
                } else {
                    w[d][1] = (float)f * inv;
                    w[d][0] = (float)(32768 - f) * inv;
                }
                ab[d] = c * S * abar[(int64_t)d * n + p];
            }
        }
        const int key = valid ? (j[2] * NC + j[1]) * NC + j[0] : -1;
        const unsigned long long vm = __ballot(valid);
        const int lead = first_lane(vm);
        const int key0 = __builtin_amdgcn_readlane(key, lead);
        const bool uniform = __ballot(valid && key != key0) == 0ull;
#pragma unroll
        for (int sz = 0; sz < P; ++sz)
#pragma unroll
            for (int sy = 0; sy < P; ++sy)
#pragma unroll
                for (int sx = 0; sx < P; ++sx) {
                    const float W = w[0][sx] * w[1][sy] * w[2][sz];
                    const int off = (sz * NC + sy) * NC + sx;
                    const unsigned long long q0 = to_fixed(W * ab[0]), q1 = to_fixed(W * ab[1]),
                                             q2 = to_fixed(W * ab[2]);
                    if (uniform) {
                        const unsigned long long t0 = wave_sum(q0), t1 = wave_sum(q1),
                                                 t2 = wave_sum(q2);
                        if (lane == lead) {
                            atomicAdd(&A[0][key0 + off], t0);
                            atomicAdd(&A[1][key0 + off], t1);
                            atomicAdd(&A[2][key0 + off], t2);
                        }
                    } else if (valid) {
                        atomicAdd(&A[0][key + off], q0);
                        atomicAdd(&A[1][key + off], q1);
                        atomicAdd(&A[2][key + off], q2);
                    }
                }
    }
    __syncthreads();
    const int A0x = ((tx * kTileFine) >> hshift) - lo, A0y = ((ty * kTileFine) >> hshift) - lo,
              A0z = ((tz * kTileFine) >> hshift) - lo;
    const int64_t m = (int64_t)n_c * n_c * n_c;
    for (int i = tid; i < NC * NC * NC; i += kBlock) {
        const int lx = i % NC, ly = (i / NC) % NC, lz = i / (NC * NC);
        const int64_t g = ((int64_t)wrapn(A0z + lz, n_c) * n_c + wrapn(A0y + ly, n_c)) * n_c +
                          wrapn(A0x + lx, n_c);
        for (int d = 0; d < 3; ++d) {
            const unsigned long long q = A[d][i];
            if (q != 0ull) atomicAdd(&Amesh[d * m + g], q);   // two's complement: exact
        }
    }
}

__global__ void fill_u64(unsigned long long *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// phibar(m) = sum_d (2/3)(A_d(m+e_d) - A_d(m-e_d)) - (1/12)(A_d(m+2e_d) - A_d(m-2e_d))
// on the fixed-point mesh: the differences are exact 64-bit integers, each
// rounded once to FP32 and scaled by 1/S (S of the scatter).
__global__ void divergence_kernel(const unsigned long long *__restrict__ A, int n, float c,
                                  const unsigned int *__restrict__ amax_bits,
                                  float *__restrict__ out) {
    const int64_t m3 = (int64_t)n * n * n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m3) return;
    const float invS = 1.0f / fixed_scale(amax_bits, c);
    const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((int64_t)n * n));
    auto at = [&](int d, int xx, int yy, int zz) {
        return A[d * m3 + ((int64_t)wrapn(zz, n) * n + wrapn(yy, n)) * n + wrapn(xx, n)];
    };
    auto dif = [](unsigned long long a, unsigned long long b) { return fixed_to_float((long long)(a - b)); };
    float s = (2.0f / 3.0f) * dif(at(0, x + 1, y, z), at(0, x - 1, y, z)) -
              (1.0f / 12.0f) * dif(at(0, x + 2, y, z), at(0, x - 2, y, z));
    s += (2.0f / 3.0f) * dif(at(1, x, y + 1, z), at(1, x, y - 1, z)) -
         (1.0f / 12.0f) * dif(at(1, x, y + 2, z), at(1, x, y - 2, z));
    s += (2.0f / 3.0f) * dif(at(2, x, y, z + 1), at(2, x, y, z - 1)) -
         (1.0f / 12.0f) * dif(at(2, x, y, z + 2), at(2, x, y, z - 2));
    out[i] = s * invS;
}

// ---------------------------------------------------------------------------
// xbar gather: sum over the 8 CIC nodes of grad W times
//   T = c (abar . E) + rhobar   (PM adjoint)   or   T = rhobar (deposit adjoint)
// ---------------------------------------------------------------------------

// Staged tiles per level (side S, first node o below the tile origin): the
// potential with the stencil halo and the rhobar nodes of the footprints.
template <int P> struct GatherGeo {
    static constexpr int PLO = P == 3 ? 3 : 2;   // potential: nodes from -PLO
    static constexpr int PX = P == 3 ? 7 : 5;    // potential side = tile nodes + PX
    static constexpr int RLO = P == 3 ? 1 : 0;   // rhobar: nodes from -RLO
    static constexpr int RX = P == 3 ? 3 : 1;    // rhobar side = tile nodes + RX
    static constexpr int FS = kTileFine + PX, RS = kTileFine + RX;
    static constexpr int CSMAX = kTileFine / 2 + PX, CRMAX = kTileFine / 2 + RX;
};

__device__ __forceinline__ float fd_at(const float *P, int idx, int st) {
    return -((2.0f / 3.0f) * (P[idx + st] - P[idx - st]) -
             (1.0f / 12.0f) * (P[idx + 2 * st] - P[idx - 2 * st]));
}

// adds invH sum_s grad W_s T_s to xb; j is the first footprint node (tile
// coordinates), w the weights and dw their slopes in level units
template <bool WITH_E, int P>
__device__ __forceinline__ void level_gather(const float *Pt, int S, const float *Rb, int SR,
                                             const int (&j)[3], const float (&w)[3][P],
                                             const float (&dw)[3][P], const float (&ab)[3],
                                             float c, float invH, float (&xb)[3]) {
    constexpr int PLO = GatherGeo<P>::PLO, RLO = GatherGeo<P>::RLO;
    float g[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int sz = 0; sz < P; ++sz)
#pragma unroll
        for (int sy = 0; sy < P; ++sy)
#pragma unroll
            for (int sx = 0; sx < P; ++sx) {
                float T = Rb[((j[2] + sz + RLO) * SR + j[1] + sy + RLO) * SR + j[0] + sx + RLO];
                if (WITH_E) {
                    const int idx = ((j[2] + sz + PLO) * S + j[1] + sy + PLO) * S + j[0] + sx + PLO;
                    const float ex = fd_at(Pt, idx, 1), ey = fd_at(Pt, idx, S), ez = fd_at(Pt, idx, S * S);
                    T += c * (ab[0] * ex + ab[1] * ey + ab[2] * ez);
                }
                g[0] += dw[0][sx] * w[1][sy] * w[2][sz] * T;
                g[1] += dw[1][sy] * w[0][sx] * w[2][sz] * T;
                g[2] += dw[2][sz] * w[0][sx] * w[1][sy] * T;
            }
    xb[0] += g[0] * invH;
    xb[1] += g[1] * invH;
    xb[2] += g[2] * invH;
}

// weights, slopes and first footprint node of one axis from the 15-bit
// fraction f of the level coordinate whose cell is j
template <int P>
__device__ __forceinline__ int axis_footprint(int j, int f, float (&w)[P], float (&dw)[P]) {
    if constexpr (P == 3) {
        return j + tsc_axis_grad<float>(f, w, dw) - 1;
    } else {
        const float inv = 1.0f / 32768.0f;
        w[1] = (float)f * inv;
        w[0] = (float)(32768 - f) * inv;
        dw[0] = -1.0f;
        dw[1] = 1.0f;
        return j;
    }
}

// HS > 0 fixes log2 of the coarse ratio at compile time (the coarse tiles'
// LDS strides then fold into immediate offsets); HS = 0 reads it from hshift.
template <bool WITH_E, bool TWO, int P, int HS = 0>
__global__ __launch_bounds__(kBlock) void xbar_gather_kernel(
    const uint16_t *__restrict__ pos, const uint32_t *__restrict__ cs,
    const float *__restrict__ abar, int n, int n_f, int nt, const float *__restrict__ phi_f,
    const float *__restrict__ rb_f, float c_f, const float *__restrict__ phi_c,
    const float *__restrict__ rb_c, float c_c, int n_c, int hshift_arg, float *__restrict__ xbar,
    int accumulate) {
    const int hshift = HS > 0 ? HS : hshift_arg;
    using G = GatherGeo<P>;
    constexpr int kFS = G::FS, kRS = G::RS, kCSMax = G::CSMAX, kCRMax = G::CRMAX;
    __shared__ float pf[WITH_E ? kFS * kFS * kFS : 1];
    __shared__ float rf[kRS * kRS * kRS];
    __shared__ float pc[(WITH_E && TWO) ? kCSMax * kCSMax * kCSMax : 1];
    __shared__ float rc[TWO ? kCRMax * kCRMax * kCRMax : 1];
    __shared__ uint32_t cst[kTileCells + 1];
    int tx, ty, tz;
    tile_of_block(blockIdx.x, nt, tx, ty, tz);
    const int tid = threadIdx.x;
    const uint32_t key0 = (uint32_t)((tz * nt + ty) * nt + tx) * kTileCells;
    stage_cell_starts<kBlock>(cst, cs, key0);
    const int a0x = tx * kTileFine, a0y = ty * kTileFine, a0z = tz * kTileFine;
    if (WITH_E) stage_block<kFS, kBlock>(pf, phi_f, n_f, a0x - G::PLO, a0y - G::PLO, a0z - G::PLO);
    if (rb_f) {
        stage_block<kRS, kBlock>(rf, rb_f, n_f, a0x - G::RLO, a0y - G::RLO, a0z - G::RLO);
    } else {
        for (int i = tid; i < kRS * kRS * kRS; i += kBlock) rf[i] = 0.0f;
    }
    const int CS = (kTileFine >> hshift) + G::PX, CR = (kTileFine >> hshift) + G::RX;
    if (TWO) {
        const int cx0 = a0x >> hshift, cy0 = a0y >> hshift, cz0 = a0z >> hshift;
        if (WITH_E)
            for (int i = tid; i < CS * CS * CS; i += kBlock) {
                const int lx = i % CS, ly = (i / CS) % CS, lz = i / (CS * CS);
                pc[i] = phi_c[((int64_t)wrapn(cz0 + lz - G::PLO, n_c) * n_c +
                               wrapn(cy0 + ly - G::PLO, n_c)) * n_c + wrapn(cx0 + lx - G::PLO, n_c)];
            }
        for (int i = tid; i < CR * CR * CR; i += kBlock) {
            const int lx = i % CR, ly = (i / CR) % CR, lz = i / (CR * CR);
            rc[i] = rb_c[((int64_t)wrapn(cz0 + lz - G::RLO, n_c) * n_c +
                          wrapn(cy0 + ly - G::RLO, n_c)) * n_c + wrapn(cx0 + lx - G::RLO, n_c)];
        }
    }
    __syncthreads();
    for (uint32_t p = cst[0] + tid; p < cst[kTileCells]; p += kBlock) {
        const int u = seg_search_n<kTileCells>(cst, p);
        const int uc[3] = {u & 7, (u >> 3) & 7, u >> 6};
        int jf[3], jc[3];
        float wf[3][P], dwf[3][P], wc[3][P], dwc[3][P], ab[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const uint32_t o = pos[(int64_t)d * n + p];
            jf[d] = axis_footprint<P>(2 * uc[d] + (int)(o >> 15), (int)(o & 0x7FFFu), wf[d], dwf[d]);
            ab[d] = WITH_E ? abar[(int64_t)d * n + p] : 0.0f;
            if (TWO) {
                const uint32_t q = ((uint32_t)uc[d] << 16) + o;
                jc[d] = axis_footprint<P>((int)(q >> (kFracBits + hshift)), (int)((q >> hshift) & 0x7FFFu),
                                          wc[d], dwc[d]);
            }
        }
        float xb[3] = {0.f, 0.f, 0.f};
        level_gather<WITH_E, P>(pf, kFS, rf, kRS, jf, wf, dwf, ab, c_f, 1.0f, xb);
        if (TWO)
            level_gather<WITH_E, P>(pc, CS, rc, CR, jc, wc, dwc, ab, c_c, 1.0f / (float)(1 << hshift),
                                    xb);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float *dst = xbar + (int64_t)d * n + p;
            *dst = accumulate ? *dst + xb[d] : xb[d];
        }
    }
}

}  // namespace

namespace {

template <int P>
void launch_deposit_backward_p(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                               int level, const float *rho_bar, float *x_bar, int accumulate,
                               hipStream_t s) {
    const int nt = ctx->nt;
    const unsigned blocks = (unsigned)(nt * nt * nt);
    if (level == 0) {
        xbar_gather_kernel<false, false, P><<<blocks, kBlock, 0, s>>>(
            pos, cs, nullptr, (int)n, ctx->n_f, nt, nullptr, rho_bar, 0.f, nullptr, nullptr, 0.f, 1,
            0, x_bar, accumulate);
    } else {
        // coarse only: a zero fine rhobar contributes nothing
        const Level &C = ctx->lv[1];
        xbar_gather_kernel<false, true, P><<<blocks, kBlock, 0, s>>>(
            pos, cs, nullptr, (int)n, ctx->n_f, nt, nullptr, nullptr, 0.f, nullptr, rho_bar, 0.f,
            C.n, C.hshift, x_bar, accumulate);
    }
}

template <int P>
int launch_pm_backward_p(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                         const float *acc_bar, float *x_bar, int accumulate, unsigned char *work,
                         const WorkLayout &L, hipStream_t s) {
    const int nt = ctx->nt;
    const unsigned blocks = (unsigned)(nt * nt * nt);
    const double gm = ctx->cfg.g_newton * ctx->cfg.m_p;
    float *rf = reinterpret_cast<float *>(work + L.real_f);
    float *rc = ctx->n_levels > 1 ? reinterpret_cast<float *>(work + L.real_c) : nullptr;
    float *bf = reinterpret_cast<float *>(work + L.bar_f);
    float *bc = ctx->n_levels > 1 ? reinterpret_cast<float *>(work + L.bar_c) : nullptr;
    float2 *spec = reinterpret_cast<float2 *>(work + L.spec);
    // The fine cotangent scatter (max |abar|, then phibar of the fine level)
    // on the context's second stream, beside the recomputed forward
    // potentials on s; they share no buffer (amax and bf against the
    // deposit's regions, rf, rc and the spectrum), and s waits for the
    // scatter before the spectrum is reused for rhobar.
    hipStream_t s2 = ctx->side2;
    CUBE2_CHECK_HIP(hipEventRecord(ctx->ev_fork2, s));
    CUBE2_CHECK_HIP(hipStreamWaitEvent(s2, ctx->ev_fork2, 0));
    unsigned int *amax = reinterpret_cast<unsigned int *>(work + L.red);
    set_u32<<<1, 1, 0, s2>>>(amax, 0u);
    CUBE2_LAUNCH_CHECK();
    if (n > 0) {
        const int64_t m3 = 3 * n;
        const unsigned gb = (unsigned)std::min<int64_t>(4096, (m3 + 255) / 256);
        absmax_kernel<<<gb, 256, 0, s2>>>(acc_bar, m3, amax);
        CUBE2_LAUNCH_CHECK();
    }
    fine_phibar_kernel<P><<<blocks, kPhiBlock, 0, s2>>>(pos, cs, acc_bar, (int)n, ctx->n_f, nt,
                                                     (float)gm, amax, bf);
    CUBE2_LAUNCH_CHECK();
    // forward potentials (recomputed); s joins the scatter whatever happens
    int r = launch_deposit(ctx, pos, cs, n, rf, nullptr, rc, nullptr, work, L, s);
    for (int l = 0; r == CUBE2_OK && l < ctx->n_levels; ++l) {
        float *m = l == 0 ? rf : rc;
        r = launch_potential(ctx, l, m, m, spec, s);
    }
    if (hipEventRecord(ctx->ev_join2, s2) != hipSuccess ||
        hipStreamWaitEvent(s, ctx->ev_join2, 0) != hipSuccess) {
        (void)hipStreamSynchronize(s2);
        return r ? r : CUBE2_EHIP;
    }
    if (r) return r;
    // rhobar = K phibar in place
    r = launch_potential(ctx, 0, bf, bf, spec, s);
    if (r) return r;
    float cc = 0.0f;
    if (ctx->n_levels > 1) {
        const Level &C = ctx->lv[1];
        const int64_t m = (int64_t)C.n * C.n * C.n;
        cc = (float)(gm / ((double)C.H * C.H));
        // the coarse 3-component fixed-point Abar mesh (24 B per coarse node,
        // at most 3/8 of the fine spectrum's bytes for ratios >= 2) lives in
        // the (free) spectrum buffer
        unsigned long long *Am = reinterpret_cast<unsigned long long *>(spec);
        fill_u64<<<(unsigned)((3 * m + 255) / 256), 256, 0, s>>>(Am, 3 * m);
        CUBE2_LAUNCH_CHECK();
        coarse_abar_kernel<P><<<blocks, kBlock, 0, s>>>(pos, cs, acc_bar, (int)n, nt, C.n, C.hshift,
                                                        cc, amax, Am);
        CUBE2_LAUNCH_CHECK();
        divergence_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(Am, C.n, cc, amax, bc);
        CUBE2_LAUNCH_CHECK();
        r = launch_potential(ctx, 1, bc, bc, spec, s);
        if (r) return r;
        auto *k = C.hshift == 2 ? xbar_gather_kernel<true, true, P, 2>
                                : xbar_gather_kernel<true, true, P>;
        k<<<blocks, kBlock, 0, s>>>(pos, cs, acc_bar, (int)n, ctx->n_f, nt, rf, bf, (float)gm, rc,
                                    bc, cc, C.n, C.hshift, x_bar, accumulate);
    } else {
        xbar_gather_kernel<true, false, P><<<blocks, kBlock, 0, s>>>(
            pos, cs, acc_bar, (int)n, ctx->n_f, nt, rf, bf, (float)gm, nullptr, nullptr, 0.f, 1, 0,
            x_bar, accumulate);
    }
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

}  // namespace

int launch_deposit_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                            int level, const float *rho_bar, float *x_bar, int accumulate,
                            hipStream_t s) {
    if (ctx->tsc)
        launch_deposit_backward_p<3>(ctx, pos, cs, n, level, rho_bar, x_bar, accumulate, s);
    else
        launch_deposit_backward_p<2>(ctx, pos, cs, n, level, rho_bar, x_bar, accumulate, s);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

int launch_pm_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cs, int64_t n,
                       const float *acc_bar, float *x_bar, int accumulate, unsigned char *work,
                       const WorkLayout &L, hipStream_t s) {
    if (ctx->tsc)
        return launch_pm_backward_p<3>(ctx, pos, cs, n, acc_bar, x_bar, accumulate, work, L, s);
    return launch_pm_backward_p<2>(ctx, pos, cs, n, acc_bar, x_bar, accumulate, work, L, s);
}

}  // namespace cube2
