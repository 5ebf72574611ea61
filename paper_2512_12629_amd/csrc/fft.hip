// fft.hip -- 3D real FFT and the Green's-function multiply (section 2.1.2:
// phi(k) = G(k) rho(k)), hand-written for gfx950.
//
// Layout.  A level mesh is real n^3, [z][y][x].  Its half spectrum is complex
// [kz][ky][kx] with kx in [0, n/2] stored in rows of `pitch` complex values
// (pitch = n/2+1 rounded up to 16, pad columns are zero), so every 16-column
// group is 128-byte aligned.
//
// Passes (each reads and writes the spectrum once):
//   r2c_x   rows along x: an n/2-point complex FFT of (x[2m], x[2m+1]) plus the
//           real-to-complex split, n/2+1 outputs per row;
//   col_fft lines along y (stride pitch) and along z (stride n*pitch), COLS
//           adjacent columns per workgroup so that each row access is a
//           contiguous COLS*8-byte chunk;
//   the z pass multiplies by G/n^3 between its forward and inverse halves;
//   c2r_x   the inverse of r2c_x.
// Every line transform is a four-step FFT N = N1*N2: each thread holds one
// N1-point sub-sequence in registers (radix-2, compile-time twiddles), the
// N1 x N2 transpose goes through LDS, then an N2-point register FFT.
// Every kernel is templated on the real type: float for the production path,
// double for the FP64 plain form (same passes, FP64 twiddles and G).
#include "common.hpp"

#include <type_traits>

namespace cube2 {
namespace {

// ---- compile-time trigonometry for the in-register butterflies ----------

constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double cx_sin_poly(double x) {  // |x| <= pi/4
    double x2 = x * x, term = x, sum = x;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double cx_cos_poly(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
// cos and sin of 2 pi p / q for integers 0 <= p < q, by octant reduction.
constexpr double cx_cos_frac(int p, int q) {
    // angle in units of pi/4: a = 8p/q
    const int num = 8 * p;        // a = num / q
    const int oct = num / q;      // 0..7
    const double r = (double)(num - oct * q) / q * (kPi / 4.0);  // in [0, pi/4)
    switch (oct) {
        case 0: return cx_cos_poly(r);
        case 1: return cx_sin_poly(kPi / 4.0 - r);
        case 2: return -cx_sin_poly(r);
        case 3: return -cx_cos_poly(kPi / 4.0 - r);
        case 4: return -cx_cos_poly(r);
        case 5: return -cx_sin_poly(kPi / 4.0 - r);
        case 6: return cx_sin_poly(r);
        default: return cx_cos_poly(kPi / 4.0 - r);
    }
}
constexpr double cx_sin_frac(int p, int q) {
    const int num = 8 * p;
    const int oct = num / q;
    const double r = (double)(num - oct * q) / q * (kPi / 4.0);
    switch (oct) {
        case 0: return cx_sin_poly(r);
        case 1: return cx_cos_poly(kPi / 4.0 - r);
        case 2: return cx_cos_poly(r);
        case 3: return cx_sin_poly(kPi / 4.0 - r);
        case 4: return -cx_sin_poly(r);
        case 5: return -cx_cos_poly(kPi / 4.0 - r);
        case 6: return -cx_cos_poly(r);
        default: return -cx_sin_poly(kPi / 4.0 - r);
    }
}

template <int R>
struct RootTable {  // exp(-2 pi i k / R), k = 0..R-1, rounded per use
    double re[R];
    double im[R];
    constexpr RootTable() : re(), im() {
        for (int k = 0; k < R; ++k) {
            re[k] = cx_cos_frac(k, R);
            im[k] = -cx_sin_frac(k, R);
        }
    }
};

template <int R>
struct Roots {
    static constexpr RootTable<R> t{};
};

template <typename T> struct Cx;
template <> struct Cx<float> { using c = float2; };
template <> struct Cx<double> { using c = double2; };

__device__ __forceinline__ float2 cmk(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ double2 cmk(double x, double y) { return make_double2(x, y); }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmk(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmk(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {  // a * conj(b)
    return cmk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
constexpr int bitrev(int v, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
    return r;
}

__device__ __forceinline__ float fmac3(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac3(double a, double b, double c) { return __builtin_fma(a, b, c); }

// In-register radix-2 DIT DFT of size R, natural order in and out.
// SIGN = -1: forward (exp(-i...)), +1: inverse (unnormalised).  A butterfly
// with a general twiddle w = (wr, wi) factors out the larger component:
// for |wr| >= |wi|, t w = wr (t.x - q t.y, t.y + q t.x) with q = wi / wr
// (a compile-time constant, |q| <= 1), and u +- t w is then two FMAs per
// component after one FMA for the bracket: 6 instructions instead of 8
// (2 multiplies and 2 FMAs for t w, 4 adds); the other case uses q = wr / wi.
template <int R, int SIGN, typename C>
__device__ __forceinline__ void dft(C (&v)[R]) {
    using S = decltype(v[0].x);
    constexpr int B = ilog2c(R);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int j = bitrev(i, B);
        if (j > i) {
            C t = v[i];
            v[i] = v[j];
            v[j] = t;
        }
    }
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
        const int half = len >> 1;
#pragma unroll
        for (int i = 0; i < R; i += len) {
#pragma unroll
            for (int j = 0; j < half; ++j) {
                C u = v[i + j], t = v[i + j + half];
                if (j == 0) {
                } else if (4 * j == len) {
                    // w = exp(SIGN * i * pi / 2) = SIGN * i
                    t = SIGN < 0 ? cmk(t.y, -t.x) : cmk(-t.y, t.x);
                } else {
                    const int k = j * (R / len);
                    const double dr = Roots<R>::t.re[k];
                    const double di = SIGN < 0 ? Roots<R>::t.im[k] : -Roots<R>::t.im[k];
                    S m, a, b;
                    if (dr * dr >= di * di) {  // t w = wr (t.x - q t.y, t.y + q t.x)
                        const S q = (S)(di / dr);
                        m = (S)dr;
                        a = fmac3(-q, t.y, t.x);
                        b = fmac3(q, t.x, t.y);
                    } else {                   // t w = wi (q t.x - t.y, q t.y + t.x)
                        const S q = (S)(dr / di);
                        m = (S)di;
                        a = fmac3(q, t.x, -t.y);
                        b = fmac3(q, t.y, t.x);
                    }
                    v[i + j] = cmk(fmac3(m, a, u.x), fmac3(m, b, u.y));
                    v[i + j + half] = cmk(fmac3(-m, a, u.x), fmac3(-m, b, u.y));
                    continue;
                }
                v[i + j] = cadd(u, t);
                v[i + j + half] = csub(u, t);
            }
        }
    }
}

template <int N>
struct Split {
    static constexpr int LOG = ilog2c(N);
    static constexpr int N1 = 1 << ((LOG + 1) / 2);
    static constexpr int N2 = N / N1;
    static constexpr int TMAX = N1 > N2 ? N1 : N2;
};

// ---- column (strided) line FFTs ------------------------------------------

template <int N, typename T>
constexpr bool split_exchange() { return sizeof(T) == 4 && N >= 512; }

// MODE 0: one transform with sign SIGN.  MODE 2: forward, times G/n^3,
// inverse (the z pass).  Workgroup = COLS adjacent columns x one line.
// The 1024- and 512-point FP32 transforms move their LDS exchanges as real
// and imaginary halves in two rounds: 66 KB of LDS instead of 128 KB, so two
// workgroups share a CU and one's loads overlap the other's arithmetic.  The
// z pass issues its G loads before the second forward sub-transform, from a
// copy of the table laid out so that each workgroup's values are one
// contiguous block.
template <int N, int COLS, int SIGN, int MODE, typename T>
__global__ __launch_bounds__(COLS *Split<N>::TMAX)
__attribute__((amdgpu_waves_per_eu(split_exchange<N, T>() ? 4 : 1))) void col_fft(
    typename Cx<T>::c *__restrict__ data, int64_t jstride, int64_t line_stride,
    const typename Cx<T>::c *__restrict__ tw, const T *__restrict__ G, int n, int pitch, T scale) {
    using C = typename Cx<T>::c;
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    constexpr bool SPLIT = split_exchange<N, T>();
    // complex exchange: rows padded by COLS values below 16 columns
    constexpr int PAD = COLS < 16 ? COLS : 0;
    constexpr int RS1 = N2 * COLS + PAD;  // row stride of the forward exchange
    constexpr int RS2 = N1 * COLS + PAD;  // row stride of the inverse exchange
    constexpr int LDS1 = N1 * RS1, LDS2 = (MODE == 2) ? N2 * RS2 : 0;
    constexpr int LDSN = LDS1 > LDS2 ? LDS1 : LDS2;
    // split exchange: rows of floats padded by 16
    constexpr int RF1 = N2 * COLS + 16, RF2 = N1 * COLS + 16;
    constexpr int LDF1 = N1 * RF1, LDF2 = (MODE == 2) ? N2 * RF2 : 0;
    constexpr int LDSF = LDF1 > LDF2 ? LDF1 : LDF2;
    __shared__ C sh[SPLIT ? 1 : LDSN];
    __shared__ T shf[SPLIT ? LDSF : 1];

    const int t = threadIdx.x;
    const int col = t % COLS;
    const int64_t base = (int64_t)blockIdx.y * line_stride + (int64_t)blockIdx.x * COLS + col;
    C *line = data + base;

    // z pass: the G values of this thread's k1 (kz = k1 + N1 k2).  FP32
    // reads the z-ordered copy [my][kx / 16][mz][kx % 16] (one contiguous
    // block per workgroup, zero in the pad columns), FP64 the octant table.
    constexpr int NG = MODE == 2 ? N2 : 1;
    constexpr bool ZORDER = sizeof(T) == 4;
    static_assert(!ZORDER || COLS == 16, "the z-ordered table is in groups of 16 columns");
    T g[NG];
    auto load_g = [&]() {
        if (MODE != 2 || t >= COLS * N1) return;
        const int h = n / 2 + 1;
        const int kx = blockIdx.x * COLS + col;
        const int ky = blockIdx.y;
        const int my = ky <= n - ky ? ky : n - ky;
        const int q = t / COLS;
        // (the z-ordered table has fewer than 2^31 entries for n <= 1024)
        const uint32_t gb = ((uint32_t)my * gridDim.x + blockIdx.x) * (uint32_t)h * COLS + col;
#pragma unroll
        for (int k2 = 0; k2 < NG; ++k2) {
            const int kz = q + N1 * k2;
            const int mz = kz <= n - kz ? kz : n - kz;
            if (ZORDER)
                g[k2] = G[gb + (uint32_t)mz * COLS];
            else
                g[k2] = kx < h ? G[((int64_t)mz * h + my) * h + kx] : T(0);
        }
    };

    // forward (or the single) transform, phase 1: thread owns j2, all j1
    C v1[N1];
    // split-exchange transforms read their twiddles from an LDS copy (8 KB,
    // still two workgroups per CU): fewer registers held by global loads
    __shared__ C twl[SPLIT ? N : 1];
    if (t < COLS * N2) {
        const int j2 = t / COLS;
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1) v1[j1] = line[(int64_t)(j1 * N2 + j2) * jstride];
    }
    if (SPLIT) {
        for (int i = t; i < N; i += COLS * Split<N>::TMAX) twl[i] = tw[i];
        __syncthreads();
    }
    const C *twp = SPLIT ? twl : tw;
    if (t < COLS * N2) {
        const int j2 = t / COLS;
        dft<N1, SIGN>(v1);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) {
            const C w = twp[(j2 * k1) & (N - 1)];
            v1[k1] = (SIGN < 0) ? cmul(v1[k1], w) : cmulc(v1[k1], w);
        }
        if constexpr (SPLIT) {
#pragma unroll
            for (int k1 = 0; k1 < N1; ++k1) shf[k1 * RF1 + j2 * COLS + col] = v1[k1].x;
        } else {
#pragma unroll
            for (int k1 = 0; k1 < N1; ++k1) sh[k1 * RS1 + j2 * COLS + col] = v1[k1];
        }
    }
    __syncthreads();
    // phase 2: thread owns k1, all j2
    C v2[N2];
    const int k1 = t / COLS;
    if constexpr (SPLIT) {
        if (t < COLS * N1) {
#pragma unroll
            for (int j2 = 0; j2 < N2; ++j2) v2[j2].x = shf[k1 * RF1 + j2 * COLS + col];
        }
        __syncthreads();
        if (t < COLS * N2) {
            const int j2 = t / COLS;
#pragma unroll
            for (int kk = 0; kk < N1; ++kk) shf[kk * RF1 + j2 * COLS + col] = v1[kk].y;
        }
        __syncthreads();
        if (t < COLS * N1) {
#pragma unroll
            for (int j2 = 0; j2 < N2; ++j2) v2[j2].y = shf[k1 * RF1 + j2 * COLS + col];
        }
    }
    if (t < COLS * N1) {
        if constexpr (!SPLIT) {
#pragma unroll
            for (int j2 = 0; j2 < N2; ++j2) v2[j2] = sh[k1 * RS1 + j2 * COLS + col];
        }
        load_g();  // z pass: in flight during the second sub-transform
        dft<N2, SIGN>(v2);  // v2[k2] = X[k1 + N1 k2]
    }
    if (MODE == 0) {
        if (t < COLS * N1) {
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) line[(int64_t)(k1 + N1 * k2) * jstride] = v2[k2];
        }
        return;
    }
    // ---- z pass: times G / n^3, then the inverse transform ----
    __syncthreads();  // all reads of the forward exchange are done
    if (t < COLS * N1) {
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
            const T gs = g[k2 < NG ? k2 : 0] * scale;
            v2[k2] = cmk(v2[k2].x * gs, v2[k2].y * gs);
        }
        // inverse phase 1: thread owns b = k1, holds X[a*N1 + b], a = k2
        dft<N2, +1>(v2);
#pragma unroll
        for (int ka = 0; ka < N2; ++ka) v2[ka] = cmulc(v2[ka], twp[(k1 * ka) & (N - 1)]);
        if constexpr (SPLIT) {
#pragma unroll
            for (int ka = 0; ka < N2; ++ka) shf[ka * RF2 + k1 * COLS + col] = v2[ka].x;
        } else {
#pragma unroll
            for (int ka = 0; ka < N2; ++ka) sh[ka * RS2 + k1 * COLS + col] = v2[ka];
        }
    }
    __syncthreads();
    // inverse phase 2: thread owns ka, all b
    C v[N1];
    const int ka = t / COLS;
    if constexpr (SPLIT) {
        if (t < COLS * N2) {
#pragma unroll
            for (int b = 0; b < N1; ++b) v[b].x = shf[ka * RF2 + b * COLS + col];
        }
        __syncthreads();
        if (t < COLS * N1) {
#pragma unroll
            for (int kk = 0; kk < N2; ++kk) shf[kk * RF2 + k1 * COLS + col] = v2[kk].y;
        }
        __syncthreads();
        if (t < COLS * N2) {
#pragma unroll
            for (int b = 0; b < N1; ++b) v[b].y = shf[ka * RF2 + b * COLS + col];
        }
    }
    if (t < COLS * N2) {
        if constexpr (!SPLIT) {
#pragma unroll
            for (int b = 0; b < N1; ++b) v[b] = sh[ka * RS2 + b * COLS + col];
        }
        dft<N1, +1>(v);  // v[kb] = x[ka + N2 kb]
#pragma unroll
        for (int kb = 0; kb < N1; ++kb) line[(int64_t)(ka + N2 * kb) * jstride] = v[kb];
    }
}

// ---- x pass: real-to-complex and complex-to-real rows ---------------------

// Row geometry: M = M1 * M2 points per row, TR threads per row, M1 <= M2:
// the first phase of each row transform runs M2 threads (in r2c_x the one
// that loads the row from HBM), so that for M = 512 every thread of a row
// issues loads; measured faster than the opposite split in both directions.
template <int M>
struct RowGeo {
    static constexpr int M1 = Split<M>::N2;
    static constexpr int M2 = Split<M>::N1;
    static constexpr int TR = Split<M>::TMAX;
    static constexpr int ROWS = 256 / TR > 0 ? 256 / TR : 1;
    static constexpr int RS = M2 + 1;                       // exchange row stride
    static constexpr int XLEN = (M + 1) > M1 * RS ? (M + 1) : M1 * RS;  // per-row LDS
};

template <int M, typename T>
__global__ __launch_bounds__(256) void r2c_x(const T *__restrict__ in,
                                             typename Cx<T>::c *__restrict__ out, int pitch,
                                             const typename Cx<T>::c *__restrict__ tw,
                                             int64_t nrows) {
    using C = typename Cx<T>::c;
    using Gm = RowGeo<M>;
    constexpr int M1 = Gm::M1, M2 = Gm::M2, TR = Gm::TR, RS = Gm::RS, XL = Gm::XLEN;
    constexpr int N = 2 * M;
    __shared__ C sh[Gm::ROWS * XL];
    const int t = threadIdx.x;
    const int rl = t / TR, tl = t % TR;
    const int64_t row = (int64_t)blockIdx.x * Gm::ROWS + rl;
    const bool live = row < nrows;
    const C *src = reinterpret_cast<const C *>(in + (live ? row : 0) * N);
    C *x = sh + rl * XL;

    if (tl < M2) {
        const int j2 = tl;
        C v[M1];
#pragma unroll
        for (int j1 = 0; j1 < M1; ++j1) v[j1] = src[j1 * M2 + j2];
        dft<M1, -1>(v);
#pragma unroll
        for (int k1 = 0; k1 < M1; ++k1) x[k1 * RS + j2] = cmul(v[k1], tw[(2 * j2 * k1) & (N - 1)]);
    }
    __syncthreads();
    C v2[M2];
    if (tl < M1) {
#pragma unroll
        for (int j2 = 0; j2 < M2; ++j2) v2[j2] = x[tl * RS + j2];
        dft<M2, -1>(v2);
    }
    __syncthreads();
    if (tl < M1) {
#pragma unroll
        for (int k2 = 0; k2 < M2; ++k2) x[tl + M1 * k2] = v2[k2];  // Z in natural order
    }
    __syncthreads();
    if (!live) return;
    C *dst = out + row * pitch;
    const T half = T(0.5);
    for (int k = tl; k < pitch; k += TR) {
        C r = cmk(T(0), T(0));
        if (k <= M) {
            const C zk = x[k & (M - 1)], zm = x[(M - k) & (M - 1)];
            // even part E = (Zk + conj Zm)/2, odd part O = (Zk - conj Zm)/(2i)
            const C e = cmk(half * (zk.x + zm.x), half * (zk.y - zm.y));
            const C o = cmk(half * (zk.y + zm.y), -half * (zk.x - zm.x));
            r = cadd(e, cmul(o, tw[k]));  // X[k] = E + W_N^k O
        }
        dst[k] = r;
    }
}

template <int M, typename T>
__global__ __launch_bounds__(256) void c2r_x(const typename Cx<T>::c *__restrict__ in,
                                             T *__restrict__ out, int pitch,
                                             const typename Cx<T>::c *__restrict__ tw,
                                             int64_t nrows) {
    using C = typename Cx<T>::c;
    using Gm = RowGeo<M>;
    constexpr int M1 = Gm::M1, M2 = Gm::M2, TR = Gm::TR, RS = Gm::RS, XL = Gm::XLEN;
    constexpr int N = 2 * M;
    __shared__ C sh[Gm::ROWS * XL];
    const int t = threadIdx.x;
    const int rl = t / TR, tl = t % TR;
    const int64_t row = (int64_t)blockIdx.x * Gm::ROWS + rl;
    const bool live = row < nrows;
    const C *src = in + (live ? row : 0) * pitch;
    C *x = sh + rl * XL;
    {
        // all loads of the row issued before the LDS stores
        constexpr int KL = (M + 1 + TR - 1) / TR;
        C vin[KL];
#pragma unroll
        for (int i = 0; i < KL; ++i) {
            const int k = tl + i * TR;
            if (k <= M) vin[i] = src[k];
        }
#pragma unroll
        for (int i = 0; i < KL; ++i) {
            const int k = tl + i * TR;
            if (k <= M) {
                C v = vin[i];
                if (k == 0 || k == M) v.y = T(0);  // DC and Nyquist are real
                x[k] = v;
            }
        }
    }
    __syncthreads();
    C v[M1];
    if (tl < M2) {
        const int b = tl;
#pragma unroll
        for (int a = 0; a < M1; ++a) {
            const int k = a * M2 + b;
            const C xk = x[k], xm = x[M - k];
            // Z = (Xk + conj Xm) + i W_N^-k (Xk - conj Xm) = 2 (E + i O)
            const C d = cmk(xk.x - xm.x, xk.y + xm.y);
            const C c = cmulc(d, tw[k]);
            v[a] = cmk(xk.x + xm.x - c.y, xk.y - xm.y + c.x);
        }
        dft<M1, +1>(v);
    }
    __syncthreads();
    if (tl < M2) {
#pragma unroll
        for (int ka = 0; ka < M1; ++ka) x[ka * RS + tl] = cmulc(v[ka], tw[(2 * tl * ka) & (N - 1)]);
    }
    __syncthreads();
    if (tl < M1 && live) {
        C w[M2];
#pragma unroll
        for (int b = 0; b < M2; ++b) w[b] = x[tl * RS + b];
        dft<M2, +1>(w);  // w[kb] = z[tl + M1 kb]
        C *dst = reinterpret_cast<C *>(out + row * N);
#pragma unroll
        for (int kb = 0; kb < M2; ++kb) dst[tl + M1 * kb] = w[kb];
    }
}

// ---- dispatch ------------------------------------------------------------

// Adjacent columns per col_fft workgroup: 16 complex64 (128 B rows) in FP32;
// 8 complex128 in FP64, which keeps the 1024-point exchange within LDS.
template <typename T>
constexpr int cols_for() { return sizeof(T) == 8 ? 8 : 16; }

template <int N, int SIGN, int MODE, typename T>
int run_col(typename Cx<T>::c *data, int64_t jstride, int64_t line_stride, int lines,
            const typename Cx<T>::c *tw, const T *G, int n, int pitch, T scale, hipStream_t s) {
    constexpr int COLS = cols_for<T>();
    dim3 grid(pitch / COLS, lines);
    col_fft<N, COLS, SIGN, MODE, T><<<grid, COLS * Split<N>::TMAX, 0, s>>>(
        data, jstride, line_stride, tw, G, n, pitch, scale);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

template <int N, typename T>
int run_level(int op, const T *rin, T *rout, typename Cx<T>::c *spec,
              const typename Cx<T>::c *tw, const T *G, int pitch, hipStream_t s) {
    constexpr int M = N / 2;
    using Gm = RowGeo<M>;
    const int64_t rows = (int64_t)N * N;
    const int64_t plane = (int64_t)N * pitch;
    int r;
    const unsigned xblocks = (unsigned)((rows + Gm::ROWS - 1) / Gm::ROWS);
    r2c_x<M, T><<<xblocks, 256, 0, s>>>(rin, spec, pitch, tw, rows);
    CUBE2_LAUNCH_CHECK();
    // y pass: lines along y inside each z plane
    r = run_col<N, -1, 0, T>(spec, pitch, plane, N, tw, G, N, pitch, T(1), s);
    if (r) return r;
    if (op == 0) {  // forward spectrum only: z pass forward
        return run_col<N, -1, 0, T>(spec, plane, pitch, N, tw, G, N, pitch, T(1), s);
    }
    const T scale = (T)(1.0 / ((double)N * N * N));
    r = run_col<N, -1, 2, T>(spec, plane, pitch, N, tw, G, N, pitch, scale, s);
    if (r) return r;
    r = run_col<N, +1, 0, T>(spec, pitch, plane, N, tw, G, N, pitch, T(1), s);
    if (r) return r;
    c2r_x<M, T><<<xblocks, 256, 0, s>>>(spec, rout, pitch, tw, rows);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

template <typename T>
int run(cube2_ctx *ctx, int level, int op, const T *rin, T *rout, typename Cx<T>::c *spec,
        hipStream_t s) {
    using C = typename Cx<T>::c;
    const Level &L = ctx->lv[level];
    const bool f64 = sizeof(T) == 8;
    const C *tw = reinterpret_cast<const C *>(ctx->tables + (f64 ? L.tw64_off : L.tw_off));
    const T *G = reinterpret_cast<const T *>(ctx->tables + (f64 ? L.g64_off : L.gz_off));
    switch (L.n) {
        case 8: return run_level<8, T>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 16: return run_level<16, T>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 32: return run_level<32, T>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 64: return run_level<64, T>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 128: return run_level<128, T>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 256: return run_level<256, T>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 512: return run_level<512, T>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 1024: return run_level<1024, T>(op, rin, rout, spec, tw, G, L.pitch, s);
        default: return CUBE2_EUNSUPPORTED;
    }
}

}  // namespace

int launch_fft_r2c(cube2_ctx *ctx, int level, const float *mesh, float2 *spec, hipStream_t s) {
    return run<float>(ctx, level, 0, mesh, nullptr, spec, s);
}

int launch_potential(cube2_ctx *ctx, int level, const float *rho, float *phi, float2 *spec,
                     hipStream_t s) {
    return run<float>(ctx, level, 1, rho, phi, spec, s);
}

int launch_potential64(cube2_ctx *ctx, int level, const double *rho, double *phi, double2 *spec,
                       hipStream_t s) {
    return run<double>(ctx, level, 1, rho, phi, spec, s);
}

}  // namespace cube2
