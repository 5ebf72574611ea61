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
#include "common.hpp"

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
struct RootTable {  // exp(-2 pi i k / R), k = 0..R-1
    float re[R];
    float im[R];
    constexpr RootTable() : re(), im() {
        for (int k = 0; k < R; ++k) {
            re[k] = (float)cx_cos_frac(k, R);
            im[k] = (float)-cx_sin_frac(k, R);
        }
    }
};

template <int R>
struct Roots {
    static constexpr RootTable<R> t{};
};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
constexpr int bitrev(int v, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
    return r;
}

// In-register radix-2 DIT DFT of size R, natural order in and out.
// SIGN = -1: forward (exp(-i...)), +1: inverse (unnormalised).
template <int R, int SIGN>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
    constexpr int B = ilog2c(R);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int j = bitrev(i, B);
        if (j > i) {
            float2 t = v[i];
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
                float2 u = v[i + j], t = v[i + j + half];
                if (j == 0) {
                } else if (4 * j == len) {
                    // w = exp(SIGN * i * pi / 2) = SIGN * i
                    t = SIGN < 0 ? make_float2(t.y, -t.x) : make_float2(-t.y, t.x);
                } else {
                    const int k = j * (R / len);
                    const float wr = Roots<R>::t.re[k];
                    const float wi = SIGN < 0 ? Roots<R>::t.im[k] : -Roots<R>::t.im[k];
                    t = make_float2(t.x * wr - t.y * wi, t.x * wi + t.y * wr);
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

// MODE 0: one transform with sign SIGN.  MODE 2: forward, times G/n^3,
// inverse (the z pass).  Workgroup = COLS adjacent columns x one line.
template <int N, int COLS, int SIGN, int MODE>
__global__ __launch_bounds__(COLS *Split<N>::TMAX) void col_fft(
    float2 *__restrict__ data, int64_t jstride, int64_t line_stride, const float2 *__restrict__ tw,
    const float *__restrict__ G, int n, int pitch, float scale) {
    constexpr int N1 = Split<N>::N1, N2 = Split<N>::N2;
    constexpr int PAD = COLS < 16 ? COLS : 0;
    constexpr int RS1 = N2 * COLS + PAD;  // row stride of the forward exchange
    constexpr int RS2 = N1 * COLS + PAD;  // row stride of the inverse exchange
    constexpr int LDS1 = N1 * RS1, LDS2 = (MODE == 2) ? N2 * RS2 : 0;
    constexpr int LDSN = LDS1 > LDS2 ? LDS1 : LDS2;
    __shared__ float2 sh[LDSN];

    const int t = threadIdx.x;
    const int col = t % COLS;
    const int64_t base = (int64_t)blockIdx.y * line_stride + (int64_t)blockIdx.x * COLS + col;
    float2 *line = data + base;

    // forward (or the single) transform, phase 1: thread owns j2, all j1
    if (t < COLS * N2) {
        const int j2 = t / COLS;
        float2 v[N1];
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1) v[j1] = line[(int64_t)(j1 * N2 + j2) * jstride];
        dft<N1, SIGN>(v);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) {
            float2 w = tw[(j2 * k1) & (N - 1)];
            float2 y = (SIGN < 0) ? cmul(v[k1], w) : cmulc(v[k1], w);
            sh[k1 * RS1 + j2 * COLS + col] = y;
        }
    }
    __syncthreads();
    float2 v2[N2];
    int k1 = t / COLS;
    if (t < COLS * N1) {
#pragma unroll
        for (int j2 = 0; j2 < N2; ++j2) v2[j2] = sh[k1 * RS1 + j2 * COLS + col];
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
        const int h = n / 2 + 1;
        const int kx = blockIdx.x * COLS + col;
        const int ky = blockIdx.y;
        const int my = ky <= n - ky ? ky : n - ky;
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
            const int kz = k1 + N1 * k2;
            const int mz = kz <= n - kz ? kz : n - kz;
            const float g = kx < h ? G[((int64_t)mz * h + my) * h + kx] * scale : 0.0f;
            v2[k2] = make_float2(v2[k2].x * g, v2[k2].y * g);
        }
        // inverse phase 1: thread owns b = k1, holds X[a*N1 + b], a = k2
        dft<N2, +1>(v2);
#pragma unroll
        for (int ka = 0; ka < N2; ++ka) {
            float2 w = tw[(k1 * ka) & (N - 1)];
            sh[ka * RS2 + k1 * COLS + col] = cmulc(v2[ka], w);
        }
    }
    __syncthreads();
    if (t < COLS * N2) {
        const int ka = t / COLS;
        float2 v[N1];
#pragma unroll
        for (int b = 0; b < N1; ++b) v[b] = sh[ka * RS2 + b * COLS + col];
        dft<N1, +1>(v);  // v[kb] = x[ka + N2 kb]
#pragma unroll
        for (int kb = 0; kb < N1; ++kb) line[(int64_t)(ka + N2 * kb) * jstride] = v[kb];
    }
}

// ---- x pass: real-to-complex and complex-to-real rows ---------------------

template <int M>
struct RowGeo {
    static constexpr int M1 = Split<M>::N1, M2 = Split<M>::N2, TR = Split<M>::TMAX;
    static constexpr int ROWS = 256 / TR > 0 ? 256 / TR : 1;
    static constexpr int RS = M2 + 1;                       // exchange row stride
    static constexpr int XLEN = (M + 1) > M1 * RS ? (M + 1) : M1 * RS;  // per-row LDS
};

template <int M>
__global__ __launch_bounds__(256) void r2c_x(const float *__restrict__ in, float2 *__restrict__ out,
                                             int pitch, const float2 *__restrict__ tw, int64_t nrows) {
    using Gm = RowGeo<M>;
    constexpr int M1 = Gm::M1, M2 = Gm::M2, TR = Gm::TR, RS = Gm::RS, XL = Gm::XLEN;
    constexpr int N = 2 * M;
    __shared__ float2 sh[Gm::ROWS * XL];
    const int t = threadIdx.x;
    const int rl = t / TR, tl = t % TR;
    const int64_t row = (int64_t)blockIdx.x * Gm::ROWS + rl;
    const bool live = row < nrows;
    const float2 *src = reinterpret_cast<const float2 *>(in + (live ? row : 0) * N);
    float2 *x = sh + rl * XL;

    if (tl < M2) {
        const int j2 = tl;
        float2 v[M1];
#pragma unroll
        for (int j1 = 0; j1 < M1; ++j1) v[j1] = src[j1 * M2 + j2];
        dft<M1, -1>(v);
#pragma unroll
        for (int k1 = 0; k1 < M1; ++k1) x[k1 * RS + j2] = cmul(v[k1], tw[(2 * j2 * k1) & (N - 1)]);
    }
    __syncthreads();
    float2 v2[M2];
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
    float2 *dst = out + row * pitch;
    for (int k = tl; k < pitch; k += TR) {
        float2 r = make_float2(0.f, 0.f);
        if (k <= M) {
            const float2 zk = x[k & (M - 1)], zm = x[(M - k) & (M - 1)];
            // even part E = (Zk + conj Zm)/2, odd part O = (Zk - conj Zm)/(2i)
            const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            const float2 o = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
            r = cadd(e, cmul(o, tw[k]));  // X[k] = E + W_N^k O
        }
        dst[k] = r;
    }
}

template <int M>
__global__ __launch_bounds__(256) void c2r_x(const float2 *__restrict__ in, float *__restrict__ out,
                                             int pitch, const float2 *__restrict__ tw, int64_t nrows) {
    using Gm = RowGeo<M>;
    constexpr int M1 = Gm::M1, M2 = Gm::M2, TR = Gm::TR, RS = Gm::RS, XL = Gm::XLEN;
    constexpr int N = 2 * M;
    __shared__ float2 sh[Gm::ROWS * XL];
    const int t = threadIdx.x;
    const int rl = t / TR, tl = t % TR;
    const int64_t row = (int64_t)blockIdx.x * Gm::ROWS + rl;
    const bool live = row < nrows;
    const float2 *src = in + (live ? row : 0) * pitch;
    float2 *x = sh + rl * XL;
    for (int k = tl; k <= M; k += TR) {
        float2 v = src[k];
        if (k == 0 || k == M) v.y = 0.0f;  // DC and Nyquist are real
        x[k] = v;
    }
    __syncthreads();
    float2 v[M1];
    if (tl < M2) {
        const int b = tl;
#pragma unroll
        for (int a = 0; a < M1; ++a) {
            const int k = a * M2 + b;
            const float2 xk = x[k], xm = x[M - k];
            // Z = (Xk + conj Xm) + i W_N^-k (Xk - conj Xm) = 2 (E + i O)
            const float2 d = make_float2(xk.x - xm.x, xk.y + xm.y);
            const float2 c = cmulc(d, tw[k]);
            v[a] = make_float2(xk.x + xm.x - c.y, xk.y - xm.y + c.x);
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
        float2 w[M2];
#pragma unroll
        for (int b = 0; b < M2; ++b) w[b] = x[tl * RS + b];
        dft<M2, +1>(w);  // w[kb] = z[tl + M1 kb]
        float2 *dst = reinterpret_cast<float2 *>(out + row * N);
#pragma unroll
        for (int kb = 0; kb < M2; ++kb) dst[tl + M1 * kb] = w[kb];
    }
}

// ---- dispatch ------------------------------------------------------------

template <int N>
constexpr int cols_for() { return 16; }

template <int N, int SIGN, int MODE>
int run_col(float2 *data, int64_t jstride, int64_t line_stride, int lines, const float2 *tw,
            const float *G, int n, int pitch, float scale, hipStream_t s) {
    constexpr int COLS = cols_for<N>();
    dim3 grid(pitch / COLS, lines);
    col_fft<N, COLS, SIGN, MODE><<<grid, COLS * Split<N>::TMAX, 0, s>>>(data, jstride, line_stride,
                                                                       tw, G, n, pitch, scale);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

template <int N>
int run_level(int op, const float *rin, float *rout, float2 *spec, const float2 *tw, const float *G,
              int pitch, hipStream_t s) {
    constexpr int M = N / 2;
    using Gm = RowGeo<M>;
    const int64_t rows = (int64_t)N * N;
    const int64_t plane = (int64_t)N * pitch;
    int r;
    const unsigned xblocks = (unsigned)((rows + Gm::ROWS - 1) / Gm::ROWS);
    r2c_x<M><<<xblocks, 256, 0, s>>>(rin, spec, pitch, tw, rows);
    CUBE2_LAUNCH_CHECK();
    // y pass: lines along y inside each z plane
    r = run_col<N, -1, 0>(spec, pitch, plane, N, tw, G, N, pitch, 1.0f, s);
    if (r) return r;
    if (op == 0) {  // forward spectrum only: z pass forward
        return run_col<N, -1, 0>(spec, plane, pitch, N, tw, G, N, pitch, 1.0f, s);
    }
    const float scale = (float)(1.0 / ((double)N * N * N));
    r = run_col<N, -1, 2>(spec, plane, pitch, N, tw, G, N, pitch, scale, s);
    if (r) return r;
    r = run_col<N, +1, 0>(spec, pitch, plane, N, tw, G, N, pitch, 1.0f, s);
    if (r) return r;
    c2r_x<M><<<xblocks, 256, 0, s>>>(spec, rout, pitch, tw, rows);
    CUBE2_LAUNCH_CHECK();
    return CUBE2_OK;
}

int run(cube2_ctx *ctx, int level, int op, const float *rin, float *rout, float2 *spec,
        hipStream_t s) {
    const Level &L = ctx->lv[level];
    const float2 *tw = reinterpret_cast<const float2 *>(ctx->tables + L.tw_off);
    const float *G = reinterpret_cast<const float *>(ctx->tables + L.g_off);
    switch (L.n) {
        case 8: return run_level<8>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 16: return run_level<16>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 32: return run_level<32>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 64: return run_level<64>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 128: return run_level<128>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 256: return run_level<256>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 512: return run_level<512>(op, rin, rout, spec, tw, G, L.pitch, s);
        case 1024: return run_level<1024>(op, rin, rout, spec, tw, G, L.pitch, s);
        default: return CUBE2_EUNSUPPORTED;
    }
}

}  // namespace

int launch_fft_r2c(cube2_ctx *ctx, int level, const float *mesh, float2 *spec, hipStream_t s) {
    return run(ctx, level, 0, mesh, nullptr, spec, s);
}

int launch_potential(cube2_ctx *ctx, int level, const float *rho, float *phi, float2 *spec,
                     hipStream_t s) {
    return run(ctx, level, 1, rho, phi, spec, s);
}

}  // namespace cube2
