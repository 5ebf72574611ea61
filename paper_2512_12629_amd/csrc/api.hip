// api.hip -- the C ABI of include/cube2.h: argument checks, buffer layout
// and the order of the launches.  All arithmetic is in the kernel files.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"

using namespace cube2;

namespace {

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) { int r = 0; while ((1 << r) < v) ++r; return r; }
int pitch_of(int n) { return (int)align_up((size_t)(n / 2 + 1), 16); }

size_t table_layout(cube2_ctx *c) {
    size_t off = 256;  // status word block
    for (int l = 0; l < c->n_levels; ++l) {
        Level &L = c->lv[l];
        L.tw_off = off;
        off = align_up(off + (size_t)L.n * sizeof(float2), 256);
    }
    for (int l = 0; l < c->n_levels; ++l) {
        Level &L = c->lv[l];
        size_t h = (size_t)(L.n / 2 + 1);
        L.g_off = off;
        off = align_up(off + h * h * h * sizeof(float), 256);
        // z-pass copy: [my][kx / 16][mz][kx % 16], kx padded to the pitch
        L.gz_off = off;
        off = align_up(off + h * (size_t)pitch_of(L.n) * h * sizeof(float), 256);
    }
    c->pp_soff = off;
    off = align_up(off + (size_t)kSRows * 4 * sizeof(float), 256);
    if (c->fp64) {
        for (int l = 0; l < c->n_levels; ++l) {
            Level &L = c->lv[l];
            size_t h = (size_t)(L.n / 2 + 1);
            L.tw64_off = off;
            off = align_up(off + (size_t)L.n * sizeof(double2), 256);
            L.g64_off = off;
            off = align_up(off + h * h * h * sizeof(double), 256);
        }
        c->pp64_off = off;
        off = align_up(off + (size_t)(kPairKMax + 1) * kPairRow * sizeof(double), 256);
    }
    return off;
}

}  // namespace

namespace cube2 {

WorkLayout work_layout(const cube2_ctx *c, int64_t n) {
    WorkLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
    const size_t nf3 = (size_t)c->n_f * c->n_f * c->n_f;
    const size_t nc = c->n_levels > 1 ? (size_t)c->lv[1].n : 0;
    const size_t nc3 = nc * nc * nc;
    L.real_f = take(nf3 * sizeof(float));
    L.real_c = take(nc3 * sizeof(float));
    L.bar_f = take(nf3 * sizeof(float));
    L.bar_c = take(nc3 * sizeof(float));
    L.spec = take((size_t)c->n_f * c->n_f * c->lv[0].pitch * sizeof(float2));
    L.coarse_acc = take(nc3 * sizeof(uint64_t));
    size_t nn = (size_t)(n > 0 ? n : 1);
    L.keys = take(nn * 4);
    L.vals = take(nn * 4);
    L.keys2 = take(nn * 4);
    L.vals2 = take(nn * 4);
    const size_t ntiles = (size_t)c->nt * c->nt * c->nt;
    size_t nblk = (std::max(nn, ntiles) + 4095) / 4096;
    L.hist = take(nblk * 256 * 4 + 1024);
    L.tile_order = take((ntiles * 4 + 64) * sizeof(uint32_t));  // + the tile work counter
    L.vel_tmax = take(ntiles * sizeof(float));
    const size_t scan_len = std::max((size_t)(c->n_cells + 1), nblk * 256);
    L.scan_tmp = take((scan_len / 1024 + 64) * 4 * 2 + 4096);
    L.offs_tmp = take(nn * 3 * sizeof(uint16_t));
    L.red = take(8192 * 8 * sizeof(double));
    {
        const size_t tblk = (ntiles + 4095) / 4096;
        L.pp_order = take((ntiles * 4 + 64) * sizeof(uint32_t));
        L.pp_hist = take(tblk * 256 * 4 + 1024);
        L.pp_scan = take((tblk * 256 / 1024 + 64) * 4 * 2 + 4096);
        L.acc_pp = take(nn * 3 * sizeof(float));
    }
    if (c->fp64) {
        L.real64_f = take(nf3 * sizeof(double));
        L.real64_c = take(nc3 * sizeof(double));
        L.spec64 = take((size_t)c->n_f * c->n_f * c->lv[0].pitch * sizeof(double2));
    }
    L.total = off;
    return L;
}

}  // namespace cube2

#define CHECK_WORK(n)                                                      \
    WorkLayout L_ = work_layout(ctx, (n));                                 \
    if (!work || work_bytes < L_.total) return CUBE2_EWORKSPACE;           \
    unsigned char *work_ = static_cast<unsigned char *>(work)

#define CHECK_READY()                                          \
    if (!ctx) return CUBE2_EINVAL;                             \
    if (!ctx->tables) return CUBE2_ESTATE

extern "C" {

int cube2_create(const cube2_config *cfg, cube2_ctx **out) {
    if (!cfg || !out) return CUBE2_EINVAL;
    *out = nullptr;
    const cube2_config &c = *cfg;
    if (!is_pow2(c.n_fine) || c.n_fine < 16 || c.n_fine > 1024) return CUBE2_EUNSUPPORTED;
    if (c.coarse_ratio != 0) {
        if (c.coarse_ratio != 2 && c.coarse_ratio != 4 && c.coarse_ratio != 8)
            return CUBE2_EUNSUPPORTED;
        if (c.n_fine / c.coarse_ratio < 8) return CUBE2_EUNSUPPORTED;
        if (!(c.b_coarse > c.b_fine)) return CUBE2_EINVAL;
    }
    if (!(c.b_fine > 0.0) || c.b_fine > 4.0) return CUBE2_EUNSUPPORTED;
    if (!(c.b_pp > 0.0) || !(c.b_pp < c.b_fine)) return CUBE2_EINVAL;
    if (!(c.m_p > 0.0) || !std::isfinite(c.g_newton)) return CUBE2_EINVAL;
    if (c.alias_nmax < 0 || c.alias_nmax > 4) return CUBE2_EUNSUPPORTED;

    cube2_ctx *ctx = new (std::nothrow) cube2_ctx();
    if (!ctx) return CUBE2_EINVAL;
    ctx->cfg = c;
    ctx->n_f = c.n_fine;
    ctx->pp_halo = c.b_fine > 2.0 ? 2 : 1;  // PP cutoff within 1 or 2 IOS cells (2 fine cells each)
    ctx->n_ios = c.n_fine / 2;
    ctx->nt = ctx->n_ios / kTileIos;
    ctx->n_cells = (int64_t)ctx->n_ios * ctx->n_ios * ctx->n_ios;
    ctx->n_levels = c.coarse_ratio ? 2 : 1;
    ctx->fp64 = (c.flags & CUBE2_FP64_FORM) != 0;
    ctx->tsc = (c.flags & CUBE2_ASSIGN_TSC) != 0;
    ctx->isolated = (c.flags & CUBE2_ISOLATED) != 0;
    Level &F = ctx->lv[0];
    F.n = c.n_fine;
    F.H = 1;
    F.hshift = 0;
    F.pitch = pitch_of(F.n);
    F.b_a = c.b_fine;
    F.b_prev = c.coarse_ratio ? c.b_coarse : -1.0;
    if (c.coarse_ratio) {
        Level &C = ctx->lv[1];
        C.n = c.n_fine / c.coarse_ratio;
        C.H = c.coarse_ratio;
        C.hshift = ilog2(c.coarse_ratio);
        C.pitch = pitch_of(C.n);
        C.b_a = c.b_coarse;
        C.b_prev = -1.0;
    }
    ctx->table_bytes = table_layout(ctx);
    if (build_pair_table(ctx)) {
        delete ctx;
        return CUBE2_EUNSUPPORTED;
    }
    *out = ctx;
    return CUBE2_OK;
}

void cube2_destroy(cube2_ctx *ctx) {
    if (!ctx) return;
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->ev_fork2) (void)hipEventDestroy(ctx->ev_fork2);
    if (ctx->ev_join2) (void)hipEventDestroy(ctx->ev_join2);
    if (ctx->side2) (void)hipStreamDestroy(ctx->side2);
    delete ctx;
}

int cube2_sizes(const cube2_ctx *ctx, int64_t n_max, size_t *table_bytes, size_t *work_bytes) {
    if (!ctx || n_max < 0 || n_max > INT32_MAX) return CUBE2_EINVAL;
    if (table_bytes) *table_bytes = ctx->table_bytes;
    if (work_bytes) *work_bytes = work_layout(ctx, n_max).total;
    return CUBE2_OK;
}

int cube2_self_check(const cube2_ctx *ctx, int64_t n_max) {
    if (!ctx || n_max < 0 || n_max > INT32_MAX) return CUBE2_EINVAL;
    const WorkLayout L = work_layout(ctx, n_max);
    const size_t ntiles = (size_t)ctx->nt * ctx->nt * ctx->nt;
    auto fits = [&](size_t off, size_t bytes) { return off + bytes <= L.total; };
    // the PM adjoint's 3-component 64-bit coarse mesh lives in the spectrum area
    if (ctx->n_levels > 1) {
        const size_t nc = (size_t)ctx->lv[1].n;
        const size_t spec = (size_t)ctx->n_f * ctx->n_f * ctx->lv[0].pitch * 8;
        if (3 * nc * nc * nc * sizeof(uint64_t) > spec) return CUBE2_EWORKSPACE;
    }
    if (!fits(L.acc_pp, (size_t)3 * n_max * sizeof(float))) return CUBE2_EWORKSPACE;
    if (!fits(L.tile_order, (ntiles * 4 + 64) * sizeof(uint32_t))) return CUBE2_EWORKSPACE;
    if (!fits(L.vel_tmax, ntiles * sizeof(float))) return CUBE2_EWORKSPACE;
    return vel_layout_check(ctx, L);
}

int cube2_level_shape(const cube2_ctx *ctx, int level, int32_t *n, int32_t *pitch) {
    if (!ctx || level < 0 || level >= ctx->n_levels) return CUBE2_EINVAL;
    if (n) *n = ctx->lv[level].n;
    if (pitch) *pitch = ctx->lv[level].pitch;
    return CUBE2_OK;
}

int cube2_init_tables(cube2_ctx *ctx, void *tables, size_t table_bytes, cube2_stream_t stream) {
    if (!ctx || !tables) return CUBE2_EINVAL;
    if (table_bytes < ctx->table_bytes) return CUBE2_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // cube2_force's side stream and its fork/join events, made once per
    // context; on a partial failure nothing is kept, so a later call retries
    if (!ctx->side) {
        hipStream_t side = nullptr;
        hipEvent_t fork = nullptr, join = nullptr;
        if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
            if (join) (void)hipEventDestroy(join);
            if (fork) (void)hipEventDestroy(fork);
            if (side) (void)hipStreamDestroy(side);
            return CUBE2_EHIP;
        }
        ctx->ev_fork = fork;
        ctx->ev_join = join;
        ctx->side = side;
    }
    if (!ctx->side2) {
        hipStream_t side = nullptr;
        hipEvent_t fork = nullptr, join = nullptr;
        if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
            if (join) (void)hipEventDestroy(join);
            if (fork) (void)hipEventDestroy(fork);
            if (side) (void)hipStreamDestroy(side);
            return CUBE2_EHIP;
        }
        ctx->ev_fork2 = fork;
        ctx->ev_join2 = join;
        ctx->side2 = side;
    }
    // the no-allocation PP entry point's scratch address on this device
    const int sr = noalloc_setup(nullptr);
    if (sr) return sr;
    ctx->tables = static_cast<unsigned char *>(tables);
    CUBE2_CHECK_HIP(hipMemsetAsync(ctx->tables, 0, 256, s));
    CUBE2_CHECK_HIP(hipMemcpyAsync(ctx->tables + ctx->pp_soff, ctx->pp_srows.data(),
                                   ctx->pp_srows.size() * sizeof(float), hipMemcpyHostToDevice, s));
    if (ctx->fp64)
        CUBE2_CHECK_HIP(hipMemcpyAsync(ctx->tables + ctx->pp64_off, ctx->pp_rows64.data(),
                                       ctx->pp_rows64.size() * sizeof(double),
                                       hipMemcpyHostToDevice, s));
    return launch_green(ctx, s);
}

int cube2_green_table(const cube2_ctx *ctx, int level, float *out, cube2_stream_t stream) {
    CHECK_READY();
    if (level < 0 || level >= ctx->n_levels || !out) return CUBE2_EINVAL;
    size_t h = (size_t)(ctx->lv[level].n / 2 + 1);
    CUBE2_CHECK_HIP(hipMemcpyAsync(out, ctx->tables + ctx->lv[level].g_off, h * h * h * 4,
                                   hipMemcpyDeviceToDevice,
                                   reinterpret_cast<hipStream_t>(stream)));
    return CUBE2_OK;
}

int cube2_pack(cube2_ctx *ctx, const float *x, int64_t n, uint16_t *pos, uint32_t *cell_start,
               int32_t *perm, void *work, size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!x || !pos || !perm)))
        return CUBE2_EINVAL;
    CHECK_WORK(n);
    return launch_pack(ctx, x, n, pos, cell_start, perm, work_, L_,
                       reinterpret_cast<hipStream_t>(stream));
}

int cube2_deposit(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                  int level, float *rho, uint64_t *rho_fx, void *work, size_t work_bytes,
                  cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || !rho || (n > 0 && !pos)) return CUBE2_EINVAL;
    if (level < 0 || level >= ctx->n_levels) return CUBE2_EINVAL;
    CHECK_WORK(n);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (level == 0)
        return launch_deposit(ctx, pos, cell_start, n, rho, rho_fx, nullptr, nullptr, work_, L_, s);
    return launch_deposit(ctx, pos, cell_start, n, nullptr, nullptr, rho, rho_fx, work_, L_, s);
}

int cube2_fft_r2c(cube2_ctx *ctx, int level, const float *mesh, float *spec, void *work,
                  size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (level < 0 || level >= ctx->n_levels || !mesh || !spec) return CUBE2_EINVAL;
    (void)work;
    (void)work_bytes;
    return launch_fft_r2c(ctx, level, mesh, reinterpret_cast<float2 *>(spec),
                          reinterpret_cast<hipStream_t>(stream));
}

int cube2_potential(cube2_ctx *ctx, int level, const float *rho, float *phi, void *work,
                    size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (level < 0 || level >= ctx->n_levels || !rho || !phi) return CUBE2_EINVAL;
    CHECK_WORK(0);
    return launch_potential(ctx, level, rho, phi, reinterpret_cast<float2 *>(work_ + L_.spec),
                            reinterpret_cast<hipStream_t>(stream));
}

int cube2_interp(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                 const float *phi_fine, const float *phi_coarse, float *acc, int accumulate,
                 cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || !phi_fine) return CUBE2_EINVAL;
    if (n > 0 && (!pos || !acc)) return CUBE2_EINVAL;
    if (ctx->n_levels > 1 && !phi_coarse) return CUBE2_EINVAL;
    return launch_interp(ctx, pos, cell_start, n, phi_fine, phi_coarse, acc, accumulate,
                         reinterpret_cast<hipStream_t>(stream));
}

int cube2_pm_force(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                   float *acc, int accumulate, void *work, size_t work_bytes,
                   cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!pos || !acc))) return CUBE2_EINVAL;
    CHECK_WORK(n);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float *rf = reinterpret_cast<float *>(work_ + L_.real_f);
    float *rc = ctx->n_levels > 1 ? reinterpret_cast<float *>(work_ + L_.real_c) : nullptr;
    float2 *spec = reinterpret_cast<float2 *>(work_ + L_.spec);
    int rcode = launch_deposit(ctx, pos, cell_start, n, rf, nullptr, rc, nullptr, work_, L_, s);
    if (rcode) return rcode;
    for (int l = 0; l < ctx->n_levels; ++l) {
        float *m = l == 0 ? rf : rc;
        rcode = launch_potential(ctx, l, m, m, spec, s);
        if (rcode) return rcode;
    }
    if (n == 0) return CUBE2_OK;
    return launch_interp(ctx, pos, cell_start, n, rf, rc, acc, accumulate, s);
}

int cube2_pm_level_force(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                         int64_t n, int level, float *acc, int accumulate, void *work,
                         size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!pos || !acc))) return CUBE2_EINVAL;
    if (level < 0 || level >= ctx->n_levels) return CUBE2_EINVAL;
    CHECK_WORK(n);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float *m = reinterpret_cast<float *>(work_ + (level == 0 ? L_.real_f : L_.real_c));
    float2 *spec = reinterpret_cast<float2 *>(work_ + L_.spec);
    int rcode = level == 0
                    ? launch_deposit(ctx, pos, cell_start, n, m, nullptr, nullptr, nullptr, work_, L_, s)
                    : launch_deposit(ctx, pos, cell_start, n, nullptr, nullptr, m, nullptr, work_, L_, s);
    if (rcode) return rcode;
    rcode = launch_potential(ctx, level, m, m, spec, s);
    if (rcode) return rcode;
    if (n == 0) return CUBE2_OK;
    return launch_interp_levels(ctx, pos, cell_start, n, level == 0 ? m : nullptr,
                                level == 1 ? m : nullptr, acc, accumulate, level == 0 ? 1 : 2, s);
}

int cube2_tile_gather(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                      const int32_t *origins, int32_t n_tiles, int32_t tile, int32_t buffer,
                      float *x_local, int32_t *idx, int64_t m_max, int64_t *m, void *work,
                      size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || !origins || !m || m_max < 0) return CUBE2_EINVAL;
    if (n > 0 && !pos) return CUBE2_EINVAL;
    if (m_max > 0 && (!x_local || !idx)) return CUBE2_EINVAL;
    if (n_tiles < 1 || n_tiles > 4096) return CUBE2_EINVAL;
    const int64_t n_slot = (int64_t)tile + 2 * (int64_t)buffer;
    if (tile < 2 || buffer < 0 || (tile & 1) || (buffer & 1)) return CUBE2_EINVAL;
    if (n_slot < 32 || (n_slot & (n_slot - 1)) || n_slot > ctx->n_f) return CUBE2_EUNSUPPORTED;
    const int k = tile_slots(n_tiles);
    if (n_slot * k > 512) return CUBE2_EUNSUPPORTED;   // exact FP32 box-unit positions
    const int R = (int)(n_slot / 2);
    // the per-cell scan must fit the scan area sized for the IOS cells
    if ((int64_t)n_tiles * R * R * R > ctx->n_cells) return CUBE2_EWORKSPACE;
    std::vector<int32_t> r0((size_t)3 * n_tiles);
    for (int t = 0; t < n_tiles; ++t)
        for (int d = 0; d < 3; ++d) {
            const int32_t o = origins[3 * t + d];
            if (o < 0 || o >= ctx->n_f || (o & 1)) return CUBE2_EINVAL;
            r0[3 * t + d] = (int32_t)((((o - buffer) / 2) % ctx->n_ios + ctx->n_ios) % ctx->n_ios);
        }
    CHECK_WORK(n);
    *m = 0;
    return launch_tile_gather(ctx, pos, cell_start, n, r0.data(), n_tiles, R, x_local, idx, m_max,
                              m, work_, L_, reinterpret_cast<hipStream_t>(stream));
}

int cube2_tile_scatter_add(int64_t m, const int32_t *perm_local, const float *x_local,
                           const int32_t *idx, int32_t n_tiles, int32_t tile, int32_t buffer,
                           float scale, const float *acc_local, float *acc, int64_t n,
                           cube2_stream_t stream) {
    if (m < 0 || n < 0 || m > INT32_MAX || n > INT32_MAX) return CUBE2_EINVAL;
    if (m > 0 && (!perm_local || !x_local || !idx || !acc_local || !acc)) return CUBE2_EINVAL;
    if (tile < 2 || buffer < 0 || n_tiles < 1 || n_tiles > 4096) return CUBE2_EINVAL;
    return launch_tile_scatter_add(m, perm_local, x_local, idx, n_tiles, buffer, buffer + tile,
                                   tile + 2 * buffer, scale, acc_local, acc, n,
                                   reinterpret_cast<hipStream_t>(stream));
}

int cube2_pp_force(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                   float *acc, int accumulate, void *work, size_t work_bytes,
                   cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!pos || !acc))) return CUBE2_EINVAL;
    CHECK_WORK(n);
    (void)work_;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (n == 0) return CUBE2_OK;
    if (ctx->cfg.flags & CUBE2_PP_OFF) {
        if (!accumulate) CUBE2_CHECK_HIP(hipMemsetAsync(acc, 0, (size_t)n * 3 * 4, s));
        return CUBE2_OK;
    }
    return launch_pp(ctx, pos, cell_start, n, acc, accumulate, work_, L_, s);
}

int cube2_pp_force_skip(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                        int64_t n, const uint8_t *skip_tiles, float *acc, int accumulate,
                        void *work, size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!pos || !acc))) return CUBE2_EINVAL;
    CHECK_WORK(n);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (n == 0 || (ctx->cfg.flags & CUBE2_PP_OFF)) return CUBE2_OK;
    return launch_pp(ctx, pos, cell_start, n, acc, accumulate, work_, L_, s, skip_tiles);
}

namespace {

// The PM part on `stream` and the PP part on the context's side stream,
// joined on `stream`, then out = PM + PP.  abar == nullptr: the force; else
// the adjoint for the cotangents abar.
int force_concurrent(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                     const float *abar, float *out, int accumulate, void *work, size_t work_bytes,
                     cube2_stream_t stream, unsigned char *work_, const cube2::WorkLayout &L_) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!ctx->side) return CUBE2_ESTATE;   // made by cube2_init_tables
    float *acc_pp = reinterpret_cast<float *>(work_ + L_.acc_pp);
    // PP first (it starts with a reduced persistent grid), the PM part beside it
    CUBE2_CHECK_HIP(hipEventRecord(ctx->ev_fork, s));
    CUBE2_CHECK_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
    int rcode = launch_pp_concurrent(ctx, pos, cell_start, n, abar, acc_pp, work_, L_, ctx->side);
    if (rcode == CUBE2_OK)
        rcode = abar ? cube2_pm_force_backward(ctx, pos, cell_start, n, abar, out, accumulate,
                                               work, work_bytes, stream)
                     : cube2_pm_force(ctx, pos, cell_start, n, out, 0, work, work_bytes, stream);
    // the caller's stream waits for the side stream on every path; if the
    // join cannot be recorded, the side stream is drained before returning,
    // so that no PP kernel still writes the work buffer
    if (hipEventRecord(ctx->ev_join, ctx->side) != hipSuccess ||
        hipStreamWaitEvent(s, ctx->ev_join, 0) != hipSuccess) {
        (void)hipStreamSynchronize(ctx->side);
        return rcode ? rcode : CUBE2_EHIP;
    }
    if (rcode) return rcode;
    return launch_add3(out, acc_pp, 3 * n, s);
}

}  // namespace

int cube2_force(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                float *acc, void *work, size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!pos || !acc))) return CUBE2_EINVAL;
    CHECK_WORK(n);
    if (n == 0 || (ctx->cfg.flags & CUBE2_PP_OFF))
        return cube2_pm_force(ctx, pos, cell_start, n, acc, 0, work, work_bytes, stream);
    return force_concurrent(ctx, pos, cell_start, n, nullptr, acc, 0, work, work_bytes, stream,
                            work_, L_);
}

int cube2_force_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                         int64_t n, const float *acc_bar, float *x_bar, int accumulate, void *work,
                         size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!pos || !acc_bar || !x_bar)))
        return CUBE2_EINVAL;
    CHECK_WORK(n);
    if (n == 0 || (ctx->cfg.flags & CUBE2_PP_OFF))
        return cube2_pm_force_backward(ctx, pos, cell_start, n, acc_bar, x_bar, accumulate, work,
                                       work_bytes, stream);
    return force_concurrent(ctx, pos, cell_start, n, acc_bar, x_bar, accumulate, work, work_bytes,
                            stream, work_, L_);
}

int cube2_kick_drift(cube2_ctx *ctx, const uint16_t *pos_in, const uint32_t *cell_start_in,
                     const float *vel_in, const float *acc, int64_t n, double kick, double drift,
                     uint16_t *pos_out, uint32_t *cell_start_out, float *vel_out,
                     int32_t *perm_out, void *work, size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start_in || !cell_start_out) return CUBE2_EINVAL;
    if (n > 0 && (!pos_in || !vel_in || !acc || !pos_out || !vel_out || !perm_out))
        return CUBE2_EINVAL;
    if (!std::isfinite(kick) || !std::isfinite(drift)) return CUBE2_EINVAL;
    if (n > 0 && ((const void *)pos_in == (const void *)pos_out ||
                  (const void *)vel_in == (const void *)vel_out))
        return CUBE2_EINVAL;
    if ((const void *)cell_start_in == (const void *)cell_start_out) return CUBE2_EINVAL;
    CHECK_WORK(n);
    return launch_kick_drift(ctx, pos_in, cell_start_in, vel_in, acc, n, kick, drift, pos_out,
                             cell_start_out, vel_out, perm_out, work_, L_,
                             reinterpret_cast<hipStream_t>(stream));
}

int cube2_reduce(cube2_ctx *ctx, const float *vel, const float *acc, int64_t n, double *out8,
                 void *work, size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !out8 || (n > 0 && !acc)) return CUBE2_EINVAL;
    CHECK_WORK(n);
    return launch_reduce(ctx, vel, acc, n, out8, work_, L_,
                         reinterpret_cast<hipStream_t>(stream));
}

int cube2_vel_bulk_side(const cube2_ctx *ctx, int *side) {
    CHECK_READY();
    if (!side) return CUBE2_EINVAL;
    *side = vel_bulk_side(ctx);
    return CUBE2_OK;
}

int cube2_vel_encode(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                     const float *vel, int16_t *vq, float *v_bulk, float *v_scale, void *work,
                     size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || !v_bulk || !v_scale) return CUBE2_EINVAL;
    if (n > 0 && (!pos || !vel || !vq)) return CUBE2_EINVAL;
    CHECK_WORK(n);
    return launch_vel_encode(ctx, pos, cell_start, n, vel, vq, v_bulk, v_scale, work_, L_,
                             reinterpret_cast<hipStream_t>(stream));
}

int cube2_vel_decode(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start, int64_t n,
                     const int16_t *vq, const float *v_bulk, const float *v_scale, float *vel,
                     cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || !v_bulk || !v_scale) return CUBE2_EINVAL;
    if (n > 0 && (!pos || !vq || !vel)) return CUBE2_EINVAL;
    return launch_vel_decode(ctx, pos, cell_start, n, vq, v_bulk, v_scale, vel,
                             reinterpret_cast<hipStream_t>(stream));
}

int cube2_status(cube2_ctx *ctx, cube2_stream_t stream) {
    CHECK_READY();
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint32_t word = 0;
    CUBE2_CHECK_HIP(hipMemcpyAsync(&word, status_word(ctx), 4, hipMemcpyDeviceToHost, s));
    CUBE2_CHECK_HIP(hipStreamSynchronize(s));
    CUBE2_CHECK_HIP(hipMemsetAsync(status_word(ctx), 0, 4, s));
    CUBE2_CHECK_HIP(hipStreamSynchronize(s));
    if (word & kStatusNonFinite) return CUBE2_ENONFINITE;
    return word ? CUBE2_EOVERFLOW : CUBE2_OK;
}

int cube2_deposit_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                           int64_t n, int level, const float *rho_bar, float *x_bar,
                           int accumulate, void *work, size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || !rho_bar || (n > 0 && (!pos || !x_bar)))
        return CUBE2_EINVAL;
    if (level < 0 || level >= ctx->n_levels) return CUBE2_EINVAL;
    (void)work;
    (void)work_bytes;
    if (n == 0) return CUBE2_OK;
    return launch_deposit_backward(ctx, pos, cell_start, n, level, rho_bar, x_bar, accumulate,
                                   reinterpret_cast<hipStream_t>(stream));
}

int cube2_pm_force_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                            int64_t n, const float *acc_bar, float *x_bar, int accumulate,
                            void *work, size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!pos || !acc_bar || !x_bar)))
        return CUBE2_EINVAL;
    CHECK_WORK(n);
    if (n == 0) return CUBE2_OK;
    return launch_pm_backward(ctx, pos, cell_start, n, acc_bar, x_bar, accumulate, work_, L_,
                              reinterpret_cast<hipStream_t>(stream));
}

int cube2_pp_force_backward(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                            int64_t n, const float *acc_bar, float *x_bar, int accumulate,
                            void *work, size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!pos || !acc_bar || !x_bar)))
        return CUBE2_EINVAL;
    CHECK_WORK(n);
    if (n == 0) return CUBE2_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (ctx->cfg.flags & CUBE2_PP_OFF) {
        if (!accumulate) CUBE2_CHECK_HIP(hipMemsetAsync(x_bar, 0, (size_t)n * 3 * 4, s));
        return CUBE2_OK;
    }
    return launch_pp_backward(ctx, pos, cell_start, n, acc_bar, x_bar, accumulate, work_, L_, s);
}

int cube2_kick_drift_backward(cube2_ctx *ctx, int64_t n, const int32_t *perm,
                              const float *xbar_out, const float *vbar_out, double kick,
                              double drift, float *xbar_in, float *vbar_in, float *acc_bar,
                              cube2_stream_t stream) {
    if (!ctx) return CUBE2_EINVAL;
    if (n < 0 || n > INT32_MAX) return CUBE2_EINVAL;
    if (n > 0 && (!perm || !xbar_out || !vbar_out || !xbar_in || !vbar_in || !acc_bar))
        return CUBE2_EINVAL;
    if (!std::isfinite(kick) || !std::isfinite(drift)) return CUBE2_EINVAL;
    if (n == 0) return CUBE2_OK;
    return launch_kick_drift_backward(ctx, n, perm, xbar_out, vbar_out, kick, drift, xbar_in,
                                      vbar_in, acc_bar, reinterpret_cast<hipStream_t>(stream));
}

int cube2_potential_f64(cube2_ctx *ctx, int level, const double *rho, double *phi, void *work,
                        size_t work_bytes, cube2_stream_t stream) {
    CHECK_READY();
    if (!ctx->fp64) return CUBE2_ESTATE;
    if (level < 0 || level >= ctx->n_levels || !rho || !phi) return CUBE2_EINVAL;
    CHECK_WORK(0);
    return launch_potential64(ctx, level, rho, phi,
                              reinterpret_cast<double2 *>(work_ + L_.spec64),
                              reinterpret_cast<hipStream_t>(stream));
}

int cube2_pm_force_f64(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                       int64_t n, double *acc, int accumulate, void *work, size_t work_bytes,
                       cube2_stream_t stream) {
    CHECK_READY();
    if (!ctx->fp64) return CUBE2_ESTATE;
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!pos || !acc))) return CUBE2_EINVAL;
    CHECK_WORK(n);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool two = ctx->n_levels > 1;
    // the deposit writes its FP32 density into the FP32 scratch meshes and the
    // exact accumulators into the FP64 meshes, converted there in place
    float *rf = reinterpret_cast<float *>(work_ + L_.real_f);
    float *rc = two ? reinterpret_cast<float *>(work_ + L_.real_c) : nullptr;
    uint64_t *ff = reinterpret_cast<uint64_t *>(work_ + L_.real64_f);
    uint64_t *fc = two ? reinterpret_cast<uint64_t *>(work_ + L_.real64_c) : nullptr;
    double2 *spec = reinterpret_cast<double2 *>(work_ + L_.spec64);
    int rcode = launch_deposit(ctx, pos, cell_start, n, rf, ff, rc, fc, work_, L_, s);
    if (rcode) return rcode;
    for (int l = 0; l < ctx->n_levels; ++l) {
        uint64_t *m = l == 0 ? ff : fc;
        const int64_t nl = ctx->lv[l].n;
        rcode = launch_fx_to_f64(m, nl * nl * nl, ctx->tsc ? 0x1p-48 : 0x1p-45, s);
        if (rcode) return rcode;
        double *md = reinterpret_cast<double *>(m);
        rcode = launch_potential64(ctx, l, md, md, spec, s);
        if (rcode) return rcode;
    }
    if (n == 0) return CUBE2_OK;
    return launch_interp64(ctx, pos, cell_start, n, reinterpret_cast<double *>(ff),
                           reinterpret_cast<double *>(fc), acc, accumulate, s);
}

int cube2_pp_force_f64(cube2_ctx *ctx, const uint16_t *pos, const uint32_t *cell_start,
                       int64_t n, double *acc, int accumulate, void *work, size_t work_bytes,
                       cube2_stream_t stream) {
    CHECK_READY();
    if (!ctx->fp64) return CUBE2_ESTATE;
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!pos || !acc))) return CUBE2_EINVAL;
    CHECK_WORK(n);
    (void)work_;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (n == 0) return CUBE2_OK;
    if (ctx->cfg.flags & CUBE2_PP_OFF) {
        if (!accumulate) CUBE2_CHECK_HIP(hipMemsetAsync(acc, 0, (size_t)n * 3 * 8, s));
        return CUBE2_OK;
    }
    return launch_pp64(ctx, pos, cell_start, n, acc, accumulate, s);
}

const char *cube2_strerror(int code) {
    switch (code) {
        case CUBE2_OK: return "ok";
        case CUBE2_EINVAL: return "invalid argument";
        case CUBE2_EUNSUPPORTED: return "unsupported configuration";
        case CUBE2_EWORKSPACE: return "tables or work buffer too small";
        case CUBE2_EOVERFLOW: return "deposit accumulator overflow guard tripped";
        case CUBE2_ENONFINITE: return "kick-drift met a non-finite velocity or displacement";
        case CUBE2_EHIP: return "HIP runtime error";
        case CUBE2_ESTATE: return "tables not initialised";
        default: return "unknown status code";
    }
}

}  // extern "C"
