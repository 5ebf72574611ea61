// noalloc.hip -- cube2_pp_force without a caller-provided work buffer, for
// callers that cannot allocate.  The PP kernel's scratch (the heaviest-first
// tile order, its radix-sort histogram and scan temporaries, and the tile
// work counter) lives in one file-scope device array of a fixed size.  Each
// device holds its own copy at its own address, taken once per device with
// hipGetSymbolAddress (at cube2_init_tables, else at the entry point's first
// call on that device); host code only ever passes that address on, never the
// array's name.  Every call on one device shares the array, so calls that
// overlap on one device race; the work counter is cleared by a kernel before
// every use, so nothing else carries over between calls.
#include <mutex>

#include "common.hpp"

namespace cube2 {

// Enough for every supported mesh: at n_fine = 1024 there are 64^3 tiles,
// whose order needs (4 * 64^3 + 64) words (4.2 MB), the histogram 66.6 KB
// and the scan temporaries 4.7 KB.
constexpr size_t kNoallocScratchBytes = size_t(5) << 20;

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Offsets of the PP kernel's scratch regions inside the array, in the
// layout that launch_pp reads from a WorkLayout.
bool noalloc_layout(const cube2_ctx *c, WorkLayout &L) {
    L = WorkLayout{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
    const size_t ntiles = (size_t)c->nt * c->nt * c->nt;
    const size_t nblk = (ntiles + 4095) / 4096;
    L.tile_order = take((ntiles * 4 + 64) * sizeof(uint32_t));  // + the tile work counter
    L.hist = take(nblk * 256 * 4 + 1024);
    L.scan_tmp = take((nblk * 256 / 1024 + 64) * 4 * 2 + 4096);
    L.total = off;
    return off <= kNoallocScratchBytes;
}

__global__ void zero_f32(float *p, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = 0.0f;
}

}  // namespace

// The array's address on the current device, taken once per device.
int noalloc_setup(unsigned char **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CUBE2_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return CUBE2_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CUBE2_EHIP;
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    if (out) *out = g_scratch_ptr[dev];
    return CUBE2_OK;
}

}  // namespace cube2

extern "C" int cube2_pp_force_noalloc(cube2_ctx *ctx, const uint16_t *pos,
                                      const uint32_t *cell_start, int64_t n, float *acc,
                                      int accumulate, cube2_stream_t stream) {
    using namespace cube2;
    if (!ctx) return CUBE2_EINVAL;
    if (!ctx->tables) return CUBE2_ESTATE;
    if (n < 0 || n > INT32_MAX || !cell_start || (n > 0 && (!pos || !acc))) return CUBE2_EINVAL;
    WorkLayout L;
    if (!noalloc_layout(ctx, L)) return CUBE2_EWORKSPACE;   // never for n_fine <= 1024
    unsigned char *base = nullptr;
    const int r = noalloc_setup(&base);
    if (r) return r;
    if (n == 0) return CUBE2_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (ctx->cfg.flags & CUBE2_PP_OFF) {
        if (!accumulate) {   // a fill kernel, not a memset node, for graph capture
            zero_f32<<<(unsigned)((3 * n + 255) / 256), 256, 0, s>>>(acc, 3 * n);
            CUBE2_LAUNCH_CHECK();
        }
        return CUBE2_OK;
    }
    return launch_pp(ctx, pos, cell_start, n, acc, accumulate, base, L, s);
}
