// Allocation-free variant of the stand-alone pressure solve
// (les_pressure_solve_noalloc, include/les.h), for callers that cannot
// allocate device memory.  Its workspace -- the ten colour arrays of one
// pressure system -- is a static array of this code object's own device
// memory, one copy per device, present from module load until the process
// ends.  The solve itself is the one of les_pressure_solve_dev (same
// kernels, same iterates), launched kernel by kernel: no captured graphs,
// no timing events.
#include <cmath>
#include <cstdio>
#include <mutex>

#include "les_impl.h"

using namespace les;

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

// In host code `scratch` names a host-side stand-in, not the device array:
// kernels and fills get the address from hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

int na_err(les_handle* h, int code, const char* what, hipError_t e = hipSuccess) {
    char buf[512];
    if (e != hipSuccess)
        std::snprintf(buf, sizeof buf, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    else
        std::snprintf(buf, sizeof buf, "%s", what);
    h->err = buf;
    return code;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device address of `scratch` on device h->device: taken once per device,
// with that device current.
int scratch_address(les_handle* h, unsigned char** out) {
    if (h->device < 0 || h->device >= kMaxDevices) return na_err(h, LES_EDEVICE, "device index");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[h->device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return na_err(h, LES_EDEVICE, "hipGetDevice", e);
        if (cur != h->device && (e = hipSetDevice(h->device)) != hipSuccess)
            return na_err(h, LES_EDEVICE, "hipSetDevice", e);
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != h->device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) return na_err(h, LES_EDEVICE, "hipGetSymbolAddress(scratch)", e);
        g_ptr[h->device] = ptr;
    }
    *out = (unsigned char*)g_ptr[h->device];
    return LES_OK;
}

#define NCK(expr)                                                          \
    do {                                                                   \
        hipError_t e_ = (expr);                                            \
        if (e_ != hipSuccess) return na_err(h, LES_EDEVICE, #expr, e_);    \
    } while (0)

}  // namespace

extern "C" int les_pressure_solve_noalloc(les_handle* h, const float* d_rhs, float* d_p, double tol,
                                          int32_t max_iter, les_solve_stats* st, void* stream) {
    if (!h || !d_rhs || !d_p) return LES_EINVAL;
    if (!(std::isfinite(tol) && tol > 0.0) || max_iter < 0) return na_err(h, LES_EINVAL, "tol/max_iter");
    const Geo& g = h->g;
    const size_t cb = align256((size_t)g.ctot * sizeof(float));
    if (10 * cb > kScratchBytes)
        return na_err(h, LES_EINVAL,
                      "grid too large for the allocation-free solve (its workspace is 64 MiB per device)");
    unsigned char* base = nullptr;
    int rc = scratch_address(h, &base);
    if (rc != LES_OK) return rc;
    PBufs S{};
    for (int c = 0; c < 2; ++c) {
        S.ph[c] = (float*)(base + (0 + c) * cb);
        S.pd[c] = (float*)(base + (2 + c) * cb);
        S.r0[c] = (float*)(base + (4 + c) * cb);
        S.rhs[c] = (float*)(base + (6 + c) * cb);
        S.pa[c] = (float*)(base + (8 + c) * cb);
    }
    hipStream_t saved = h->stream;
    if (stream) h->stream = (hipStream_t)stream;
    hipStream_t s = h->stream;
    auto body = [&]() -> int {
        // The array keeps the last call's contents, maybe in another grid's
        // layout: clear the whole workspace (ghost rows and padding must read
        // zero) with a fill kernel, then scatter the inputs.
        NCK(launch_fill(s, (float*)base, (long long)(10 * cb / sizeof(float)), 0.f));
        NCK(launch_cells_to_colour(g, s, d_rhs, S.rhs));
        NCK(launch_cells_to_colour(g, s, d_p, S.ph));
        const int r = solve_system(h, tol, max_iter, st, S, true);
        if (r < 0) return r;
        NCK(launch_pair_to_cells(g, s, S, d_p));
        return r;
    };
    rc = body();
    h->stream = saved;
    return rc;
}
