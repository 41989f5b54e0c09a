// Coupling of the warm-start network to the LES time step.
//
// Before the solve of a step (right-hand side built, p_prev = ph + pd in
// the pressure pair):
//   1. r = rhs - A p_prev in float64 per cell, stored float32 on the
//      network grid with p_prev; float64 partials of sum r^2, sum p^2
//   2. the input channels (r / RMS r, building mask, p_prev / RMS p)
//   3. the network forward pass -> y
//   4. p0 = p_prev + y RMS(r) / dbar * scale as a (base, correction) pair
//      in colour layout; float64 partials of sum (rhs - A p0)^2
//   5. on the device: if that sum is strictly below sum r^2, the pressure
//      pair becomes p0's; the solve then runs to the usual tolerance.
// After the solve (capture only): target (p* - p_prev) dbar / RMS(r).
// sum r^2 is the squared residual norm of p_prev itself, so the choice
// compares the two starts' residual norms.
#include <cmath>
#include <new>
#include <string>

#include "les_bodies.h"
#include "lesnet_kernels.h"

using namespace les;

struct WarmCtl {
    double r2_prev;   // sum (rhs - A p_prev)^2
    double p2;        // sum p_prev^2
    double r2_net;    // sum (rhs - A p0)^2 (-1: no candidate this step)
    int taken;        // 1: the solve started from p0
    int pad_;
    double s2_prev;   // smoothed-residual rule: sum of the smoothed r^2 of each start
    double s2_net;
};

struct WarmPair {   // candidate start, colour layout, ghosts zero
    float* h[2];
    float* d[2];
};

struct WarmView {
    int D = 0, H = 0, W = 0;     // network grid
    float* tr = nullptr;         // r on the network grid
    float* tp = nullptr;         // p_prev on the network grid
    float* tn = nullptr;         // residual of the candidate (smoothed-residual rule)
    float* ts = nullptr;         // smoothing scratch
    WarmPair cand{};             // candidate p0
    double* part = nullptr;      // 2 * kRedBlocks partials
    WarmCtl* ctl = nullptr;
    WarmCtl* h_ctl = nullptr;    // pinned mirror
    bool candidate = false;      // the last warm_pre computed p0
    // choice made on the host (trial or forced modes) for the last step
    bool host_choice = false;
    int taken = 0;
    double r_prev = -1.0, r_net = -1.0;
};

namespace {

int werr(les_handle* h, int code, const char* what, hipError_t e = hipSuccess) {
    h->err = what;
    if (e != hipSuccess) h->err += std::string(": ") + hipGetErrorString(e);
    return code;
}

#define WCK(expr)                                                        \
    do {                                                                 \
        hipError_t e_ = (expr);                                          \
        if (e_ != hipSuccess) return werr(h, LES_EDEVICE, #expr, e_);    \
    } while (0)

int rup4(int x) { return (x + 3) / 4 * 4; }

__device__ __forceinline__ long long net_vox(const Geo& g, int W, int H, int i0, int j0, int k0) {
    return ((long long)k0 * H + j0) * W + i0;
}

// Step 1: residual and previous pressure, partials [2 lb] = sum r^2,
// [2 lb + 1] = sum p^2.
__global__ __launch_bounds__(kBlock) void k_w_resid(Geo g, PBufs P, int H, int W, float* tr, float* tp,
                                                    double* part) {
    const unsigned lb = blockIdx.x, nb = gridDim.x;
    long long t0, t1;
    red_chunk(g, lb, nb, t0, t1);
    double ar = 0.0, ap = 0.0;
    for (long long t = t0 + threadIdx.x; t < t1; t += kBlock) {
        int ii, j0, k0;
        half_cell(g, t, ii, j0, k0);
        const long long e = g.col(ii, j0, k0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int s = (c + j0 + k0) & 1;
            const int i0 = 2 * ii + s;
            if (i0 < g.nx) {
                const double d = diag64(g, i0, j0, k0);
                const double r = (double)P.rhs[c][e] - apply_A64(g, P.ph[c], P.ph[1 - c], e, s, d) -
                                 apply_A64(g, P.pd[c], P.pd[1 - c], e, s, d);
                const float p = P.ph[c][e] + P.pd[c][e];
                const long long v = net_vox(g, W, H, i0, j0, k0);
                tr[v] = (float)r;
                tp[v] = p;
                ar += r * r;
                ap += (double)p * (double)p;
            }
        }
    }
    const double sr = block_sum(ar);
    const double sp = block_sum(ap);
    if (threadIdx.x == 0) {
        part[2 * lb] = sr;
        part[2 * lb + 1] = sp;
    }
}

// Single block: fold n partial pairs (stride 2) in a fixed order.
__global__ __launch_bounds__(kBlock) void k_w_fin(const double* part, int n, WarmCtl* wc, int which) {
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    a = block_sum(a);
    b = block_sum(b);
    if (threadIdx.x == 0) {
        if (which == 0) {
            wc->r2_prev = a;
            wc->p2 = b;
            wc->r2_net = -1.0;
            wc->s2_prev = -1.0;
            wc->s2_net = -1.0;
            wc->taken = 0;
        } else if (which == 1) {
            wc->r2_net = a;
        } else {
            wc->s2_prev = a;
            wc->s2_net = b;
        }
    }
}

// Step 2: input channels on the whole network grid (padding zero).
__global__ __launch_bounds__(kBlock) void k_w_pack(Geo g, int D, int H, int W, const float* tr,
                                                   const float* tp, const uint8_t* flags, const WarmCtl* wc,
                                                   double ncell, net::bf16* xb, float* cap_x) {
    const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (v >= (long long)D * H * W) return;
    const int x = (int)(v % W);
    const int y = (int)((v / W) % H);
    const int z = (int)(v / ((long long)W * H));
    float c0 = 0.f, c1 = 0.f, c2 = 0.f;
    if (x < g.nx && y < g.ny && z < g.nz) {
        const double rr = sqrt(wc->r2_prev / ncell), rp = sqrt(wc->p2 / ncell);
        c0 = rr > 0.0 ? (float)((double)tr[v] / rr) : 0.f;
        c1 = (flags[g.nat(x + 1, y + 1, z + 1)] & F_CSOLID) ? 1.f : 0.f;
        c2 = rp > 0.0 ? (float)((double)tp[v] / rp) : 0.f;
    }
    if (xb) {
        net::bf16* o = xb + v * 8;
        o[0] = (net::bf16)c0;
        o[1] = (net::bf16)c1;
        o[2] = (net::bf16)c2;
#pragma unroll
        for (int q = 3; q < 8; ++q) o[q] = (net::bf16)0.f;
    }
    if (cap_x) {
        cap_x[v * 3 + 0] = c0;
        cap_x[v * 3 + 1] = c1;
        cap_x[v * 3 + 2] = c2;
    }
}

// Step 4a: the candidate start p0 as a pair like the pressure's own:
// base ph + dp rounded, correction pd plus the rounding error of that sum
// (TwoSum), so a zero proposal reproduces (ph, pd) exactly.
__global__ __launch_bounds__(kBlock) void k_w_cand(Geo g, PBufs P, int H, int W, const float* y,
                                                   const WarmCtl* wc, double ncell, double scale, WarmPair C) {
    int ii, j0, k0;
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (!half_cell(g, t, ii, j0, k0)) return;
    const long long e = g.col(ii, j0, k0);
    const float s = (float)(sqrt(wc->r2_prev / ncell) * scale);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int i0 = 2 * ii + ((c + j0 + k0) & 1);
        if (i0 < g.nx) {
            const float a = P.ph[c][e], b = s * y[net_vox(g, W, H, i0, j0, k0)];
            const float sum = a + b;
            const float bb = sum - a;
            const float err = (a - (sum - bb)) + (b - bb);
            C.h[c][e] = sum;
            C.d[c][e] = P.pd[c][e] + err;
        }
    }
}

// Step 4b: partials of sum (rhs - A p0)^2 (second slot unused), formed as
// for the previous pressure; the residual itself to tn if given.
__global__ __launch_bounds__(kBlock) void k_w_resid_cand(Geo g, PBufs P, WarmPair C, int H, int W, float* tn,
                                                         double* part) {
    const unsigned lb = blockIdx.x, nb = gridDim.x;
    long long t0, t1;
    red_chunk(g, lb, nb, t0, t1);
    double ar = 0.0;
    for (long long t = t0 + threadIdx.x; t < t1; t += kBlock) {
        int ii, j0, k0;
        half_cell(g, t, ii, j0, k0);
        const long long e = g.col(ii, j0, k0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int s = (c + j0 + k0) & 1;
            const int i0 = 2 * ii + s;
            if (i0 < g.nx) {
                const double d = diag64(g, i0, j0, k0);
                const double r = (double)P.rhs[c][e] - apply_A64(g, C.h[c], C.h[1 - c], e, s, d) -
                                 apply_A64(g, C.d[c], C.d[1 - c], e, s, d);
                if (tn) tn[net_vox(g, W, H, i0, j0, k0)] = (float)r;
                ar += r * r;
            }
        }
    }
    const double sr = block_sum(ar);
    if (threadIdx.x == 0) {
        part[2 * lb] = sr;
        part[2 * lb + 1] = 0.0;
    }
}

// One pass of the 7-point mean over the cells: each cell becomes the mean
// of itself and its neighbours inside the domain (constants are kept).
// Repeated passes keep the smooth part of a field, the part SOR removes
// slowly: used on residuals (smoothed-residual rule), on the network's
// output and on captured targets.
__global__ __launch_bounds__(kBlock) void k_w_smooth(Geo g, int H, int W, const float* in, float* out) {
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (long long)g.nx * g.ny * g.nz) return;
    const int x = (int)(t % g.nx);
    const int y = (int)((t / g.nx) % g.ny);
    const int z = (int)(t / ((long long)g.nx * g.ny));
    const long long v = ((long long)z * H + y) * W + x;
    const long long sy = W, sz = (long long)W * H;
    float a = in[v];
    int n = 1;
    if (x > 0) a += in[v - 1], ++n;
    if (x < g.nx - 1) a += in[v + 1], ++n;
    if (y > 0) a += in[v - sy], ++n;
    if (y < g.ny - 1) a += in[v + sy], ++n;
    if (z > 0) a += in[v - sz], ++n;
    if (z < g.nz - 1) a += in[v + sz], ++n;
    out[v] = a / (float)n;
}

// Partials [2 lb] = sum a^2, [2 lb + 1] = sum b^2 over the cells.
__global__ __launch_bounds__(kBlock) void k_w_sumsq2(Geo g, int H, int W, const float* a, const float* b,
                                                     double* part) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    const long long per = (n + gridDim.x - 1) / gridDim.x;
    const long long t0 = (long long)blockIdx.x * per, t1 = t0 + per < n ? t0 + per : n;
    double sa = 0.0, sb = 0.0;
    for (long long t = t0 + threadIdx.x; t < t1; t += kBlock) {
        const int x = (int)(t % g.nx);
        const int y = (int)((t / g.nx) % g.ny);
        const int z = (int)(t / ((long long)g.nx * g.ny));
        const long long v = ((long long)z * H + y) * W + x;
        sa += (double)a[v] * (double)a[v];
        sb += (double)b[v] * (double)b[v];
    }
    sa = block_sum(sa);
    sb = block_sum(sb);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sa;
        part[2 * blockIdx.x + 1] = sb;
    }
}

// Step 5: take p0 if its residual is strictly smaller (every element of
// the colour arrays, ghosts included: both are zero there).
__global__ __launch_bounds__(kBlock) void k_w_select(long long n, PBufs P, WarmPair C, WarmCtl* wc, int rule) {
    const bool take = rule == LES_WARM_ALWAYS ||
                      (rule == LES_WARM_RESIDUAL && wc->r2_net >= 0.0 && wc->r2_net < wc->r2_prev) ||
                      (rule == LES_WARM_SMOOTH && wc->s2_net >= 0.0 && wc->s2_net < wc->s2_prev);
    const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (e == 0) wc->taken = take ? 1 : 0;
    if (!take || e >= n) return;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        P.ph[c][e] = C.h[c][e];
        P.pd[c][e] = C.d[c][e];
    }
}

// After the solve: training target on the network grid (padding zero).
__global__ __launch_bounds__(kBlock) void k_w_target(Geo g, PBufs P, int D, int H, int W, const float* tp,
                                                     const WarmCtl* wc, double ncell, double dbar, float* cap_t) {
    const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (v >= (long long)D * H * W) return;
    const int x = (int)(v % W);
    const int y = (int)((v / W) % H);
    const int z = (int)(v / ((long long)W * H));
    float t = 0.f;
    if (x < g.nx && y < g.ny && z < g.nz) {
        const double rr = sqrt(wc->r2_prev / ncell);
        const int c = (x + y + z) & 1;
        const long long e = g.col(x >> 1, y, z);
        const float p = P.ph[c][e] + P.pd[c][e];
        t = rr > 0.0 ? (float)(((double)p - (double)tp[v]) * dbar / rr) : 0.f;
    }
    cap_t[v] = t;
}

unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

double dbar_of(const Geo& g) { return 2.0 * ((double)g.cx + (double)g.cy + (double)g.cz); }

int ensure_warm(les_handle* h) {
    if (h->warm) return LES_OK;
    const Geo& g = h->g;
    WarmView* w = new (std::nothrow) WarmView();
    if (!w) return werr(h, LES_ENOMEM, "warm-start view");
    w->D = rup4(g.nz);
    w->H = rup4(g.ny);
    w->W = rup4(g.nx);
    const long long V = (long long)w->D * w->H * w->W;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t bv = al((size_t)V * 4), bc = al((size_t)g.ctot * 4), bp = al(2 * (size_t)kRedBlocks * 8),
                 bw = al(sizeof(WarmCtl));
    const size_t total = 4 * bv + 4 * bc + bp + bw;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, total);
    if (e != hipSuccess) {
        delete w;
        return werr(h, LES_ENOMEM, "hipMalloc(warm-start workspace)", e);
    }
    e = hipHostMalloc((void**)&w->h_ctl, sizeof(WarmCtl), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipFree(p);
        delete w;
        return werr(h, LES_ENOMEM, "hipHostMalloc(warm-start mirror)", e);
    }
    char* c = (char*)p;
    w->tr = (float*)c;
    c += bv;
    w->tp = (float*)c;
    c += bv;
    w->tn = (float*)c;
    c += bv;
    w->ts = (float*)c;
    c += bv;
    for (int q = 0; q < 2; ++q) {
        w->cand.h[q] = (float*)c;
        c += bc;
        w->cand.d[q] = (float*)c;
        c += bc;
    }
    w->part = (double*)c;
    c += bp;
    w->ctl = (WarmCtl*)c;
    h->warm_arena = p;
    h->warm = w;
    WCK(hipMemsetAsync(p, 0, total, h->stream));
    WCK(hipStreamSynchronize(h->stream));
    return LES_OK;
}

}  // namespace

namespace les {

int warm_pre(les_handle* h) {
    if (!h->warm_net && !h->cap_x) return LES_OK;
    int rc = ensure_warm(h);
    if (rc != LES_OK) return rc;
    const Geo& g = h->g;
    WarmView* w = h->warm;
    w->host_choice = false;
    hipStream_t s = h->stream;
    const double ncell = (double)g.nx * g.ny * g.nz;
    const long long V = (long long)w->D * w->H * w->W;
    const unsigned rb = red_blocks(g);
    hipLaunchKernelGGL(k_w_resid, dim3(rb), dim3(kBlock), 0, s, g, h->f.P, w->H, w->W, w->tr, w->tp, w->part);
    hipLaunchKernelGGL(k_w_fin, dim3(1), dim3(kBlock), 0, s, w->part, (int)rb, w->ctl, 0);
    WCK(hipGetLastError());
    net::bf16* xb = nullptr;
    if (h->warm_net) {
        if ((rc = net::ws_prepare(h->warm_net, 1, w->D, w->H, w->W)) != LES_OK)
            return werr(h, rc, lesnet_last_error(h->warm_net));
        xb = net::ws_input(h->warm_net);
    }
    hipLaunchKernelGGL(k_w_pack, dim3(nblk(V)), dim3(kBlock), 0, s, g, w->D, w->H, w->W, w->tr, w->tp,
                       h->f.flags, w->ctl, ncell, xb, h->cap_x);
    WCK(hipGetLastError());
    w->candidate = false;
    if (!h->warm_net) return LES_OK;
    if ((rc = net::ws_forward(h->warm_net, s, 1, w->D, w->H, w->W)) != LES_OK)
        return werr(h, rc, lesnet_last_error(h->warm_net));
    const double scale = h->warm_scale / dbar_of(g);
    const unsigned cb = nblk((long long)g.nx * g.ny * g.nz);
    const float* y = net::ws_output(h->warm_net);
    for (int q = 0; q < h->warm_smooth; ++q) {   // smoothed output: y -> ts -> tn -> ts ...
        float* dst = q % 2 ? w->tn : w->ts;
        hipLaunchKernelGGL(k_w_smooth, dim3(cb), dim3(kBlock), 0, s, g, w->H, w->W, y, dst);
        y = dst;
    }
    hipLaunchKernelGGL(k_w_cand, dim3(half_blocks(g)), dim3(kBlock), 0, s, g, h->f.P, w->H, w->W, y, w->ctl,
                       ncell, scale, w->cand);
    const int rule = h->warm_rule;
    hipLaunchKernelGGL(k_w_resid_cand, dim3(rb), dim3(kBlock), 0, s, g, h->f.P, w->cand, w->H, w->W,
                       rule == LES_WARM_SMOOTH ? w->tn : nullptr, w->part);
    hipLaunchKernelGGL(k_w_fin, dim3(1), dim3(kBlock), 0, s, w->part, (int)rb, w->ctl, 1);
    if (rule == LES_WARM_SMOOTH) {
        // the same passes over both residuals, ping-ponging through ts
        // (an even count leaves the result in tr / tn)
        const int passes = 2 * ((h->warm_param + 1) / 2);
        for (float* f : {w->tr, w->tn})
            for (int q = 0; q < passes; ++q)
                hipLaunchKernelGGL(k_w_smooth, dim3(cb), dim3(kBlock), 0, s, g, w->H, w->W, q % 2 ? w->ts : f,
                                   q % 2 ? f : w->ts);
        hipLaunchKernelGGL(k_w_sumsq2, dim3(rb), dim3(kBlock), 0, s, g, w->H, w->W, w->tr, w->tn, w->part);
        hipLaunchKernelGGL(k_w_fin, dim3(1), dim3(kBlock), 0, s, w->part, (int)rb, w->ctl, 2);
    }
    // residual, smoothed-residual and always rules decide on the device,
    // the trial rule on the host (warm_take)
    if (rule != LES_WARM_TRIAL)
        hipLaunchKernelGGL(k_w_select, dim3(nblk(g.ctot)), dim3(kBlock), 0, s, (long long)g.ctot, h->f.P,
                           w->cand, w->ctl, rule);
    WCK(hipGetLastError());
    w->candidate = true;
    return LES_OK;
}

PBufs warm_candidate(les_handle* h) {
    PBufs c{};
    for (int q = 0; q < 2; ++q) {
        c.ph[q] = h->warm->cand.h[q];
        c.pd[q] = h->warm->cand.d[q];
    }
    return c;
}

int warm_take(les_handle* h, int take, double r_prev, double r_net) {
    WarmView* w = h->warm;
    if (take)
        hipLaunchKernelGGL(k_w_select, dim3(nblk(h->g.ctot)), dim3(kBlock), 0, h->stream, (long long)h->g.ctot,
                           h->f.P, w->cand, w->ctl, (int)LES_WARM_ALWAYS);
    WCK(hipGetLastError());
    w->host_choice = true;
    w->taken = take;
    w->r_prev = r_prev;
    w->r_net = r_net;
    return LES_OK;
}

int warm_post(les_handle* h) {
    if (!h->cap_t || !h->warm) return LES_OK;
    const Geo& g = h->g;
    WarmView* w = h->warm;
    const long long V = (long long)w->D * w->H * w->W;
    hipLaunchKernelGGL(k_w_target, dim3(nblk(V)), dim3(kBlock), 0, h->stream, g, h->f.P, w->D, w->H, w->W, w->tp,
                       w->ctl, (double)g.nx * g.ny * g.nz, dbar_of(g), h->cap_t);
    // smoothed target (an even number of passes ends in cap_t)
    const unsigned cb = nblk((long long)g.nx * g.ny * g.nz);
    for (int q = 0; q < 2 * ((h->cap_smooth + 1) / 2); ++q)
        hipLaunchKernelGGL(k_w_smooth, dim3(cb), dim3(kBlock), 0, h->stream, g, w->H, w->W,
                           q % 2 ? w->ts : h->cap_t, q % 2 ? h->cap_t : w->ts);
    WCK(hipGetLastError());
    return LES_OK;
}

int warm_result(les_handle* h, int* taken, double* r_prev, double* r_net) {
    *taken = 0;
    *r_prev = -1.0;
    *r_net = -1.0;
    if (!h->warm || !h->warm->candidate) return LES_OK;
    if (h->warm->host_choice) {
        *taken = h->warm->taken;
        *r_prev = h->warm->r_prev;
        *r_net = h->warm->r_net;
        return LES_OK;
    }
    WCK(hipMemcpyAsync(h->warm->h_ctl, h->warm->ctl, sizeof(WarmCtl), hipMemcpyDeviceToHost, h->stream));
    WCK(hipStreamSynchronize(h->stream));
    const WarmCtl& c = *h->warm->h_ctl;
    // relative to ||rhs|| of this step (the solve's own normaliser)
    WCK(hipMemcpyAsync(h->h_ctl, h->f.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
    WCK(hipStreamSynchronize(h->stream));
    const double rn = std::sqrt(h->h_ctl->rhs2);
    *taken = c.taken;
    const bool sm = h->warm_rule == LES_WARM_SMOOTH;
    const double a = sm ? c.s2_prev : c.r2_prev, b = sm ? c.s2_net : c.r2_net;
    if (rn > 0.0) {
        *r_prev = a >= 0.0 ? std::sqrt(a) / rn : -1.0;
        *r_net = b >= 0.0 ? std::sqrt(b) / rn : -1.0;
    }
    return LES_OK;
}

void warm_free(les_handle* h) {
    if (h->warm) {
        if (h->warm->h_ctl) (void)hipHostFree(h->warm->h_ctl);
        delete h->warm;
        h->warm = nullptr;
    }
    if (h->warm_arena) (void)hipFree(h->warm_arena);
    h->warm_arena = nullptr;
}

}  // namespace les

extern "C" {

int les_warm_grid(const les_handle* h, int32_t* D, int32_t* H, int32_t* W) {
    if (!h || !D || !H || !W) return LES_EINVAL;
    *D = rup4(h->g.nz);
    *H = rup4(h->g.ny);
    *W = rup4(h->g.nx);
    return LES_OK;
}

int les_set_warm_start(les_handle* h, lesnet* n, double target_scale, int32_t rule, int32_t param,
                       int32_t smooth) {
    if (!h) return LES_EINVAL;
    if (n && h->g.stretched) return werr(h, LES_EINVAL, "no learned warm start on a stretched grid");
    if (smooth < 0 || smooth > 100000) return werr(h, LES_EINVAL, "smoothing passes");
    if (n && !(std::isfinite(target_scale) && target_scale > 0.0)) return werr(h, LES_EINVAL, "target_scale");
    if (rule < LES_WARM_RESIDUAL || rule > LES_WARM_ALWAYS) return werr(h, LES_EINVAL, "warm-start rule");
    if ((rule == LES_WARM_TRIAL || rule == LES_WARM_SMOOTH) && (param < 1 || param > 100000))
        return werr(h, LES_EINVAL, "warm-start rule parameter");
    WCK(hipStreamSynchronize(h->stream));
    h->warm_net = n;
    h->warm_scale = n ? target_scale : 1.0;
    h->warm_rule = n ? rule : LES_WARM_RESIDUAL;
    h->warm_param = param;
    h->warm_smooth = smooth;
    if (h->warm) h->warm->candidate = false;
    return LES_OK;
}

int les_set_capture(les_handle* h, float* d_x, float* d_t, int32_t smooth) {
    if (!h) return LES_EINVAL;
    if ((d_x == nullptr) != (d_t == nullptr)) return werr(h, LES_EINVAL, "capture buffers: both or neither");
    if (d_x && h->g.stretched) return werr(h, LES_EINVAL, "no training-pair capture on a stretched grid");
    if (smooth < 0 || smooth > 100000) return werr(h, LES_EINVAL, "smoothing passes");
    WCK(hipStreamSynchronize(h->stream));
    h->cap_x = d_x;
    h->cap_t = d_t;
    h->cap_smooth = smooth;
    return LES_OK;
}

}  // extern "C"
