// Host runtime of the MI355X LES library: the C ABI of include/les.h.
//
// Owns one arena of device memory per handle (every field at a 256-byte
// aligned offset), the handle's stream, the pinned control-block mirror and
// the SOR driver, which enqueues check intervals ahead of the convergence
// test and reads the device's stop flag one batch behind, so the GPU never
// waits for the host between SOR iterations.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "les_impl.h"

using namespace les;

namespace {

constexpr uint32_t kStateMagic = 0x4C455332u;   // "LES2"

int set_err(les_handle* h, int code, const char* what, hipError_t e = hipSuccess) {
    if (h) {
        char buf[512];
        if (e != hipSuccess)
            std::snprintf(buf, sizeof buf, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
        else
            std::snprintf(buf, sizeof buf, "%s", what);
        h->err = buf;
    }
    return code;
}

#define CK(expr)                                                   \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return set_err(h, LES_EDEVICE, #expr, e_); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
int round_up(int x, int m) { return (x + m - 1) / m * m; }
unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

bool valid_params(const les_params& p) {
    if (!(p.omega > 0.0 && p.omega < 2.0)) return false;
    if (!finite_pos(p.tol)) return false;
    if (p.check_every < 1 || p.max_iter < 0 || p.rebase_every < 1) return false;
    if (!(std::isfinite(p.cs) && p.cs >= 0.0)) return false;
    if (!(std::isfinite(p.nu) && p.nu >= 0.0)) return false;
    if (!std::isfinite(p.alpha) || !std::isfinite(p.beta)) return false;
    if (!(p.bc[LES_XM] == LES_BC_INFLOW || p.bc[LES_XM] == LES_BC_FREESLIP ||
          p.bc[LES_XM] == LES_BC_NOSLIP))
        return false;
    if (!(p.bc[LES_XP] == LES_BC_OUTFLOW || p.bc[LES_XP] == LES_BC_FREESLIP ||
          p.bc[LES_XP] == LES_BC_NOSLIP))
        return false;
    for (int f = LES_YM; f <= LES_ZP; ++f)
        if (p.bc[f] != LES_BC_FREESLIP && p.bc[f] != LES_BC_NOSLIP) return false;
    return true;
}

float tsign(int bc) { return (bc == LES_BC_FREESLIP || bc == LES_BC_OUTFLOW) ? 1.f : -1.f; }

Geo make_geo(int nx, int ny, int nz, const les_spacing& s, double dt, const les_params& p) {
    Geo g{};
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.sx = round_up(nx + 2, 32);
    g.sxy = (long long)g.sx * (ny + 2);
    g.ntot = g.sxy * (nz + 2);
    g.H = (nx + 1) / 2;
    g.S = round_up(g.H + 1, 32);
    g.SP = (long long)g.S * (ny + 2);
    g.ctot = g.SP * (nz + 2) + 2LL * g.S;   // guard row in front and behind
    g.dx = (float)s.dx; g.dy = (float)s.dy; g.dz = (float)s.dz; g.dt = (float)dt;
    g.idx = (float)(1.0 / s.dx); g.idy = (float)(1.0 / s.dy); g.idz = (float)(1.0 / s.dz);
    g.idt = (float)(1.0 / dt);
    g.cx = (float)(1.0 / (s.dx * s.dx));
    g.cy = (float)(1.0 / (s.dy * s.dy));
    g.cz = (float)(1.0 / (s.dz * s.dz));
    g.cxd = 1.0 / (s.dx * s.dx);
    g.cyd = 1.0 / (s.dy * s.dy);
    g.czd = 1.0 / (s.dz * s.dz);
    g.outflow = p.bc[LES_XP] == LES_BC_OUTFLOW;
    g.inflow = p.bc[LES_XM] == LES_BC_INFLOW;
    g.u_last = g.outflow ? nx : nx - 1;
    g.s_xm = tsign(p.bc[LES_XM]); g.s_xp = tsign(p.bc[LES_XP]);
    g.s_ym = tsign(p.bc[LES_YM]); g.s_yp = tsign(p.bc[LES_YP]);
    g.s_zm = tsign(p.bc[LES_ZM]); g.s_zp = tsign(p.bc[LES_ZP]);
    return g;
}

bool singular(const les_handle* h) { return !h->g.outflow; }

// --- host-side packing of owned arrays into / out of the ghosted layout
// (pure data movement, no arithmetic)
void pack_u(const Geo& g, const float* src, float* box) {
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i <= g.nx; ++i)
                box[g.nat(i, j + 1, k + 1)] = src[((size_t)k * g.ny + j) * (g.nx + 1) + i];
}
void pack_v(const Geo& g, const float* src, float* box) {
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j <= g.ny; ++j)
            for (int i = 0; i < g.nx; ++i)
                box[g.nat(i + 1, j, k + 1)] = src[((size_t)k * (g.ny + 1) + j) * g.nx + i];
}
void pack_w(const Geo& g, const float* src, float* box) {
    for (int k = 0; k <= g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i)
                box[g.nat(i + 1, j + 1, k)] = src[((size_t)k * g.ny + j) * g.nx + i];
}
void unpack_u(const Geo& g, const float* box, float* dst) {
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i <= g.nx; ++i)
                dst[((size_t)k * g.ny + j) * (g.nx + 1) + i] = box[g.nat(i, j + 1, k + 1)];
}
void unpack_v(const Geo& g, const float* box, float* dst) {
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j <= g.ny; ++j)
            for (int i = 0; i < g.nx; ++i)
                dst[((size_t)k * (g.ny + 1) + j) * g.nx + i] = box[g.nat(i + 1, j, k + 1)];
}
void unpack_w(const Geo& g, const float* box, float* dst) {
    for (int k = 0; k <= g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i)
                dst[((size_t)k * g.ny + j) * g.nx + i] = box[g.nat(i + 1, j + 1, k)];
}
void unpack_cells(const Geo& g, const float* box, float* dst) {
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i)
                dst[((size_t)k * g.ny + j) * g.nx + i] = box[g.nat(i + 1, j + 1, k + 1)];
}
// Wall-normal faces carry zero normal velocity.
void zero_walls(const Geo& g, const les_params& p, float* u, float* v, float* w) {
    for (int k = 0; k < g.nz + 2; ++k)
        for (int i = 0; i < g.nx + 2; ++i) {
            v[g.nat(i, 0, k)] = 0.f;
            v[g.nat(i, g.ny, k)] = 0.f;
        }
    for (int j = 0; j < g.ny + 2; ++j)
        for (int i = 0; i < g.nx + 2; ++i) {
            w[g.nat(i, j, 0)] = 0.f;
            w[g.nat(i, j, g.nz)] = 0.f;
        }
    for (int k = 0; k < g.nz + 2; ++k)
        for (int j = 0; j < g.ny + 2; ++j) {
            if (p.bc[LES_XM] != LES_BC_INFLOW) u[g.nat(0, j, k)] = 0.f;
            if (p.bc[LES_XP] != LES_BC_OUTFLOW) u[g.nat(g.nx, j, k)] = 0.f;
        }
}

// Per-cell flag byte: cell solid, and solidity of the east / north / top
// face (a face is solid when either cell it separates is solid; a boundary
// face looks at its one cell).
std::vector<uint8_t> build_flags(const Geo& g, const std::vector<uint8_t>& mask) {
    std::vector<uint8_t> fl((size_t)g.ntot, 0);
    auto solid = [&](int i, int j, int k) {   // 1-based, clamped
        i = std::min(std::max(i, 1), g.nx);
        j = std::min(std::max(j, 1), g.ny);
        k = std::min(std::max(k, 1), g.nz);
        return mask[((size_t)(k - 1) * g.ny + (j - 1)) * g.nx + (i - 1)] != 0;
    };
    for (int k = 1; k <= g.nz; ++k)
        for (int j = 1; j <= g.ny; ++j)
            for (int i = 0; i <= g.nx; ++i) {
                uint8_t b = 0;
                if (i >= 1 && solid(i, j, k)) b |= F_CSOLID;
                if (solid(i, j, k) || solid(i + 1, j, k)) b |= F_USOLID;
                if (i >= 1 && (solid(i, j, k) || solid(i, j + 1, k))) b |= F_VSOLID;
                if (i >= 1 && (solid(i, j, k) || solid(i, j, k + 1))) b |= F_WSOLID;
                fl[g.nat(i, j, k)] = b;
            }
    return fl;
}

int upload_velocity(les_handle* h, const std::vector<float>& u, const std::vector<float>& v,
                    const std::vector<float>& w) {
    const size_t bytes = (size_t)h->g.ntot * sizeof(float);
    for (int b = 0; b < 2; ++b) {
        CK(hipMemcpyAsync(h->f.u[b], u.data(), bytes, hipMemcpyHostToDevice, h->stream));
        CK(hipMemcpyAsync(h->f.v[b], v.data(), bytes, hipMemcpyHostToDevice, h->stream));
        CK(hipMemcpyAsync(h->f.w[b], w.data(), bytes, hipMemcpyHostToDevice, h->stream));
        CK(launch_bc(h->g, h->stream, h->f.u[b], h->f.v[b], h->f.w[b]));
    }
    CK(hipStreamSynchronize(h->stream));
    return LES_OK;
}

int download(les_handle* h, const float* dev, std::vector<float>& host) {
    host.resize((size_t)h->g.ntot);
    CK(hipMemcpyAsync(host.data(), dev, host.size() * sizeof(float), hipMemcpyDeviceToHost,
                      h->stream));
    CK(hipStreamSynchronize(h->stream));
    return LES_OK;
}

// ------------------------------------------------------------- timing
enum Kind { KN_NUT = 0, KN_TEND, KN_INFLOW, KN_RHS, KN_SOR, KN_CHECK, KN_REBASE, KN_PROJECT, KN_BC };
constexpr long long kNoTag = -1;

// Record one pooled event on the handle's stream; returns its index.
size_t tmark(les_handle* h) {
    if (h->tev_used == h->tev.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return (size_t)-1;
        h->tev.push_back(e);
    }
    if (hipEventRecord(h->tev[h->tev_used], h->stream) != hipSuccess) return (size_t)-1;
    return h->tev_used++;
}

// Launch through f(), bracketed by two events when timing is on.  tag >= 0
// names the SOR check interval the launch belongs to (launches after the
// solve stopped return at once and are not counted).
template <class F>
hipError_t timed(les_handle* h, int kind, long long tag, F&& f, int count = 1) {
    if (!h->prm.timing) return f();
    const size_t a = tmark(h);
    const hipError_t e = f();
    const size_t b = tmark(h);
    if (a != (size_t)-1 && b != (size_t)-1) h->tpending.push_back({kind, a, b, tag, count});
    return e;
}

// After a stream synchronisation: fold the pending brackets into the
// counters.  SOR-family launches tagged with a check interval beyond the
// last one executed (last_check) are dropped.
void tresolve(les_handle* h, long long last_check) {
    for (const auto& br : h->tpending) {
        if (br.tag != kNoTag && br.tag > last_check) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->tev[br.a], h->tev[br.b]) == hipSuccess) {
            h->tms[br.kind] += ms;
            h->tcount[br.kind] += br.count;
        }
    }
    h->tpending.clear();
    h->tev_used = 0;
}

// ----------------------------------------------------- solve graphs
// Graph cache of run_solve, keyed by the pressure system and the sweep
// settings baked into the captured launches; the least recently used entry
// is replaced.
SolveGraph* solve_graph(les_handle* h, const PBufs& P, int var, int K, int R, double omega) {
    SolveGraph* best = &h->sgraph[0];
    for (SolveGraph& c : h->sgraph) {
        if (c.pd == P.pd[0] && c.ph == P.ph[0] && c.rhs == P.rhs[0] && c.variant == var && c.K == K &&
            c.R == R && c.omega == omega) {
            c.used = ++h->sgraph_tick;
            return &c;
        }
        if (c.used < best->used) best = &c;
    }
    for (hipGraphExec_t& ex : best->exec)
        if (ex) {
            (void)hipGraphExecDestroy(ex);
            ex = nullptr;
        }
    best->pd = P.pd[0];
    best->ph = P.ph[0];
    best->rhs = P.rhs[0];
    best->variant = var;
    best->K = K;
    best->R = R;
    best->omega = omega;
    best->used = ++h->sgraph_tick;
    return best;
}

// ------------------------------------------------------------- SOR driver
// Preconditions: ctl initialised, P.rhs filled, ctl->rhs2 computed.
// Runs the set-up rebase, then check intervals of K iterations (two
// half-sweeps each) followed by a residual check, folding the correction
// into the base every rebase_every checks.  Batches of checks are enqueued
// ahead; the device sets ctl->done and every later kernel of the batch
// returns at once.  The host reads the flag one batch behind.
// direct: launch every kernel itself (no captured graphs, no timing
// events), so the solve creates nothing on the device.
int run_solve(les_handle* h, const PBufs& P, double tol, int max_iter, les_solve_stats* out,
              bool direct = false) {
    const Geo& g = h->g;
    hipStream_t st = h->stream;
    Ctl* ctl = h->f.ctl;
    const bool timing = h->prm.timing && !direct;
    // kernel timing brackets (only with timing on)
    auto tm = [&](int kind, long long tag, auto&& f, int count = 1) -> hipError_t {
        return timing ? timed(h, kind, tag, f, count) : f();
    };
    const int K = h->prm.check_every;
    const int R = h->prm.rebase_every;
    const float omega = (float)h->prm.omega;
    // fused iterations alternate pd -> pa -> pd: an even interval ends on pd
    const int var = ((sor_fused(h->sor_variant) && (K & 1)) || (sor_fused2(h->sor_variant) && (K & 3)))
                        ? sor_default_variant(g)
                        : h->sor_variant;
    const bool fused = sor_fused(var);
    const bool fused2 = sor_fused2(var);
    const int nrel = (int)sor_sweep_blocks(g, var);
    double* part = h->f.part[0];
    double* rel0 = h->f.part[1];
    double* rel1 = h->f.part[2];

    // one check interval: K iterations, the bound, then the check (or,
    // every R-th interval, fold + rebase + check)
    auto interval = [&](long long cidx) -> hipError_t {
        // one check interval in 8 is timed as a whole: 2K back-to-back
        // half-sweeps (K fused iterations) between one pair of events
        const bool sample = timing && (cidx % 8 == 1);
        auto sweeps = [&]() -> hipError_t {
            if (fused2) {   // K is a multiple of 4: K/2 launches end on pd
                for (int it = 0; it < K; it += 2) {
                    const hipError_t e = launch_sor_rb2(g, st, P, (it >> 1) & 1, omega, it, rel0, rel1, ctl, var);
                    if (e != hipSuccess) return e;
                }
                return hipSuccess;
            }
            if (fused) {
                for (int it = 0; it < K; ++it) {
                    const hipError_t e = launch_sor_rb(g, st, P, it & 1, omega, it, rel0, rel1, ctl, var);
                    if (e != hipSuccess) return e;
                }
                return hipSuccess;
            }
            for (int it = 0; it < K; ++it) {
                hipError_t e = launch_sor(g, st, P, 0, omega, it, rel0, ctl, var);
                if (e != hipSuccess) return e;
                e = launch_sor(g, st, P, 1, omega, it, rel1, ctl, var);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        };
        hipError_t e = sample ? tm(KN_SOR, cidx, sweeps, fused2 ? K / 2 : (fused ? K : 2 * K)) : sweeps();
        if (e != hipSuccess) return e;
        e = launch_finalize(st, FIN_BOUND, nullptr, 0, rel0, rel1, nrel, ctl, h->prm.omega);
        if (e != hipSuccess) return e;
        if (rebase_due_at(cidx, K, R)) {
            e = launch_fold(g, st, P, ctl);
            if (e != hipSuccess) return e;
            return tm(KN_REBASE, cidx, [&] { return launch_rebase(g, st, P, part, rel0, rel1, nrel, ctl, 1); });
        }
        // the checks are sampled with the sweeps (one interval in 8): an
        // event pair around every one of them would cost more than they do
        if (sample) return tm(KN_CHECK, cidx, [&] { return launch_check(g, st, P, part, rel0, rel1, nrel, ctl); });
        return launch_check(g, st, P, part, rel0, rel1, nrel, ctl);
    };
    // Without timing, aligned runs of kSolveGraphChecks intervals replay a
    // captured graph (its kernels read every decision from the control
    // block, so a replay equals the launches it was captured from).
    SolveGraph* sg = nullptr;
    if (!timing && !direct && st != nullptr && R % kSolveGraphChecks == 0) sg = solve_graph(h, P, var, K, R, h->prm.omega);
    // Rebase pattern of the aligned run of intervals c0+1 .. c0+8: 2 inside
    // the early-fold phase, 1 past it when the run ends on a multiple of R,
    // 0 otherwise; -1 for a run that straddles the phase boundary (launched
    // directly).  A shape's graph is captured from representative interval
    // numbers with the same pattern.
    const long long early_end = kEarlyFoldIters / K;   // last interval of the early phase
    const long long late0 = ((early_end + R) / R) * R;    // a multiple of R past it
    auto run_shape = [&](long long c0) -> int {
        if (c0 + kSolveGraphChecks <= early_end) return 2;
        if (c0 + 1 <= early_end) return -1;
        return rebase_due_at(c0 + kSolveGraphChecks, K, R) ? 1 : 0;
    };
    auto replay = [&](int shape) -> int {
        hipGraphExec_t& ex = sg->exec[shape];
        if (!ex) {
            const long long c0 = shape == 2 ? 0 : (shape == 1 ? late0 + R - kSolveGraphChecks : late0);
            hipGraph_t gph = nullptr;
            CK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipSuccess;
            for (int q = 0; q < kSolveGraphChecks && e == hipSuccess; ++q) e = interval(c0 + q + 1);
            const hipError_t ce = hipStreamEndCapture(st, &gph);
            CK(e);
            CK(ce);
            const hipError_t ie = hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gph);
            CK(ie);
        }
        CK(hipGraphLaunch(ex, st));
        return LES_OK;
    };

    CK(launch_fold(g, st, P, ctl));
    CK(tm(KN_REBASE, 0, [&] { return launch_rebase(g, st, P, part, nullptr, nullptr, 0, ctl, 0); }));
    const long long n_checks = max_iter > 0 ? ((long long)max_iter + K - 1) / K : 0;
    long long c = 0;
    // batches of 2, 2, 4 intervals (a solve that converges at once is
    // noticed early), then 8, 16, 32, 64 (capped below): from interval 8 on
    // every batch starts on a multiple of kSolveGraphChecks
    static const int kBatches[] = {2, 2, 4, 8, 16, 32, 64};
    // a batch spans at most ~1024 iterations (a multiple of the graph's
    // intervals): after convergence the launches still queued return at
    // once but each still costs a dispatch, and at most about two batches
    // are queued when the host sees the flag
    const int batch_cap = std::max(kSolveGraphChecks, (1024 / std::max(K, 1)) / kSolveGraphChecks * kSolveGraphChecks);
    int bi = 0;
    int slot = 0;
    bool pending = false;
    while (c < n_checks) {
        const long long nb = std::min<long long>(std::min(kBatches[bi], batch_cap), n_checks - c);
        long long q = 0;
        while (q < nb) {
            const long long c0 = c + q;   // intervals c0+1, ...
            if (sg && c0 % kSolveGraphChecks == 0 && q + kSolveGraphChecks <= nb && run_shape(c0) >= 0) {
                const int rc = replay(run_shape(c0));
                if (rc != LES_OK) return rc;
                q += kSolveGraphChecks;
            } else {
                CK(interval(c0 + 1));
                q += 1;
            }
        }
        c += nb;
        CK(hipMemcpyAsync(&h->h_flag[slot], &ctl->done, sizeof(int), hipMemcpyDeviceToHost, st));
        CK(hipEventRecord(h->ev[slot], st));
        if (pending) {
            CK(hipEventSynchronize(h->ev[1 - slot]));
            if (h->h_flag[1 - slot] != 0) break;
        }
        pending = true;
        slot = 1 - slot;
        if (bi + 1 < (int)(sizeof kBatches / sizeof kBatches[0])) ++bi;
    }
    CK(hipMemcpyAsync(h->h_ctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    const Ctl& hc = *h->h_ctl;
    // the check that stopped the solve is interval ceil(m / K)
    if (timing) tresolve(h, ((long long)hc.m + K - 1) / K);
    if (out) {
        out->iters = hc.m;
        out->resid = hc.resid;
        out->rhs_norm = std::sqrt(hc.rhs2);
        out->reltmp2 = hc.reltmp2;
        out->converged = (hc.done == 1 || (hc.done == 0 && hc.resid <= tol)) ? 1 : 0;
    }
    if (hc.done == 3 || !std::isfinite(hc.rhs2)) return set_err(h, LES_ENONFINITE, "non-finite residual norm");
    if (hc.done == 2 || (hc.done == 0 && !(hc.resid <= tol))) return LES_NOT_CONVERGED;
    return LES_OK;
}

int ensure_solve_arena(les_handle* h) {
    if (h->solve_arena) return LES_OK;
    const size_t cb = align256((size_t)h->g.ctot * sizeof(float));
    const size_t total = 10 * cb + align256(sizeof(Ctl));
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, total);
    if (e != hipSuccess) return set_err(h, LES_ENOMEM, "hipMalloc(solve workspace)", e);
    h->solve_arena = p;
    CK(hipMemsetAsync(p, 0, total, h->stream));
    char* b = (char*)p;
    for (int c = 0; c < 2; ++c) {
        h->S.ph[c] = (float*)(b + (0 + c) * cb);
        h->S.pd[c] = (float*)(b + (2 + c) * cb);
        h->S.r0[c] = (float*)(b + (4 + c) * cb);
        h->S.rhs[c] = (float*)(b + (6 + c) * cb);
        h->S.pa[c] = (float*)(b + (8 + c) * cb);
    }
    h->ctl_save = (Ctl*)(b + 10 * cb);
    CK(hipStreamSynchronize(h->stream));
    return LES_OK;
}

// Residual after `iters` SOR iterations from the pair `start` against the
// step's right-hand side, run in the solve workspace (start and the step's
// pressure are not touched; the step's control block must be saved by the
// caller).
int trial_resid(les_handle* h, const PBufs& start, int iters, double* resid) {
    const Geo& g = h->g;
    hipStream_t s = h->stream;
    const size_t cb = (size_t)g.ctot * sizeof(float);
    for (int c = 0; c < 2; ++c) {
        CK(hipMemcpyAsync(h->S.ph[c], start.ph[c], cb, hipMemcpyDeviceToDevice, s));
        CK(hipMemcpyAsync(h->S.pd[c], start.pd[c], cb, hipMemcpyDeviceToDevice, s));
    }
    PBufs T = h->S;
    T.rhs[0] = h->f.P.rhs[0];
    T.rhs[1] = h->f.P.rhs[1];
    CK(launch_ctl_init(s, h->f.ctl, 0.0, iters, h->prm.check_every));
    CK(hipMemcpyAsync(&h->f.ctl->rhs2, &h->ctl_save->rhs2, sizeof(double), hipMemcpyDeviceToDevice, s));
    les_solve_stats st{};
    const int rc = run_solve(h, T, 0.0, iters, &st);
    if (rc < 0) return rc;
    *resid = st.resid;
    return LES_OK;
}

// Trial rule of the warm start: choose between the previous pressure and
// the network's candidate on the host.
int warm_choose(les_handle* h) {
    if (!h->warm_net || h->warm_rule != LES_WARM_TRIAL) return LES_OK;
    int rc = ensure_solve_arena(h);
    if (rc != LES_OK) return rc;
    hipStream_t s = h->stream;
    CK(hipMemcpyAsync(h->ctl_save, h->f.ctl, sizeof(Ctl), hipMemcpyDeviceToDevice, s));
    double ra = 0.0, rb = 0.0;
    if ((rc = trial_resid(h, h->f.P, h->warm_param, &ra)) != LES_OK) return rc;
    if ((rc = trial_resid(h, warm_candidate(h), h->warm_param, &rb)) != LES_OK) return rc;
    CK(hipMemcpyAsync(h->f.ctl, h->ctl_save, sizeof(Ctl), hipMemcpyDeviceToDevice, s));
    return warm_take(h, rb < ra ? 1 : 0, ra, rb);
}

}  // namespace

// ======================================================================
extern "C" {

int les_default_params(les_params* p) {
    if (!p) return LES_EINVAL;
    std::memset(p, 0, sizeof *p);
    p->omega = 1.8;
    p->tol = 1e-5;
    p->check_every = 4;
    p->max_iter = 20000;
    p->cs = 0.1;
    p->nu = 1.5e-5;
    p->alpha = -10.0;
    p->beta = -1.0;
    p->bc[LES_XM] = LES_BC_INFLOW;
    p->bc[LES_XP] = LES_BC_OUTFLOW;
    p->bc[LES_YM] = LES_BC_FREESLIP;
    p->bc[LES_YP] = LES_BC_FREESLIP;
    p->bc[LES_ZM] = LES_BC_NOSLIP;
    p->bc[LES_ZP] = LES_BC_FREESLIP;
    p->zero_guess = 0;
    p->rebase_every = 32;
    p->diagnostics = 1;
    p->timing = 0;
    return LES_OK;
}

}  // extern "C"

namespace {

// Metric table of one stretched axis (MetricRow rows of n + 2 floats),
// computed in float64 from the n cell widths and rounded once, and the
// float64 rows of its pressure-operator weights (M_WM, M_WP, M_DD) in
// `op`.  x_outflow: the axis ends in the outflow face (p = 0 on the face:
// 2/h^2 more on the last cell's diagonal).
std::vector<float> axis_metrics(const double* w, int n, bool x_outflow, std::vector<double>& op) {
    const int L = n + 2;
    std::vector<double> h(L), gf(L);
    for (int c = 1; c <= n; ++c) h[c] = w[c - 1];
    h[0] = h[1];
    h[n + 1] = h[n];
    for (int f = 0; f <= n; ++f) gf[f] = 0.5 * (h[f] + h[f + 1]);
    gf[n + 1] = gf[n];
    std::vector<float> m((size_t)kMetricRows * L, 0.f);
    auto at = [&](int row, int c) -> float& { return m[(size_t)row * L + c]; };
    for (int c = 0; c < L; ++c) {
        at(M_IH, c) = (float)(1.0 / h[c]);
        at(M_IG, c) = (float)(1.0 / gf[c]);
        const int f1 = c + 1 < L ? c + 1 : c;
        at(M_LO, c) = (float)(h[f1] / (h[c] + h[f1]));
        at(M_HI, c) = (float)(h[c] / (h[c] + h[f1]));
        at(M_H23, c) = (float)std::pow(h[c], 2.0 / 3.0);
        at(M_H, c) = (float)h[c];
    }
    op.assign((size_t)3 * L, 0.0);
    for (int c = 1; c <= n; ++c) {
        const double wm = c > 1 ? 1.0 / (h[c] * gf[c - 1]) : 0.0;
        const double wp = c < n ? 1.0 / (h[c] * gf[c]) : 0.0;
        double dd = wm + wp;
        if (c == n && x_outflow) dd += 2.0 / (h[c] * h[c]);
        at(M_WM, c) = (float)wm;
        at(M_WP, c) = (float)wp;
        at(M_DD, c) = (float)dd;
        op[(size_t)0 * L + c] = wm;
        op[(size_t)1 * L + c] = wp;
        op[(size_t)2 * L + c] = dd;
    }
    return m;
}

// Shared body of les_create and les_create_stretched (widths: NULL for a
// uniform grid, else the three per-axis width arrays).
int create_impl(const les_grid* gr, const les_spacing* s, const double* const* widths, double dt,
                const uint8_t* building_mask, const les_params* prm, les_handle** out) {
    if (!gr || !s || !out) return LES_EINVAL;
    *out = nullptr;
    if (gr->nx < 4 || gr->ny < 4 || gr->nz < 4) return LES_EINVAL;
    if (gr->nx > (1 << 20) || gr->ny > (1 << 20) || gr->nz > (1 << 20)) return LES_EINVAL;
    if (!finite_pos(s->dx) || !finite_pos(s->dy) || !finite_pos(s->dz) || !finite_pos(dt))
        return LES_EINVAL;
    les_params p;
    if (prm) p = *prm;
    else les_default_params(&p);
    if (!valid_params(p)) return LES_EINVAL;
    // stretched axes need the outflow face (a nonsingular operator)
    if (widths && p.bc[LES_XP] != LES_BC_OUTFLOW) return LES_EINVAL;
    const long long ncell = (long long)gr->nx * gr->ny * gr->nz;
    if (ncell > (1LL << 31)) return LES_EINVAL;

    les_handle* h = new (std::nothrow) les_handle();
    if (!h) return LES_ENOMEM;
    h->prm = p;
    h->g = make_geo(gr->nx, gr->ny, gr->nz, *s, dt, p);
    h->dt = dt;
    h->mask.assign((size_t)ncell, 0);
    if (building_mask) std::memcpy(h->mask.data(), building_mask, (size_t)ncell);
    auto fail = [&](int code) {
        les_destroy(h);
        return code;
    };
    if (hipGetDevice(&h->device) != hipSuccess) return fail(LES_EDEVICE);
    if (hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(LES_EDEVICE);
    h->stream = h->own_stream;

    const Geo& g = h->g;
    const size_t nb = align256((size_t)g.ntot * sizeof(float));
    const size_t cb = align256((size_t)g.ctot * sizeof(float));
    const size_t fb = align256((size_t)g.ntot);
    const size_t ncells = align256((size_t)ncell * sizeof(float));
    long long maxsweep = 0;
    for (int v = 0; v < kNumSorVariants; ++v) maxsweep = std::max<long long>(maxsweep, sor_sweep_blocks(g, v));
    const size_t nparts = (size_t)std::max<long long>(2LL * nblk(ncell), 2LL * maxsweep) + 64;
    const size_t pb = align256(nparts * sizeof(double));
    const size_t mb = widths ? align256((size_t)kMetricRows * (g.nx + g.ny + g.nz + 6) * sizeof(float)) +
                                   align256((size_t)3 * (g.nx + g.ny + g.nz + 6) * sizeof(double))
                             : 0;
    const size_t total = 13 * nb + fb + 2 * align256((size_t)g.nz * sizeof(float)) + ncells + 10 * cb +
                         3 * pb + align256(sizeof(Ctl)) + mb;
    void* arena = nullptr;
    if (hipMalloc(&arena, total) != hipSuccess) return fail(LES_ENOMEM);
    h->arena = arena;
    h->arena_bytes = total;
    char* b = (char*)arena;
    auto take = [&](size_t bytes) {
        char* r = b;
        b += bytes;
        return r;
    };
    for (int q = 0; q < 2; ++q) {
        h->f.u[q] = (float*)take(nb);
        h->f.v[q] = (float*)take(nb);
        h->f.w[q] = (float*)take(nb);
    }
    h->f.nut = (float*)take(nb);
    h->f.fu = (float*)take(nb); h->f.fv = (float*)take(nb); h->f.fw = (float*)take(nb);
    h->f.su = (float*)take(nb); h->f.sv = (float*)take(nb); h->f.sw = (float*)take(nb);
    h->f.flags = (uint8_t*)take(fb);
    h->f.prof = (float*)take(align256((size_t)g.nz * sizeof(float)));
    h->f.prof1 = (float*)take(align256((size_t)g.nz * sizeof(float)));
    h->f.stage = (float*)take(ncells);
    for (int c = 0; c < 2; ++c) h->f.P.ph[c] = (float*)take(cb);
    for (int c = 0; c < 2; ++c) h->f.P.pd[c] = (float*)take(cb);
    for (int c = 0; c < 2; ++c) h->f.P.r0[c] = (float*)take(cb);
    for (int c = 0; c < 2; ++c) h->f.P.rhs[c] = (float*)take(cb);
    for (int c = 0; c < 2; ++c) h->f.P.pa[c] = (float*)take(cb);
    for (int q = 0; q < 3; ++q) h->f.part[q] = (double*)take(pb);
    h->f.ctl = (Ctl*)take(align256(sizeof(Ctl)));
    float* metric = widths ? (float*)take(mb) : nullptr;

    if (hipMemsetAsync(arena, 0, total, h->stream) != hipSuccess) return fail(LES_EDEVICE);
    if (widths) {
        const int n3[3] = {g.nx, g.ny, g.nz};
        std::vector<float> all;
        std::vector<double> all_op, op;
        for (int a = 0; a < 3; ++a) {
            const std::vector<float> m = axis_metrics(widths[a], n3[a], a == 0 && g.outflow, op);
            all.insert(all.end(), m.begin(), m.end());
            all_op.insert(all_op.end(), op.begin(), op.end());
        }
        double* metric_op =
            (double*)((char*)metric + align256((size_t)kMetricRows * (g.nx + g.ny + g.nz + 6) * sizeof(float)));
        if (hipMemcpyAsync(metric, all.data(), all.size() * sizeof(float), hipMemcpyHostToDevice,
                           h->stream) != hipSuccess ||
            hipMemcpyAsync(metric_op, all_op.data(), all_op.size() * sizeof(double),
                           hipMemcpyHostToDevice, h->stream) != hipSuccess)
            return fail(LES_EDEVICE);
        // the copies must land before the host vectors go away
        if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(LES_EDEVICE);
        h->g.stretched = 1;
        h->g.mx = metric;
        h->g.my = metric + (size_t)kMetricRows * (g.nx + 2);
        h->g.mz = metric + (size_t)kMetricRows * (g.nx + g.ny + 4);
        h->g.wx = metric_op;
        h->g.wy = metric_op + (size_t)3 * (g.nx + 2);
        h->g.wz = metric_op + (size_t)3 * (g.nx + g.ny + 4);
        for (int a = 0; a < 3; ++a) h->widths[a].assign(widths[a], widths[a] + n3[a]);
    }
    std::vector<uint8_t> flags = build_flags(g, h->mask);
    if (hipMemcpyAsync(h->f.flags, flags.data(), flags.size(), hipMemcpyHostToDevice, h->stream) !=
        hipSuccess)
        return fail(LES_EDEVICE);
    if (hipHostMalloc((void**)&h->h_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess)
        return fail(LES_ENOMEM);
    if (hipHostMalloc((void**)&h->h_flag, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return fail(LES_ENOMEM);
    for (int q = 0; q < 2; ++q)
        if (hipEventCreateWithFlags(&h->ev[q], hipEventDisableTiming) != hipSuccess)
            return fail(LES_EDEVICE);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(LES_EDEVICE);
    h->prof.assign((size_t)g.nz, 0.f);
    h->prof1.assign((size_t)g.nz, 0.f);
    h->sor_variant = sor_default_variant(g);
    *out = h;
    return LES_OK;
}

}  // namespace

extern "C" {

int les_create(const les_grid* gr, const les_spacing* s, double dt, const uint8_t* building_mask,
               const les_params* prm, les_handle** out) {
    return create_impl(gr, s, nullptr, dt, building_mask, prm, out);
}

int les_create_stretched(const les_grid* gr, const double* hx, const double* hy, const double* hz,
                         double dt, const uint8_t* building_mask, const les_params* prm,
                         les_handle** out) {
    if (!gr || !hx || !hy || !hz || !out) return LES_EINVAL;
    *out = nullptr;
    if (gr->nx < 4 || gr->ny < 4 || gr->nz < 4) return LES_EINVAL;
    if (gr->nx > (1 << 20) || gr->ny > (1 << 20) || gr->nz > (1 << 20)) return LES_EINVAL;
    const double* w[3] = {hx, hy, hz};
    const int n3[3] = {gr->nx, gr->ny, gr->nz};
    double mean[3];
    for (int a = 0; a < 3; ++a) {
        double sum = 0.0;
        for (int c = 0; c < n3[a]; ++c) {
            if (!finite_pos(w[a][c])) return LES_EINVAL;
            sum += w[a][c];
        }
        mean[a] = sum / n3[a];
    }
    // the scalar spacings of the handle hold the mean widths (informational;
    // every stage of a stretched grid reads the per-axis tables)
    const les_spacing s{mean[0], mean[1], mean[2]};
    return create_impl(gr, &s, w, dt, building_mask, prm, out);
}

void les_destroy(les_handle* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->arena) (void)hipFree(h->arena);
    if (h->solve_arena) (void)hipFree(h->solve_arena);
    warm_free(h);
    twinned_free(h);
    if (h->h_ctl) (void)hipHostFree(h->h_ctl);
    if (h->h_flag) (void)hipHostFree(h->h_flag);
    for (int q = 0; q < 2; ++q)
        if (h->ev[q]) (void)hipEventDestroy(h->ev[q]);
    for (hipEvent_t e : h->tev) (void)hipEventDestroy(e);
    for (les::SolveGraph& c : h->sgraph)
        for (hipGraphExec_t ex : c.exec)
            if (ex) (void)hipGraphExecDestroy(ex);
    if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
    delete h;
}

const char* les_last_error(const les_handle* h) { return h ? h->err.c_str() : ""; }

int les_set_stream(les_handle* h, void* stream) {
    if (!h) return LES_EINVAL;
    CK(hipStreamSynchronize(h->stream));
    h->stream = stream ? (hipStream_t)stream : h->own_stream;
    return LES_OK;
}

int les_set_inflow(les_handle* h, const float* profile, float noise_amp, uint64_t seed) {
    if (!h || !profile) return LES_EINVAL;
    if (!(std::isfinite(noise_amp) && noise_amp >= 0.f)) return set_err(h, LES_EINVAL, "noise_amp");
    const Geo& g = h->g;
    for (int k = 0; k < g.nz; ++k)
        if (!std::isfinite(profile[k])) return set_err(h, LES_EINVAL, "profile not finite");
    std::memcpy(h->prof.data(), profile, (size_t)g.nz * sizeof(float));
    h->amp = noise_amp;
    h->seed = seed;
    h->interp = false;
    CK(hipMemcpyAsync(h->f.prof, h->prof.data(), (size_t)g.nz * sizeof(float),
                      hipMemcpyHostToDevice, h->stream));
    if (!h->have_inflow) {
        // initial wind profile on fluid u-faces, zero on solid ones
        std::vector<float> u((size_t)g.ntot, 0.f), v((size_t)g.ntot, 0.f), w((size_t)g.ntot, 0.f);
        std::vector<uint8_t> flags = build_flags(g, h->mask);
        for (int k = 1; k <= g.nz; ++k)
            for (int j = 1; j <= g.ny; ++j)
                for (int i = 0; i <= g.nx; ++i)
                    u[g.nat(i, j, k)] = (flags[g.nat(i, j, k)] & F_USOLID) ? 0.f : profile[k - 1];
        zero_walls(g, h->prm, u.data(), v.data(), w.data());
        int rc = upload_velocity(h, u, v, w);
        if (rc != LES_OK) return rc;
        for (int c = 0; c < 2; ++c) {
            CK(launch_fill(h->stream, h->f.P.ph[c], g.ctot, 0.f));
            CK(launch_fill(h->stream, h->f.P.pd[c], g.ctot, 0.f));
        }
        h->have_inflow = true;
    }
    CK(hipStreamSynchronize(h->stream));
    return LES_OK;
}

int les_set_inflow_pair(les_handle* h, double t0, const float* prof0, double t1,
                        const float* prof1) {
    if (!h || !prof0 || !prof1) return LES_EINVAL;
    if (!h->have_inflow) return set_err(h, LES_ESTATE, "les_set_inflow (or les_set_fields) first");
    if (!(std::isfinite(t0) && std::isfinite(t1) && t1 > t0))
        return set_err(h, LES_EINVAL, "need finite t0 < t1");
    const Geo& g = h->g;
    for (int k = 0; k < g.nz; ++k)
        if (!std::isfinite(prof0[k]) || !std::isfinite(prof1[k]))
            return set_err(h, LES_EINVAL, "profile not finite");
    std::memcpy(h->prof.data(), prof0, (size_t)g.nz * sizeof(float));
    std::memcpy(h->prof1.data(), prof1, (size_t)g.nz * sizeof(float));
    h->t0 = t0;
    h->t1 = t1;
    h->interp = true;
    CK(hipMemcpyAsync(h->f.prof, h->prof.data(), (size_t)g.nz * sizeof(float),
                      hipMemcpyHostToDevice, h->stream));
    CK(hipMemcpyAsync(h->f.prof1, h->prof1.data(), (size_t)g.nz * sizeof(float),
                      hipMemcpyHostToDevice, h->stream));
    CK(hipStreamSynchronize(h->stream));
    return LES_OK;
}

// Weight of the second profile sample for the next step; 0 when no pair is set.
static float inflow_weight(const les_handle* h) {
    return h->interp ? inflow_weight_at(h->step, h->dt, h->t0, h->t1) : 0.f;
}

int les_step(les_handle* h, int32_t n, les_step_stats* st) {
    if (!h || n < 0) return LES_EINVAL;
    if (!h->have_inflow) return set_err(h, LES_ESTATE, "les_set_inflow (or les_set_fields) first");
    auto t0 = std::chrono::steady_clock::now();
    const Geo& g = h->g;
    const les_params& p = h->prm;
    hipStream_t s = h->stream;
    // (Cs Delta)^2 with Delta = (dx dy dz)^(1/3); a stretched grid's kernel
    // forms each cell's own filter width from the tables and takes Cs^2
    const double delta = std::cbrt((double)g.dx * g.dy * g.dz);
    const float c2 = g.stretched ? (float)(p.cs * p.cs) : (float)((p.cs * delta) * (p.cs * delta));
    les_step_stats acc{};
    if (st) acc.iters_out = st->iters_out;
    acc.div_new_last = -1.0;
    acc.cfl_last = -1.0;
    acc.warm_r_prev_last = -1.0;
    acc.warm_r_net_last = -1.0;
    int worst = LES_OK;
    for (int q = 0; q < n; ++q) {
        const int a = h->cur, b = 1 - h->cur;
        const int first = h->have_old ? 0 : 1;
        if (g.stretched) {
            CK(timed(h, KN_NUT, kNoTag, [&] { return launch_nut_str(g, s, h->f.u[a], h->f.v[a], h->f.w[a], h->f.nut, c2); }));
            CK(timed(h, KN_TEND, kNoTag, [&] {
                return launch_tendency_str(g, s, h->f.u[a], h->f.v[a], h->f.w[a], h->f.nut, h->f.fu,
                                           h->f.fv, h->f.fw, h->f.su, h->f.sv, h->f.sw, h->f.flags,
                                           h->f.u[b], h->f.v[b], h->f.w[b], (float)p.nu, (float)p.alpha,
                                           (float)p.beta, first);
            }));
        } else {
            // nu_t, tendency, feedback and AB2 in one LDS-tiled pass
            CK(timed(h, KN_TEND, kNoTag, [&] {
                return launch_step_tile(g, s, h->f.u[a], h->f.v[a], h->f.w[a], h->f.nut, h->f.fu,
                                        h->f.fv, h->f.fw, h->f.su, h->f.sv, h->f.sw, h->f.flags,
                                        h->f.u[b], h->f.v[b], h->f.w[b], c2, (float)p.nu,
                                        (float)p.alpha, (float)p.beta, first);
            }));
        }
        h->have_old = true;
        if (g.inflow)
            CK(timed(h, KN_INFLOW, kNoTag, [&] {
                return launch_inflow(g, s, h->f.u[b], h->f.prof, h->interp ? h->f.prof1 : h->f.prof,
                                     inflow_weight(h), h->f.flags, h->amp, h->seed, h->step + 1);
            }));
        CK(launch_ctl_init(s, h->f.ctl, p.tol, p.max_iter, p.check_every));
        CK(timed(h, KN_RHS, kNoTag, [&] {
            return launch_rhs(g, s, h->f.u[b], h->f.v[b], h->f.w[b], h->f.P.rhs, h->f.part[0],
                              h->f.ctl, singular(h) ? 1 : 0);
        }));
        if (singular(h)) CK(launch_remove_mean_rhs(g, s, h->f.P.rhs, h->f.part[0], h->f.ctl));
        if (p.zero_guess)
            for (int c = 0; c < 2; ++c) {
                CK(launch_fill(s, h->f.P.ph[c], g.ctot, 0.f));
                CK(launch_fill(s, h->f.P.pd[c], g.ctot, 0.f));
            }
        int wrc = warm_pre(h);
        if (wrc == LES_OK) wrc = warm_choose(h);
        if (wrc != LES_OK) return wrc;
        les_solve_stats ss{};
        int rc = run_solve(h, h->f.P, p.tol, p.max_iter, &ss);
        if (rc < 0) return rc;
        if (rc == LES_NOT_CONVERGED) {
            acc.not_converged += 1;
            worst = LES_NOT_CONVERGED;
        }
        if (singular(h)) CK(launch_remove_mean_p(g, s, h->f.P, h->f.part[0], h->f.ctl));
        if ((wrc = warm_post(h)) != LES_OK) return wrc;
        if (h->warm_net) {
            int taken = 0;
            if ((wrc = warm_result(h, &taken, &acc.warm_r_prev_last, &acc.warm_r_net_last)) != LES_OK) return wrc;
            acc.warm_taken += taken;
        }
        CK(timed(h, KN_PROJECT, kNoTag, [&] { return launch_project(g, s, h->f.u[b], h->f.v[b], h->f.w[b], h->f.P); }));
        CK(timed(h, KN_BC, kNoTag, [&] { return launch_bc(g, s, h->f.u[b], h->f.v[b], h->f.w[b]); }));
        h->cur = b;
        h->step += 1;
        acc.steps += 1;
        acc.sor_iters_total += ss.iters;
        acc.sor_iters_last = ss.iters;
        acc.resid_last = ss.resid;
        acc.reltmp2_last = ss.reltmp2;
        acc.rhs_norm_last = ss.rhs_norm;
        acc.div_star_last = (double)g.dt * ss.rhs_norm;
        if (acc.iters_out) acc.iters_out[q] = ss.iters;
        if (p.diagnostics && q == n - 1) {
            CK(launch_diag(g, s, h->f.u[b], h->f.v[b], h->f.w[b], h->f.part[0], h->f.ctl));
            CK(hipMemcpyAsync(h->h_ctl, h->f.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
            CK(hipStreamSynchronize(s));
            acc.div_new_last = std::sqrt(h->h_ctl->div2);
            acc.cfl_last = h->h_ctl->cfl;
            if (!std::isfinite(acc.div_new_last) || !std::isfinite(acc.cfl_last)) {
                if (st) *st = acc;
                return set_err(h, LES_ENONFINITE, "non-finite divergence or CFL");
            }
        }
    }
    CK(hipStreamSynchronize(s));
    if (p.timing) tresolve(h, kNoTag);
    acc.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = acc;
    return worst;
}

}  // extern "C"

// Stand-alone solve of the pressure system S (rhs and start already in S,
// correction cleared): control block, rhs norm (mean removal without an
// outflow face), SOR to tol, p mean.  direct: no graphs, no timing events.
int les::solve_system(les_handle* h, double tol, int32_t max_iter, les_solve_stats* st,
                      const PBufs& S, bool direct) {
    const Geo& g = h->g;
    hipStream_t s = h->stream;
    CK(launch_ctl_init(s, h->f.ctl, tol, max_iter, h->prm.check_every));
    if (singular(h)) {
        CK(launch_colour_norm(g, s, S.rhs, h->f.part[0], h->f.ctl, 1));
        CK(launch_remove_mean_rhs(g, s, S.rhs, h->f.part[0], h->f.ctl));
    } else {
        CK(launch_colour_norm(g, s, S.rhs, h->f.part[0], h->f.ctl, 0));
    }
    int rc = run_solve(h, S, tol, max_iter, st, direct);
    if (rc < 0) return rc;
    if (singular(h)) CK(launch_remove_mean_p(g, s, S, h->f.part[0], h->f.ctl));
    return rc;
}

extern "C" {

static int solve_common(les_handle* h, double tol, int32_t max_iter, les_solve_stats* st) {
    return solve_system(h, tol, max_iter, st, h->S, false);
}

int les_pressure_solve(les_handle* h, const float* rhs, float* p, double tol, int32_t max_iter,
                       les_solve_stats* st) {
    if (!h || !rhs || !p) return LES_EINVAL;
    if (!finite_pos(tol) || max_iter < 0) return set_err(h, LES_EINVAL, "tol/max_iter");
    int rc = ensure_solve_arena(h);
    if (rc != LES_OK) return rc;
    const Geo& g = h->g;
    hipStream_t s = h->stream;
    const size_t bytes = (size_t)g.nx * g.ny * g.nz * sizeof(float);
    // stage holds one cell array: load rhs, scatter, load p, scatter
    CK(hipMemcpyAsync(h->f.stage, rhs, bytes, hipMemcpyHostToDevice, s));
    CK(launch_cells_to_colour(g, s, h->f.stage, h->S.rhs));
    CK(hipMemcpyAsync(h->f.stage, p, bytes, hipMemcpyHostToDevice, s));
    CK(launch_cells_to_colour(g, s, h->f.stage, h->S.ph));
    for (int c = 0; c < 2; ++c) CK(launch_fill(s, h->S.pd[c], g.ctot, 0.f));
    rc = solve_common(h, tol, max_iter, st);
    if (rc < 0) return rc;
    CK(launch_pair_to_cells(g, s, h->S, h->f.stage));
    CK(hipMemcpyAsync(p, h->f.stage, bytes, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    return rc;
}

int les_pressure_solve_dev(les_handle* h, const float* d_rhs, float* d_p, double tol,
                           int32_t max_iter, les_solve_stats* st, void* stream) {
    if (!h || !d_rhs || !d_p) return LES_EINVAL;
    if (!finite_pos(tol) || max_iter < 0) return set_err(h, LES_EINVAL, "tol/max_iter");
    int rc = ensure_solve_arena(h);
    if (rc != LES_OK) return rc;
    hipStream_t saved = h->stream;
    if (stream) h->stream = (hipStream_t)stream;
    const Geo& g = h->g;
    hipStream_t s = h->stream;
    auto body = [&]() -> int {
        CK(launch_cells_to_colour(g, s, d_rhs, h->S.rhs));
        CK(launch_cells_to_colour(g, s, d_p, h->S.ph));
        for (int c = 0; c < 2; ++c) CK(launch_fill(s, h->S.pd[c], g.ctot, 0.f));
        int r = solve_common(h, tol, max_iter, st);
        if (r < 0) return r;
        CK(launch_pair_to_cells(g, s, h->S, d_p));
        return r;
    };
    rc = body();
    h->stream = saved;
    return rc;
}

int les_get_fields(les_handle* h, float* u, float* v, float* w, float* p) {
    if (!h) return LES_EINVAL;
    const Geo& g = h->g;
    std::vector<float> box;
    int rc;
    if (u) {
        if ((rc = download(h, h->f.u[h->cur], box)) != LES_OK) return rc;
        unpack_u(g, box.data(), u);
    }
    if (v) {
        if ((rc = download(h, h->f.v[h->cur], box)) != LES_OK) return rc;
        unpack_v(g, box.data(), v);
    }
    if (w) {
        if ((rc = download(h, h->f.w[h->cur], box)) != LES_OK) return rc;
        unpack_w(g, box.data(), w);
    }
    if (p) {
        CK(launch_pair_to_cells(g, h->stream, h->f.P, h->f.stage));
        CK(hipMemcpyAsync(p, h->f.stage, (size_t)g.nx * g.ny * g.nz * sizeof(float),
                          hipMemcpyDeviceToHost, h->stream));
        CK(hipStreamSynchronize(h->stream));
    }
    return LES_OK;
}

int les_get_fields_dev(les_handle* h, float* d_u, float* d_v, float* d_w, float* d_p,
                       void* stream) {
    if (!h) return LES_EINVAL;
    const Geo& g = h->g;
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    // owned sub-boxes copied row by row with 3-D copies
    auto copy3 = [&](float* dst, const float* src, int nxo, int nyo, int nzo, int i0, int j0,
                     int k0) -> hipError_t {
        hipMemcpy3DParms prm{};
        prm.srcPtr = make_hipPitchedPtr((void*)src, (size_t)g.sx * sizeof(float), g.sx, g.ny + 2);
        prm.srcPos = make_hipPos((size_t)i0 * sizeof(float), (size_t)j0, (size_t)k0);
        prm.dstPtr = make_hipPitchedPtr(dst, (size_t)nxo * sizeof(float), nxo, nyo);
        prm.dstPos = make_hipPos(0, 0, 0);
        prm.extent = make_hipExtent((size_t)nxo * sizeof(float), (size_t)nyo, (size_t)nzo);
        prm.kind = hipMemcpyDeviceToDevice;
        return hipMemcpy3DAsync(&prm, s);
    };
    if (d_u) CK(copy3(d_u, h->f.u[h->cur], g.nx + 1, g.ny, g.nz, 0, 1, 1));
    if (d_v) CK(copy3(d_v, h->f.v[h->cur], g.nx, g.ny + 1, g.nz, 1, 0, 1));
    if (d_w) CK(copy3(d_w, h->f.w[h->cur], g.nx, g.ny, g.nz + 1, 1, 1, 0));
    if (d_p) CK(launch_pair_to_cells(g, s, h->f.P, d_p));
    return LES_OK;
}

int les_set_fields(les_handle* h, const float* u, const float* v, const float* w, const float* p,
                   int32_t reset_history) {
    if (!h) return LES_EINVAL;
    const Geo& g = h->g;
    std::vector<float> U, V, W;
    int rc;
    if ((rc = download(h, h->f.u[h->cur], U)) != LES_OK) return rc;
    if ((rc = download(h, h->f.v[h->cur], V)) != LES_OK) return rc;
    if ((rc = download(h, h->f.w[h->cur], W)) != LES_OK) return rc;
    if (u) pack_u(g, u, U.data());
    if (v) pack_v(g, v, V.data());
    if (w) pack_w(g, w, W.data());
    zero_walls(g, h->prm, U.data(), V.data(), W.data());
    if ((rc = upload_velocity(h, U, V, W)) != LES_OK) return rc;
    if (p) {
        const size_t bytes = (size_t)g.nx * g.ny * g.nz * sizeof(float);
        CK(hipMemcpyAsync(h->f.stage, p, bytes, hipMemcpyHostToDevice, h->stream));
        CK(launch_cells_to_colour(g, h->stream, h->f.stage, h->f.P.ph));
        for (int c = 0; c < 2; ++c) CK(launch_fill(h->stream, h->f.P.pd[c], g.ctot, 0.f));
        CK(hipStreamSynchronize(h->stream));
    }
    if (reset_history) h->have_old = false;
    h->have_inflow = true;
    return LES_OK;
}

int les_set_initial_guess_dev(les_handle* h, const float* d_p, void* stream) {
    if (!h || !d_p) return LES_EINVAL;
    const Geo& g = h->g;
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    CK(launch_cells_to_colour(g, s, d_p, h->f.P.ph));
    for (int c = 0; c < 2; ++c) CK(launch_fill(s, h->f.P.pd[c], g.ctot, 0.f));
    return LES_OK;
}

int les_get_aux(les_handle* h, int32_t which, float* a, float* b, float* c) {
    if (!h) return LES_EINVAL;
    const Geo& g = h->g;
    std::vector<float> box;
    int rc;
    switch (which) {
        case 0:
            if (!a) return LES_OK;
            if ((rc = download(h, h->f.nut, box)) != LES_OK) return rc;
            unpack_cells(g, box.data(), a);
            return LES_OK;
        case 1:
            if (!a) return LES_OK;
            CK(launch_colour_to_cells(g, h->stream, h->f.P.rhs, h->f.stage));
            CK(hipMemcpyAsync(a, h->f.stage, (size_t)g.nx * g.ny * g.nz * sizeof(float),
                              hipMemcpyDeviceToHost, h->stream));
            CK(hipStreamSynchronize(h->stream));
            return LES_OK;
        case 2:
        case 3: {
            float* src[3] = {which == 2 ? h->f.fu : h->f.su, which == 2 ? h->f.fv : h->f.sv,
                             which == 2 ? h->f.fw : h->f.sw};
            if (a) {
                if ((rc = download(h, src[0], box)) != LES_OK) return rc;
                unpack_u(g, box.data(), a);
            }
            if (b) {
                if ((rc = download(h, src[1], box)) != LES_OK) return rc;
                unpack_v(g, box.data(), b);
            }
            if (c) {
                if ((rc = download(h, src[2], box)) != LES_OK) return rc;
                unpack_w(g, box.data(), c);
            }
            return LES_OK;
        }
        default:
            return set_err(h, LES_EINVAL, "les_get_aux: unknown which");
    }
}

int les_get_ghosted(les_handle* h, float* u, float* v, float* w) {
    if (!h) return LES_EINVAL;
    const Geo& g = h->g;
    std::vector<float> box;
    float* dst[3] = {u, v, w};
    float* src[3] = {h->f.u[h->cur], h->f.v[h->cur], h->f.w[h->cur]};
    for (int q = 0; q < 3; ++q) {
        if (!dst[q]) continue;
        int rc = download(h, src[q], box);
        if (rc != LES_OK) return rc;
        for (int k = 0; k < g.nz + 2; ++k)
            for (int j = 0; j < g.ny + 2; ++j)
                for (int i = 0; i < g.nx + 2; ++i)
                    dst[q][((size_t)k * (g.ny + 2) + j) * (g.nx + 2) + i] = box[g.nat(i, j, k)];
    }
    return LES_OK;
}

int les_autotune(les_handle* h, int32_t reps, int32_t* chosen, double* us_per_sweep) {
    if (!h || reps < 1 || reps > 1000) return LES_EINVAL;
    int rc = ensure_solve_arena(h);
    if (rc != LES_OK) return rc;
    const Geo& g = h->g;
    hipStream_t s = h->stream;
    // time the sweep variants on the stand-alone solve workspace (the
    // time-stepping state is not touched); the control block is set so that
    // no sweep is skipped
    CK(launch_ctl_init(s, h->f.ctl, 1e-30, 1 << 30, 1 << 20));
    hipEvent_t a = nullptr, b = nullptr;
    CK(hipEventCreate(&a));
    CK(hipEventCreate(&b));
    double best = 1e300;
    int best_v = h->sor_variant;
    for (int v = 0; v < kNumSorVariants; ++v) {
        // fused iterations need an even check interval, two per launch a
        // multiple of 4
        if ((sor_fused(v) && (h->prm.check_every & 1)) || (sor_fused2(v) && (h->prm.check_every & 3))) {
            if (us_per_sweep) us_per_sweep[v] = 0.0;
            continue;
        }
        // two launches: two half-sweeps, two fused iterations or four (the
        // time is charged per half-sweep below)
        auto pair = [&]() -> hipError_t {
            for (int w = 0; w < 2; ++w) {
                const hipError_t e =
                    sor_fused2(v) ? launch_sor_rb2(g, s, h->S, w, 1.0f, 0, nullptr, nullptr, h->f.ctl, v)
                    : sor_fused(v) ? launch_sor_rb(g, s, h->S, w, 1.0f, 0, nullptr, nullptr, h->f.ctl, v)
                                   : launch_sor(g, s, h->S, w, 1.0f, 0, nullptr, h->f.ctl, v);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        };
        CK(pair());
        CK(hipEventRecord(a, s));
        for (int r = 0; r < reps; ++r) CK(pair());
        CK(hipEventRecord(b, s));
        CK(hipEventSynchronize(b));
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, a, b));
        const double us = 1e3 * ms / ((sor_fused2(v) ? 8.0 : (sor_fused(v) ? 4.0 : 2.0)) * reps);
        if (us_per_sweep) us_per_sweep[v] = us;
        if (us < best) {
            best = us;
            best_v = v;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    for (int c = 0; c < 2; ++c) CK(launch_fill(s, h->S.pd[c], g.ctot, 0.f));
    for (int c = 0; c < 2; ++c) CK(launch_fill(s, h->S.pa[c], g.ctot, 0.f));
    CK(hipStreamSynchronize(s));
    h->sor_variant = best_v;
    if (chosen) *chosen = best_v;
    return LES_OK;
}

int les_set_sor_variant(les_handle* h, int32_t variant) {
    if (!h || variant < 0 || variant >= kNumSorVariants) return LES_EINVAL;
    if (sor_fused(variant) && (h->prm.check_every & 1))
        return set_err(h, LES_EINVAL, "fused sweep variants need an even check interval");
    if (sor_fused2(variant) && (h->prm.check_every & 3))
        return set_err(h, LES_EINVAL, "two-iteration sweep variants need a check interval that is a multiple of 4");
    h->sor_variant = variant;
    return LES_OK;
}

int les_get_timing(les_handle* h, les_timing* out, int32_t reset) {
    if (!h || !out) return LES_EINVAL;
    for (int q = 0; q < LES_NUM_KERNELS; ++q) {
        out->ms[q] = h->tms[q];
        out->launches[q] = h->tcount[q];
        if (reset) {
            h->tms[q] = 0.0;
            h->tcount[q] = 0;
        }
    }
    return LES_OK;
}

int les_get_step(const les_handle* h, int64_t* step) {
    if (!h || !step) return LES_EINVAL;
    *step = h->step;
    return LES_OK;
}

// ------------------------------------------------------------ checkpoint
namespace {
struct StateHeader {
    uint32_t magic;
    int32_t nx, ny, nz;
    int32_t bc[6];
    int64_t step;
    int32_t have_old, have_inflow;
    float amp;
    int32_t interp;
    uint64_t seed;
    double t0, t1;
    int64_t ntot, ctot;
};
}  // namespace

int les_state_size(const les_handle* h, int64_t* bytes) {
    if (!h || !bytes) return LES_EINVAL;
    const Geo& g = h->g;
    *bytes = (int64_t)sizeof(StateHeader) + 2LL * g.nz * 4 + 9LL * g.ntot * 4 + 4LL * g.ctot * 4;
    return LES_OK;
}

int les_get_state(les_handle* h, void* buf, int64_t bytes) {
    int64_t need = 0;
    if (!h || !buf || les_state_size(h, &need) != LES_OK || bytes != need) return LES_EINVAL;
    const Geo& g = h->g;
    StateHeader hd{};
    hd.magic = kStateMagic;
    hd.nx = g.nx; hd.ny = g.ny; hd.nz = g.nz;
    for (int f = 0; f < 6; ++f) hd.bc[f] = h->prm.bc[f];
    hd.step = h->step;
    hd.have_old = h->have_old;
    hd.have_inflow = h->have_inflow;
    hd.amp = h->amp;
    hd.seed = h->seed;
    hd.interp = h->interp;
    hd.t0 = h->t0;
    hd.t1 = h->t1;
    hd.ntot = g.ntot;
    hd.ctot = g.ctot;
    char* b = (char*)buf;
    std::memcpy(b, &hd, sizeof hd);
    b += sizeof hd;
    std::memcpy(b, h->prof.data(), (size_t)g.nz * 4);
    b += (size_t)g.nz * 4;
    std::memcpy(b, h->prof1.data(), (size_t)g.nz * 4);
    b += (size_t)g.nz * 4;
    const float* nat[9] = {h->f.u[h->cur], h->f.v[h->cur], h->f.w[h->cur], h->f.fu, h->f.fv,
                           h->f.fw, h->f.su, h->f.sv, h->f.sw};
    for (const float* src : nat) {
        CK(hipMemcpyAsync(b, src, (size_t)g.ntot * 4, hipMemcpyDeviceToHost, h->stream));
        b += (size_t)g.ntot * 4;
    }
    const float* col[4] = {h->f.P.ph[0], h->f.P.ph[1], h->f.P.pd[0], h->f.P.pd[1]};
    for (const float* src : col) {
        CK(hipMemcpyAsync(b, src, (size_t)g.ctot * 4, hipMemcpyDeviceToHost, h->stream));
        b += (size_t)g.ctot * 4;
    }
    CK(hipStreamSynchronize(h->stream));
    return LES_OK;
}

int les_set_state(les_handle* h, const void* buf, int64_t bytes) {
    int64_t need = 0;
    if (!h || !buf || les_state_size(h, &need) != LES_OK || bytes != need) return LES_EINVAL;
    const Geo& g = h->g;
    StateHeader hd;
    const char* b = (const char*)buf;
    std::memcpy(&hd, b, sizeof hd);
    if (hd.magic != kStateMagic || hd.nx != g.nx || hd.ny != g.ny || hd.nz != g.nz ||
        hd.ntot != g.ntot || hd.ctot != g.ctot)
        return set_err(h, LES_EINVAL, "checkpoint does not match this grid");
    for (int f = 0; f < 6; ++f)
        if (hd.bc[f] != h->prm.bc[f]) return set_err(h, LES_EINVAL, "checkpoint BC set differs");
    b += sizeof hd;
    std::memcpy(h->prof.data(), b, (size_t)g.nz * 4);
    b += (size_t)g.nz * 4;
    std::memcpy(h->prof1.data(), b, (size_t)g.nz * 4);
    b += (size_t)g.nz * 4;
    CK(hipMemcpyAsync(h->f.prof, h->prof.data(), (size_t)g.nz * 4, hipMemcpyHostToDevice, h->stream));
    CK(hipMemcpyAsync(h->f.prof1, h->prof1.data(), (size_t)g.nz * 4, hipMemcpyHostToDevice, h->stream));
    float* nat[9] = {h->f.u[h->cur], h->f.v[h->cur], h->f.w[h->cur], h->f.fu, h->f.fv,
                     h->f.fw, h->f.su, h->f.sv, h->f.sw};
    for (float* dst : nat) {
        CK(hipMemcpyAsync(dst, b, (size_t)g.ntot * 4, hipMemcpyHostToDevice, h->stream));
        b += (size_t)g.ntot * 4;
    }
    // the other velocity buffer gets the same walls / boundary faces
    const int o = 1 - h->cur;
    CK(hipMemcpyAsync(h->f.u[o], h->f.u[h->cur], (size_t)g.ntot * 4, hipMemcpyDeviceToDevice, h->stream));
    CK(hipMemcpyAsync(h->f.v[o], h->f.v[h->cur], (size_t)g.ntot * 4, hipMemcpyDeviceToDevice, h->stream));
    CK(hipMemcpyAsync(h->f.w[o], h->f.w[h->cur], (size_t)g.ntot * 4, hipMemcpyDeviceToDevice, h->stream));
    float* col[4] = {h->f.P.ph[0], h->f.P.ph[1], h->f.P.pd[0], h->f.P.pd[1]};
    for (float* dst : col) {
        CK(hipMemcpyAsync(dst, b, (size_t)g.ctot * 4, hipMemcpyHostToDevice, h->stream));
        b += (size_t)g.ctot * 4;
    }
    CK(hipStreamSynchronize(h->stream));
    h->step = hd.step;
    h->have_old = hd.have_old != 0;
    h->have_inflow = hd.have_inflow != 0;
    h->amp = hd.amp;
    h->seed = hd.seed;
    h->interp = hd.interp != 0;
    h->t0 = hd.t0;
    h->t1 = hd.t1;
    return LES_OK;
}

int64_t les_bc_range(const les_grid* gr) {
    if (!gr || gr->nx < 1 || gr->ny < 1 || gr->nz < 1) return 0;
    const long long n = bc_items(gr->nx, gr->ny, gr->nz);
    return (int64_t)nblk(n) * kBlock;   // launch size, padded to whole blocks
}

int les_bc_map(const les_grid* gr, int64_t item, int32_t* family, int32_t* a, int32_t* b) {
    if (!gr || !family || !a || !b || item < 0) return LES_EINVAL;
    int f, x, y;
    bc_item(gr->nx, gr->ny, gr->nz, item, f, x, y);
    *family = f;
    *a = x;
    *b = y;
    return LES_OK;
}

}  // extern "C"
