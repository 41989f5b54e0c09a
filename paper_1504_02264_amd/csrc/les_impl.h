// Internal declarations of the MI355X LES library: grid geometry, device
// field table, control block, kernel launchers.  Not part of the public ABI
// (include/les.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/les.h"
#include "../../include/lesnet.h"

namespace les {

constexpr int kBlock = 256;     // threads per block for the 1-D launches
constexpr int kNumXcd = 8;      // MI355X: 8 XCDs, blocks dispatched round-robin
constexpr int kMaxPartials = 1 << 20;
constexpr int kMaxEnsemble = 64;   // members of one ensemble

// Geometry, passed by value to every kernel.
//
// Natural ("box") layout for u, v, w and cell fields: index (i, j, k) with
// 1-based cells and one ghost layer, i in [0, nx+1], j in [0, ny+1],
// k in [0, nz+1]; x fastest, rows padded to sx floats (128-byte multiple).
//   u(i,j,k): east face of cell i (i = 0 is the x- boundary face)
//   v(i,j,k): north face of cell j, w(i,j,k): top face of cell k
//
// Colour-split layout for the pressure system (the red-black SOR of
// section 2.6 with the cells of one colour stored contiguously, so both
// half-sweeps are unit-stride): 0-based cell (i0, j0, k0) has colour
// c = (i0 + j0 + k0) & 1 and lives in colour array c at half-index
// ii = i0 >> 1 of row (j0, k0).  Rows have H = ceil(nx/2) entries and a
// pitch S >= H + 1 (128-byte multiple), with a zero ghost row before and
// after every plane, a zero ghost plane below and above, and a guard row
// in front, so every neighbour read of an SOR sweep lands in the array and
// reads exact zeros outside the domain.
struct Geo {
    int nx, ny, nz;
    int sx;             // natural row pitch (floats)
    long long sxy;      // natural plane pitch
    long long ntot;     // natural field length
    int H;              // colour row length
    int S;              // colour row pitch
    long long SP;       // colour plane pitch = S * (ny + 2)
    long long ctot;     // colour array length (incl. guard rows)
    float dx, dy, dz, dt;
    float idx, idy, idz, idt;
    float cx, cy, cz;   // 1/h^2
    int outflow;        // x+ is OUTFLOW (Dirichlet p on that face)
    int inflow;         // x- is INFLOW
    int u_last;         // last u-face index whose tendency is computed
    float s_xm, s_xp, s_ym, s_yp, s_zm, s_zp;  // tangential ghost signs
    // Stretched axes (the paper's 1-D spacing arrays, section 2.5.3):
    // stretched != 0 selects the kernels that read the per-axis metric
    // tables mx, my, mz (device memory, kMetricRows rows of n+2 floats per
    // axis, indexed by the 1-based cell or face index; see MetricRow).
    // Uniform grids keep stretched = 0 and the scalar spacings above.
    int stretched;
    const float* mx;
    const float* my;
    const float* mz;
    // The pressure operator in float64 for the residual, rebase and check
    // (the sweeps use the float32 weights): uniform 1/h^2, or per axis of a
    // stretched grid three rows of n + 2 doubles (M_WM, M_WP, M_DD order:
    // rows 0, 1, 2), so the iteration refines towards the float64
    // operator's solution however the float32 weights round.
    double cxd, cyd, czd;
    const double* wx;
    const double* wy;
    const double* wz;

    __host__ __device__ long long nat(int i, int j, int k) const {
        return (long long)k * sxy + (long long)j * sx + i;
    }
    // colour-array element of 0-based cell row (j0, k0), half-index ii
    __host__ __device__ long long col(int ii, int j0, int k0) const {
        return (long long)S + ((long long)(k0 + 1) * (ny + 2) + (j0 + 1)) * S + ii;
    }
};

// Rows of a per-axis metric table (float32, computed in float64 on the host
// and rounded once), each n+2 entries indexed by the 1-based cell index c
// (cells 1..n, ghosts 0 and n+1 mirror their neighbour's width) or by the
// face index f (face f between cells f and f+1):
//   M_IH   1 / h[c]                    (cell width h)
//   M_IG   1 / g[f], g[f] = (h[f] + h[f+1]) / 2   (centre distance across face f)
//   M_LO   h[f+1] / (h[f] + h[f+1])    weight of centre f in the linear
//   M_HI   h[f] / (h[f] + h[f+1])      interpolation onto face f (and of f+1)
//   M_WM   pressure-operator weight of the neighbour c-1 of cell c: 1/(h[c] g[c-1]),
//          0 across a boundary face
//   M_WP   weight of the neighbour c+1: 1/(h[c] g[c]), 0 across a boundary face
//   M_DD   the axis' share of the diagonal, M_WM + M_WP (+ 2/h[c]^2 at the
//          outflow face of the x axis, where p = 0 on the face)
//   M_H23  h[c]^(2/3) (the filter width (hx hy hz)^(1/3) squared is the product)
//   M_H    h[c]
enum MetricRow { M_IH = 0, M_IG, M_LO, M_HI, M_WM, M_WP, M_DD, M_H23, M_H, kMetricRows };

// Weight of the second inflow sample for the step that starts at time
// step * dt: the linear interpolation between samples at t0 and t1, held
// at the end values outside [t0, t1].  float64 without contraction, so the
// host (single handle) and the device (ensemble) give the same float.
__host__ __device__ inline float inflow_weight_at(long long step, double dt, double t0, double t1) {
#pragma clang fp contract(off)
    const double t = (double)step * dt;
    double w = (t - t0) / (t1 - t0);
    w = w < 0.0 ? 0.0 : (w > 1.0 ? 1.0 : w);
    return (float)w;
}

// Fold-and-rebase schedule of the pressure solve.  The correction pd is
// folded into the base ph (and r0 = rhs - A ph recomputed in float64)
// after every R-th check interval, and during the first kEarlyFoldIters
// iterations after every check interval that ends on a multiple of 8
// iterations: early in a solve the corrections are as large as p itself
// and float32 rounding relative to them would build up in the slowly
// converging modes, so folding often there keeps the iterate within about
// 1e-6 of the float64 one (128-iteration folds alone leave about 2e-5).
// cidx is the 1-based number of the interval, which ends at iteration
// cidx * K.
constexpr int kEarlyFoldIters = 512;
__host__ __device__ inline bool rebase_due_at(long long cidx, int K, int R) {
    if (cidx % R == 0) return true;
    const int e = K >= 8 ? 1 : 8 / K;
    return cidx * (long long)K <= kEarlyFoldIters && cidx % e == 0;
}

// Control block of one pressure solve (device memory).
struct Ctl {
    int done;           // 0 running, 1 converged, 2 hit max_iter, 3 non-finite
    int m;              // SOR iterations completed
    int K;              // check interval
    int max_iter;
    int skip;           // 1: the coming residual check is provably unsuccessful
    unsigned pad_u[3];
    double tol;
    double rhs2;        // sum rhs^2 (after mean removal)
    double rhs_sum;     // sum rhs (singular case)
    double resid;       // relative residual at the last check
    double reltmp2;     // sum reltmp^2 over the last iteration before the last check
    double div2;        // diagnostics: sum div(u)^2
    double cfl;         // diagnostics: max CFL
    double pad[4];
};

// Bits of the per-cell flag byte.
enum : uint8_t { F_USOLID = 1, F_VSOLID = 2, F_WSOLID = 4, F_CSOLID = 8 };

struct PBufs {           // one pressure system in colour layout
    float* ph[2];        // base pressure
    float* pd[2];        // correction
    float* r0[2];        // residual of the base, float32
    float* rhs[2];
    float* pa[2];        // second correction buffer of the fused sweeps (zero padding)
};

struct DevFields {
    float* u[2];
    float* v[2];
    float* w[2];
    float* nut;
    float* fu; float* fv; float* fw;     // AB2 history F^{n-1}
    float* su; float* sv; float* sw;     // feedback integral
    uint8_t* flags;
    float* prof;                         // inflow profile [nz] (first sample of a pair)
    float* prof1;                        // second sample of an interpolated pair [nz]
    float* stage;                        // natural-order staging (I/O)
    PBufs P;                             // time-stepping pressure system
    double* part[3];                     // reduction partials
    Ctl* ctl;
};

struct SolveParams {
    float omega;
    int K;
    int max_iter;
    double tol;
    int rebase_every;
};

}  // namespace les

namespace les {
// Captured runs of kSolveGraphChecks check intervals of one pressure
// system (exec[0]: check intervals only; exec[1]: the last one a rebase;
// exec[2]: the early-fold phase, a rebase every few intervals).
constexpr int kSolveGraphChecks = 8;
struct SolveGraph {
    const float* pd = nullptr;
    const float* ph = nullptr;
    const float* rhs = nullptr;
    int variant = -1, K = 0, R = 0;
    double omega = 0.0;
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
    uint64_t used = 0;
};
}  // namespace les

struct les_handle {
    int device = 0;
    les::Geo g{};
    les_params prm{};
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    std::string err;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    les::DevFields f{};
    // lazily allocated workspace of les_pressure_solve
    void* solve_arena = nullptr;
    les::PBufs S{};
    les::Ctl* ctl_save = nullptr;   // in solve_arena: the step's control block during warm-start trials
    int cur = 0;               // index of u^n in f.u/v/w
    int sor_variant = 0;       // SOR sweep tile variant (les_autotune)
    bool have_inflow = false;
    bool have_old = false;
    int64_t step = 0;
    float amp = 0.f;
    uint64_t seed = 0;
    std::vector<float> prof, prof1;
    bool interp = false;                 // inflow interpolated between prof and prof1
    double t0 = 0.0, t1 = 1.0;           // times of the two samples
    double dt = 0.0;                     // time step as given (the grid keeps it in float)
    std::vector<uint8_t> mask;
    std::vector<double> widths[3];       // cell widths per axis of a stretched grid (else empty)
    // kernel timing (les_params.timing): event pool and pending brackets
    std::vector<hipEvent_t> tev;
    size_t tev_used = 0;
    struct Bracket { int kind; size_t a, b; long long tag; int count; };
    std::vector<Bracket> tpending;
    double tms[LES_NUM_KERNELS] = {};
    int64_t tcount[LES_NUM_KERNELS] = {};
    les::Ctl* h_ctl = nullptr;   // pinned mirror of the control block
    int* h_flag = nullptr;       // pinned, 2 slots for pipelined flag reads
    hipEvent_t ev[2] = {nullptr, nullptr};
    les::SolveGraph sgraph[3];   // run_solve's graph cache (timing off)
    uint64_t sgraph_tick = 0;
    // twinned double-buffer comparison solver (twinned.hip): pairs, partials
    void* tw_q = nullptr;
    double* tw_part = nullptr;
    // learned warm start and training-pair capture (warm.hip)
    lesnet* warm_net = nullptr;
    double warm_scale = 1.0;
    int warm_rule = 0;           // LES_WARM_* (lesnet.h)
    int warm_param = 0;          // trial iterations / smoothing passes of the rule
    int warm_smooth = 0;         // smoothing passes on the network's output
    int cap_smooth = 0;          // smoothing passes on captured targets
    float* cap_x = nullptr;
    float* cap_t = nullptr;
    void* warm_arena = nullptr;
    struct WarmView* warm = nullptr;
};

namespace les {

// Finalize operations of the single-block reduction kernel.
enum FinOp { FIN_RHS2 = 0, FIN_RHS_SUM, FIN_PSUM, FIN_SETUP, FIN_CHECK, FIN_CHECK_FULL, FIN_DIAG,
             FIN_BOUND };

// ---- kernel launchers (kernels_*.hip) ----
hipError_t launch_finalize(hipStream_t st, int op, const double* part, int n, const double* rel0,
                           const double* rel1, int nrel, Ctl* ctl, double omega = 1.0);
// stretched grids: nu_t (cs2 = Cs^2; each cell's filter width from the
// tables), then the tendency, feedback forcing and AB2 reading it
hipError_t launch_nut_str(const Geo& g, hipStream_t st, const float* u, const float* v,
                          const float* w, float* nut, float cs2);
hipError_t launch_tendency_str(const Geo& g, hipStream_t st, const float* u, const float* v,
                               const float* w, const float* nut, float* fu, float* fv, float* fw,
                               float* su, float* sv, float* sw, const uint8_t* flags, float* us,
                               float* vs, float* ws, float nu, float alpha, float beta, int first);
// nu_t, tendency, feedback forcing and AB2 fused in one LDS-tiled pass
// (uniform grids); nu_t of every cell is stored as a diagnostic.
hipError_t launch_step_tile(const Geo& g, hipStream_t st, const float* u, const float* v,
                            const float* w, float* nut, float* fu, float* fv, float* fw, float* su,
                            float* sv, float* sw, const uint8_t* flags, float* us, float* vs,
                            float* ws, float c2, float nu, float alpha, float beta, int first);
hipError_t launch_inflow(const Geo& g, hipStream_t st, float* us, const float* prof,
                         const float* prof1, float wt,
                         const uint8_t* flags, float amp, uint64_t seed, int64_t step);
hipError_t launch_ctl_init(hipStream_t st, Ctl* ctl, double tol, int max_iter, int K);
hipError_t launch_rhs(const Geo& g, hipStream_t st, const float* us, const float* vs,
                      const float* ws, float* const rhs[2], double* part, Ctl* ctl,
                      int singular);
hipError_t launch_remove_mean_rhs(const Geo& g, hipStream_t st, float* const rhs[2],
                                  double* part, Ctl* ctl);
hipError_t launch_fold(const Geo& g, hipStream_t st, const PBufs& P, const Ctl* ctl);
hipError_t launch_colour_norm(const Geo& g, hipStream_t st, float* const a[2], double* part,
                              Ctl* ctl, int mode);
hipError_t launch_rebase(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                         const double* rel0, const double* rel1, int nrel, Ctl* ctl, int decide);
hipError_t launch_check(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                        const double* rel0, const double* rel1, int nrel, Ctl* ctl);
// Sweep variants: half-sweeps (nw = 0; row width tx, planes per block kt)
// and fused red-black iterations (nw wavefronts per block; needs an even
// check interval, the iterate alternating between pd and pa; kt = 0: the
// planes per block are chosen per grid, fused_kt).
struct SorVariant { int tx, kt, nw; };
constexpr int kNumSplitVariants = 8;
constexpr int kNumSorVariants = 14;
constexpr int kFirstRb2Variant = 12;   // variants 12, 13: two iterations per launch
// tile of a two-iteration launch: 64 lanes x 32 rows computed, the centre
// 58 half-cells x 26 rows written (three cells of ring per side)
constexpr int kRb2Rows = 32, kRb2RowsPerThread = 2, kRb2TXO = 58, kRb2TYO = 26;

// Planes per block of a fused variant on grid g: kt itself, or for kt = 0
// the fewest that keep the whole grid resident at once, about two
// 16-wavefront blocks per compute unit (every block then marches the same
// short column; a grid already wider than that takes 16).
__host__ __device__ inline int fused_kt(const Geo& g, int tx, int nw, int kt) {
    if (kt > 0) return kt;
    const int txo = tx - 2, tyo = (64 / tx) * nw - 2;
    const long long nxy = (long long)((g.H + txo - 1) / txo) * ((g.ny + tyo - 1) / tyo);
    constexpr long long kSlots = 2 * 256;   // two blocks on each of the 256 compute units
    if (nxy >= kSlots) return 16;
    const long long nbk = kSlots / nxy;
    const int k = (int)((g.nz + nbk - 1) / nbk);
    return k < 4 ? 4 : k;
}
extern const SorVariant kSorVariants[kNumSorVariants];
inline bool sor_fused(int variant) { return variant >= kNumSplitVariants; }
// two fused iterations per launch (needs a check interval that is a
// multiple of 4, so that an interval ends on the buffer it started from)
inline bool sor_fused2(int variant) { return variant >= kFirstRb2Variant; }
// The fused iteration's uniform-grid form addresses each colour array through
// a buffer resource whose base sits 2 SP elements before the array, so the
// array and that lead must span at most 4 GiB; larger grids take the
// general form.
__host__ __device__ inline bool rb_lean_fits(const Geo& g) {
    return (unsigned long long)(g.ctot + 2 * g.SP) * 4ull <= 0xFFFFFFFFull;
}

// Planes per block of a two-iteration launch: the block marches kt + 6
// planes, and with `slots` blocks resident at once (256 per_cu for a grid
// alone on the chip, per_cu resident blocks per compute unit) the launch
// takes about ceil(blocks / slots) such marches; the kt that minimises that
// product.
inline int rb2_kt_slots(const Geo& g, long long slots) {
    const long long nxy = (long long)((g.H + kRb2TXO - 1) / kRb2TXO) * ((g.ny + kRb2TYO - 1) / kRb2TYO);
    int best = 4;
    long long best_cost = -1;
    for (int kt = 4; kt <= 96; ++kt) {
        const long long nb = nxy * ((g.nz + kt - 1) / kt);
        const long long cost = ((nb + slots - 1) / slots) * ((kt < g.nz ? kt : g.nz) + 6);
        if (best_cost < 0 || cost < best_cost) {
            best = kt;
            best_cost = cost;
        }
    }
    return best;
}
inline int rb2_kt(const Geo& g, int per_cu) { return rb2_kt_slots(g, 256LL * per_cu); }
// blocks of a two-iteration launch with kt planes per block
inline unsigned rb2_blocks(const Geo& g, int kt) {
    return (unsigned)((g.H + kRb2TXO - 1) / kRb2TXO) * (unsigned)((g.ny + kRb2TYO - 1) / kRb2TYO) *
           (unsigned)((g.nz + kt - 1) / kt);
}
int sor_default_variant(const Geo& g);
// sweep blocks per launch: per half-sweep, or per iteration when fused
unsigned sor_sweep_blocks(const Geo& g, int variant);
hipError_t launch_sor(const Geo& g, hipStream_t st, const PBufs& P, int colour, float omega,
                      int local_iter, double* rel_part, const Ctl* ctl, int variant);
// one fused iteration: parity 0 reads pd and writes pa, parity 1 the reverse
hipError_t launch_sor_rb(const Geo& g, hipStream_t st, const PBufs& P, int parity, float omega,
                         int local_iter, double* rel0, double* rel1, const Ctl* ctl, int variant);
// two fused iterations (local iterations local_iter and local_iter + 1),
// buffers as launch_sor_rb
hipError_t launch_sor_rb2(const Geo& g, hipStream_t st, const PBufs& P, int parity, float omega,
                          int local_iter, double* rel0, double* rel1, const Ctl* ctl, int variant);
hipError_t launch_project(const Geo& g, hipStream_t st, float* us, float* vs, float* ws,
                          const PBufs& P);
hipError_t launch_bc(const Geo& g, hipStream_t st, float* u, float* v, float* w);
hipError_t launch_diag(const Geo& g, hipStream_t st, const float* u, const float* v,
                       const float* w, double* part, Ctl* ctl);
hipError_t launch_remove_mean_p(const Geo& g, hipStream_t st, const PBufs& P, double* part,
                                Ctl* ctl);
// learned warm start (warm.hip): warm_pre after the right-hand side is
// built (inputs, network, candidate start, and the choice under the
// residual rule), warm_take records a choice made on the host (trial and
// forced modes), warm_post after the solve (capture target); warm_result
// reads the choice of the last step.
// Stand-alone solve of a pressure system whose rhs and start are in S
// (les_api.hip); direct: every kernel launched itself, no graphs or timing
// events (nothing is created on the device).
int solve_system(les_handle* h, double tol, int32_t max_iter, les_solve_stats* st, const PBufs& S,
                 bool direct);
int warm_pre(les_handle* h);
PBufs warm_candidate(les_handle* h);   // the candidate pair (ph, pd only)
int warm_take(les_handle* h, int take, double r_prev, double r_net);
int warm_post(les_handle* h);
int warm_result(les_handle* h, int* taken, double* r_prev, double* r_net);
void warm_free(les_handle* h);
void twinned_free(les_handle* h);

// natural-order [nz][ny][nx] <-> colour layout
hipError_t launch_cells_to_colour(const Geo& g, hipStream_t st, const float* src, float* const dst[2]);
hipError_t launch_pair_to_cells(const Geo& g, hipStream_t st, const PBufs& P, float* dst);
hipError_t launch_colour_to_cells(const Geo& g, hipStream_t st, float* const src[2], float* dst);
hipError_t launch_fill(hipStream_t st, float* p, long long n, float v);

// boundary-range item -> (family, a, b); family -1 for padding
__host__ __device__ inline void bc_item(int nx, int ny, int nz, long long id, int& fam, int& a,
                                        int& b) {
    const long long jp = ny + 2, kp = nz + 2, ip = nx;
    const long long n0 = jp * kp, n1 = ip * kp, n2 = (long long)ip * ny;
    if (id < n0) {                       // x faces: (j, k) over the full ghosted plane
        fam = 0; b = (int)(id / jp); a = (int)(id % jp);
    } else if (id < n0 + n1) {           // y faces: (i, k), i interior, k ghosted
        long long t = id - n0;
        fam = 1; b = (int)(t / ip); a = 1 + (int)(t % ip);
    } else if (id < n0 + n1 + n2) {      // z faces: (i, j), both interior
        long long t = id - n0 - n1;
        fam = 2; b = 1 + (int)(t / ip); a = 1 + (int)(t % ip);
    } else {
        fam = -1; a = b = 0;
    }
}
__host__ __device__ inline long long bc_items(int nx, int ny, int nz) {
    return (long long)(ny + 2) * (nz + 2) + (long long)nx * (nz + 2) + (long long)nx * ny;
}

}  // namespace les
