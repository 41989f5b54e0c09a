/*
 * les.h -- C ABI of the MI355X urban-LES time step.
 *
 * One handle holds one building-resolving LES instance on one GPU: an
 * incompressible flow on a staggered (MAC) grid of nx * ny * nz cells.  A
 * time step follows the per-step subroutine list of the paper
 * (Vanderbauwhede 2014, section 2.1): Smagorinsky viscosity (les), body
 * force from advection and diffusion (velfg), building feedback forcing
 * (feedbf), Adams-Bashforth update (adam), inflow boundary (bondv1), the
 * pressure Poisson equation by red-black SOR (press, section 2.6), the
 * velocity update by the pressure gradient (velnw) and the ghost refresh
 * (bondv1, launched over the boundary range of section 2.4).
 *
 * Conventions shared by every call
 *   - Every function except les_destroy / les_last_error returns an int
 *     status: LES_OK (0), a warning (> 0) or an error (< 0).  No call
 *     aborts or prints.  Arguments are validated before any device work.
 *   - Host arrays are C order with i fastest and carry no ghosts:
 *       u [nz][ny][nx+1]  x-velocity on x-faces, face i = 0 is the x- boundary
 *       v [nz][ny+1][nx]  y-velocity on y-faces, faces 0 and ny are walls
 *       w [nz+1][ny][nx]  z-velocity on z-faces, faces 0 and nz are walls
 *       p, rhs, mask [nz][ny][nx]  cell centres
 *   - Host-pointer calls copy in/out and are synchronous on return.
 *     Device-pointer (_dev) calls borrow the pointers for the duration of
 *     the call, are ordered on the given stream and do not synchronise
 *     (NULL stream = the handle's stream).
 *   - All field arithmetic is float32; norms and residuals are accumulated
 *     in float64.
 *   - One handle per host thread.  Two handles may share a GPU.
 */
#ifndef LES_H_
#define LES_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ statuses */
enum {
    LES_OK = 0,
    LES_NOT_CONVERGED = 1,   /* warning: an SOR solve hit max_iter; fields valid */
    LES_EINVAL = -1,         /* bad argument (NULL, size, non-finite, bad BC set) */
    LES_ENOMEM = -2,         /* device or host allocation failed */
    LES_EDEVICE = -3,        /* a HIP runtime error; text in les_last_error */
    LES_ENONFINITE = -4,     /* a float64 norm came out NaN or Inf */
    LES_ESTATE = -5          /* call out of order (e.g. step before set_inflow) */
};

/* Boundary-condition kinds, one per domain face (les_params.bc). */
enum {
    LES_BC_FREESLIP = 0,     /* wall: zero normal velocity, mirrored tangential */
    LES_BC_NOSLIP = 1,       /* wall: zero normal velocity, anti-mirrored tangential */
    LES_BC_INFLOW = 2,       /* x- only: prescribed u profile plus noise */
    LES_BC_OUTFLOW = 3       /* x+ only: zero-gradient velocity, p = 0 on the face */
};
enum { LES_XM = 0, LES_XP = 1, LES_YM = 2, LES_YP = 3, LES_ZM = 4, LES_ZP = 5 };

typedef struct les_handle les_handle;

typedef struct {
    int32_t nx, ny, nz;      /* cells; each >= 4 */
} les_grid;

typedef struct {
    double dx, dy, dz;       /* uniform spacing [m]; > 0 and finite */
} les_spacing;

typedef struct {
    double omega;            /* SOR relaxation factor, 0 < omega < 2 (default 1.8) */
    double tol;              /* relative residual ||rhs - A p|| / ||rhs|| (1e-5) */
    int32_t check_every;     /* residual checked every K full iterations (4) */
    int32_t max_iter;        /* per solve (20000) */
    double cs;               /* Smagorinsky constant (0.1) */
    double nu;               /* molecular viscosity [m^2/s] (1.5e-5) */
    double alpha;            /* feedback forcing integral gain [1/s^2] (-10) */
    double beta;             /* feedback forcing proportional gain [1/s] (-1) */
    int32_t bc[6];           /* per face, LES_XM..LES_ZP (urban default:
                                INFLOW, OUTFLOW, FREESLIP, FREESLIP, NOSLIP, FREESLIP) */
    int32_t zero_guess;      /* 1: each solve starts from p = 0 (default 0: previous p) */
    int32_t rebase_every;    /* fold the correction into the base pressure every
                                R residual checks (32); see les_pressure_solve */
    int32_t diagnostics;     /* 1: compute ||div u^{n+1}|| and max CFL on the last
                                step of each les_step call (default 1) */
    int32_t timing;          /* 1: time kernels with HIP events on the handle's stream
                                (every launch of the per-step kernels and of the
                                rebase; for the SOR sweeps, one check interval in 8,
                                its 2K back-to-back half-sweeps, K fused iterations
                                or K/2 two-iteration launches between one event
                                pair, and that interval's residual check);
                                les_get_timing.  0 (default): the solver replays
                                check intervals from captured HIP graphs */
} les_params;

/* Per-call statistics of les_step.  Scalars describe the last step of the
 * call unless named _total. */
typedef struct {
    int32_t steps;           /* steps advanced */
    int32_t not_converged;   /* solves of this call that hit max_iter */
    int64_t sor_iters_total; /* SOR iterations summed over the steps */
    int32_t sor_iters_last;
    int32_t pad_;
    double resid_last;       /* final relative residual (float64) */
    double reltmp2_last;     /* sum of reltmp^2 over the last SOR iteration */
    double rhs_norm_last;    /* ||rhs||_2 */
    double div_star_last;    /* ||div u*||_2 = dt ||rhs|| (outflow case) */
    double div_new_last;     /* ||div u^{n+1}||_2 (diagnostics on), else -1 */
    double cfl_last;         /* max CFL of u^{n+1} (diagnostics on), else -1 */
    double ms_total;         /* host wall time of the call */
    int32_t* iters_out;      /* optional, caller-owned: n per-step iteration counts */
    /* learned warm start (lesnet.h, les_set_warm_start); -1 when off */
    int32_t warm_taken;      /* steps of the call whose solve started from the network */
    int32_t pad2_;
    double warm_r_prev_last; /* norm the rule compared for p_prev at the last step, over
                                ||rhs|| (residual; after the trial iterations; smoothed) */
    double warm_r_net_last;  /* the same for the network's start */
} les_step_stats;

typedef struct {
    int32_t iters;           /* SOR iterations performed */
    int32_t converged;       /* 1 if resid <= tol (or rhs == 0) */
    double resid;            /* final relative residual (float64) */
    double rhs_norm;         /* ||rhs||_2 after any mean removal */
    double reltmp2;          /* sum of reltmp^2 over the last iteration */
} les_solve_stats;

/* Fill *p with the defaults listed in les_params.  LES_EINVAL if p is NULL. */
int les_default_params(les_params* p);

/*
 * Create an instance.  building_mask (nullable = no buildings) is a uint8
 * cell mask [nz][ny][nx], 1 = solid, copied.  prm NULL = defaults.
 * Allocates every device field on the current HIP device, zeroes the state
 * and marks the Adams-Bashforth history as unset.  The caller owns *out
 * until les_destroy.  Requires nx, ny, nz >= 4, dx, dy, dz, dt > 0 and
 * finite, x- in {INFLOW, FREESLIP, NOSLIP}, x+ in {OUTFLOW, FREESLIP,
 * NOSLIP}, other faces walls.  Errors: LES_EINVAL, LES_ENOMEM, LES_EDEVICE.
 */
int les_create(const les_grid* g, const les_spacing* s, double dt, const uint8_t* building_mask,
               const les_params* prm, les_handle** out);

/*
 * Create on a stretched grid: every axis carries its own cell widths (the
 * paper's 1-D spacing arrays dx1 / dy1 / dzn of section 2.5.3, with the SOR
 * coefficients of section 2.6 built from them).  hx[nx], hy[ny], hz[nz]:
 * float64 cell widths [m], each > 0 and finite, copied.  Each stage then
 * differences over the distance between the two values it spans (a cell
 * width between a cell's faces, the distance of two centres across a
 * face), interpolates cell values onto a face of their own axis with the
 * width weights, and gives each cell its own filter width (hx hy hz)^(1/3);
 * the pressure operator A = D G keeps 12 bytes per cell per fused SOR
 * iteration (its per-axis weights are small tables, no 3-D coefficient
 * array).  Equal widths reproduce the uniform grid up to rounding.  The
 * profile of les_set_inflow is given at the stretched cell-centre heights.
 * Requires the x+ face to be OUTFLOW (a nonsingular operator), else
 * LES_EINVAL.  A stretched handle cannot join an ensemble, take a learned
 * warm start or training-pair capture, or run the twinned comparison
 * solver (each returns LES_EINVAL).  Other errors as les_create.
 */
int les_create_stretched(const les_grid* g, const double* hx, const double* hy, const double* hz,
                         double dt, const uint8_t* building_mask, const les_params* prm,
                         les_handle** out);

/* Free everything.  NULL is a no-op. */
void les_destroy(les_handle* h);

/* Text of the last error on this handle ("" if none).  Never NULL. */
const char* les_last_error(const les_handle* h);

/* Run the handle's work on this stream (a hipStream_t; NULL = the handle's
 * own stream, created at les_create).  The caller keeps it alive. */
int les_set_stream(les_handle* h, void* stream);

/*
 * Set the x- inflow profile: nz float32 speeds U(k) at the cell-centre
 * heights (k + 1/2) dz, and the relative noise amplitude a >= 0.  The
 * inflow face then carries U(k) (1 + a (2 xi - 1)) at every step, with xi a
 * counter-based uniform number from splitmix64(seed ^ (step 2^40 + k 2^20
 * + j)) (0-based j, k; top 24 bits).  On the first call it also sets the
 * initial state: u = U(k) on fluid u-faces, 0 on faces touching a solid
 * cell, v = w = p = 0 (section 2.1, bondv1: "initial wind profile").
 * Required before les_step (else LES_ESTATE).  Later calls only replace
 * the profile, amplitude and seed.
 */
int les_set_inflow(les_handle* h, const float* profile, float noise_amp, uint64_t seed);

/*
 * Inflow driven by a coarser model that delivers wind profiles at its own
 * interval (section 4, the coupled WRF/LES time loop: the LES receives a
 * profile every simulated minute, steps at half a second, and interpolates
 * between the two latest profiles, which it can do only once two exist).
 * prof0 (sample at model time t0) and prof1 (at t1 > t0) are nz float32
 * speeds as for les_set_inflow.  Every following step, started at time
 * t = n dt with n the steps done so far (les_get_step), uses
 *   U(k) = U0(k) + w (U1(k) - U0(k)),  w = (t - t0) / (t1 - t0) clamped to [0, 1]
 * (w rounded to float32, U formed on the device in float32), with the
 * noise, amplitude and seed of les_set_inflow.  A later pair replaces this
 * one; les_set_inflow switches the interpolation off.  The pair is part of
 * the checkpoint (les_get_state).  Requires les_set_inflow (or
 * les_set_fields) first, else LES_ESTATE; LES_EINVAL for NULL profiles,
 * non-finite values or t1 <= t0.  An ensemble step interpolates each
 * member's pair alike (bit for bit as the member stepped alone).
 * Synchronous.
 */
int les_set_inflow_pair(les_handle* h, double t0, const float* prof0, double t1,
                        const float* prof1);

/*
 * Advance n >= 0 steps.  Each step: nu_t, tendency with feedback forcing and
 * AB2 (u*), inflow, rhs = div(u*)/dt, red-black SOR to tol (checked every
 * check_every iterations, at most max_iter), projection u = u* - dt grad p,
 * ghost refresh.  st (nullable) receives the statistics.  Host-synchronous.
 * Returns LES_NOT_CONVERGED if any solve hit max_iter (fields still valid),
 * LES_ENONFINITE if a norm became NaN/Inf.
 */
int les_step(les_handle* h, int32_t n, les_step_stats* st);

/*
 * Stand-alone Poisson solve A p = rhs with the handle's operator (its
 * boundary conditions folded into the SOR coefficients, section 2.6).
 * rhs, p: host float32 [nz][ny][nx]; p is the initial guess on entry and
 * the solution on exit.  Without an outflow face the operator is singular:
 * the rhs mean is removed first and the p mean afterwards.  tol <= 0 or
 * max_iter < 0 is LES_EINVAL; max_iter = 0 returns the guess.  Does not
 * touch the time-stepping state.  LES_NOT_CONVERGED if max_iter was hit.
 *
 * The iterates are those of plain red-black SOR; internally p is held as a
 * float32 base plus a float32 correction that the sweeps update against a
 * float64-evaluated residual, so float32 storage does not stall the
 * iteration.
 */
int les_pressure_solve(les_handle* h, const float* rhs, float* p, double tol, int32_t max_iter,
                       les_solve_stats* st);

/* Same with device pointers (float32, [nz][ny][nx], contiguous). */
int les_pressure_solve_dev(les_handle* h, const float* d_rhs, float* d_p, double tol,
                           int32_t max_iter, les_solve_stats* st, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * stand-alone solve of les_pressure_solve_dev with the same arguments,
 * iterates and results, whose workspace is a static 64 MiB array of the
 * library's own device memory (one per device, held until the process
 * ends) instead of memory allocated on the handle's first solve.  It
 * allocates nothing and creates no graphs or events; every kernel is
 * launched on stream (NULL: the handle's own).  Grids whose ten colour
 * arrays exceed 64 MiB (about 3 million cells; the paper's 150x150x90
 * domain fits) are refused with LES_EINVAL.  Every call on a device shares
 * that device's array: calls that overlap on one device (two streams, two
 * threads, or a graph replayed while another call runs) race and give
 * undefined results.  The workspace is cleared at each call.  Statuses as
 * les_pressure_solve_dev.
 */
int les_pressure_solve_noalloc(les_handle* h, const float* d_rhs, float* d_p, double tol,
                               int32_t max_iter, les_solve_stats* st, void* stream);

/*
 * Twinned double-buffer relaxation (section 2.6: the paper's replacement
 * for the red-black scheme on the GPU), as a measured comparison solver;
 * the time step itself uses red-black SOR.  p is held as a pair (p_0, p_1)
 * of float32 per cell, interleaved; the first half of an iteration sets
 * every cell's p_1 from p_0, the second half p_0 from p_1, each by
 *   p_dst = p_src + omega (cn1 (sum_nb cn_nb p_src_nb - rhs) - p_src)
 * with the handle's operator.  All neighbours come from the previous half,
 * so this is a relaxed Jacobi iteration: its iterates differ from red-black
 * SOR's, and it is run for a fixed number of iterations (the paper's
 * default setup runs SOR for a fixed 50), not to a tolerance.
 * d_rhs, d_p: device float32 [nz][ny][nx]; d_p is the start on entry and
 * p_0 after `iters` iterations on exit.  No mean removal (for an operator
 * without outflow face, give a zero-mean rhs).  st (optional): iters,
 * resid = ||rhs - A p||_2 / ||rhs||_2 in float64, rhs_norm, converged =
 * (resid <= the handle's tol), reltmp2 = 0.  ms (optional): device time of
 * the sweeps alone (events on the stream).  Ordered on stream (NULL: the
 * handle's own), so it sees the caller's earlier writes to d_rhs and d_p on
 * that stream; returns after the stream has drained (synchronous).  Keeps a
 * workspace of (nx+2)(ny+2)(nz+2) pairs from the first call until
 * les_destroy.  LES_EINVAL for NULL pointers, iters < 0 or omega outside
 * (0, 1] (beyond 1 the iteration diverges on this operator);
 * LES_ENONFINITE if the residual is not finite.
 */
int les_pressure_solve_twinned(les_handle* h, const float* d_rhs, float* d_p, double omega,
                               int32_t iters, les_solve_stats* st, double* ms, void* stream);

/* Copy the state out (ghost-free layouts above).  NULL skips a field. */
int les_get_fields(les_handle* h, float* u, float* v, float* w, float* p);

/* Same into device buffers, ordered on stream. */
int les_get_fields_dev(les_handle* h, float* d_u, float* d_v, float* d_w, float* d_p,
                       void* stream);

/*
 * Overwrite the state from host arrays (NULL keeps a field).  Wall-normal
 * faces are forced to zero, ghosts refreshed.  reset_history = 1 makes the
 * next step a forward-Euler start.  Marks the inflow as set.
 */
int les_set_fields(les_handle* h, const float* u, const float* v, const float* w, const float* p,
                   int32_t reset_history);

/*
 * Start of the next pressure solve from a device array d_p [nz][ny][nx]
 * (e.g. a caller's own predictor): the pressure becomes d_p (its
 * correction part zero).  Borrowed for the call; ordered on stream (NULL:
 * the handle's), no synchronisation; work on another stream must be
 * ordered by the caller (or use les_set_stream).  The next les_step builds
 * its right-hand side and starts SOR from this pressure.
 */
int les_set_initial_guess_dev(les_handle* h, const float* d_p, void* stream);

/*
 * Intermediates of the most recent step, for inspection:
 *   which 0: nu_t at cell centres [nz][ny][nx]            -> a
 *   which 1: Poisson rhs = div(u*)/dt [nz][ny][nx]        -> a
 *   which 2: tendency F^n on u, v, w faces                -> a, b, c
 *   which 3: feedback integral usum on u, v, w faces      -> a, b, c
 * NULL pointers skip.  LES_EINVAL for an unknown which.
 */
int les_get_aux(les_handle* h, int32_t which, float* a, float* b, float* c);

/* Full ghosted velocity boxes, float32 [nz+2][ny+2][nx+2] each (index 0 and
 * n+1 are ghosts / boundary faces), for boundary-condition checks. */
int les_get_ghosted(les_handle* h, float* u, float* v, float* w);

/* Kernel timing collected while les_params.timing = 1: for each kernel
 * family, the summed event-bracketed device time and the number of timed
 * launches.  Families: 0 nu_t, 1 tendency, 2 inflow, 3 rhs, 4 SOR sweep
 * launch (a half-sweep, a whole iteration with the fused variants 8-11,
 * two with 12-13), 5 residual check (sampled like the sweeps: the launches
 * count is that of the sampled intervals), 6 rebase, 7 projection, 8
 * boundary refresh.  reset = 1 clears the counters after reading. */
#define LES_NUM_KERNELS 9
typedef struct {
    double ms[LES_NUM_KERNELS];
    int64_t launches[LES_NUM_KERNELS];
} les_timing;
int les_get_timing(les_handle* h, les_timing* out, int32_t reset);

/*
 * SOR sweep variants.  0-7: one launch per colour half-sweep (section 2.6),
 * tiles of 64 or 32 half-cells per wavefront row x 1, 2, 4 or 8 planes per
 * block (index 2 log2(planes) + (row width == 32)).  8-11: one launch per
 * red-black iteration that updates colour 0 and then colour 1 in one pass
 * over tiles of 30 x 30 (8, 10) or 62 x 14 (9, 11) half-cells x rows, 12
 * (8) or 16 (9) planes, or for 10 and 11 as many planes as keep the whole
 * grid resident at about two blocks per compute unit (16 where the grid is
 * wider), recomputing colour 0 on a one-cell ring around the tile: 12
 * instead of 16 bytes per cell per iteration; the iterate alternates
 * between two buffers, so these need an even check_every.  12-13: two
 * whole iterations per launch (temporal blocking): the four colour updates
 * run one plane behind another in one k-march over tiles of 64 half-cells
 * x 32 rows, of which the 58 x 26 centre is written (the ring shrinks by
 * one cell per update), so 12 bytes per cell move for two iterations; the
 * planes per block are chosen per grid for one (12) or two (13) resident
 * blocks per compute unit; they need check_every to be a multiple of 4 and
 * are not used by ensembles.  Every variant computes the same per-cell
 * arithmetic, so results are bitwise independent of the choice.
 *
 * Autotuner: times every variant for reps back-to-back pairs of launches
 * on this handle's grid, keeps the fastest for all later solves of the
 * handle and reports its index in *chosen (nullable) and the per-variant
 * microseconds per half-sweep (for 8-11: half a fused iteration; for
 * 12-13 a quarter of a launch; 0 when not timed because check_every does
 * not allow the variant) in
 * us_per_sweep[LES_NUM_SOR_VARIANTS] (nullable).  Runs on a scratch
 * pressure system: the time-stepping state is unchanged.  LES_EINVAL
 * unless 1 <= reps <= 1000.
 */
#define LES_NUM_SOR_VARIANTS 14
int les_autotune(les_handle* h, int32_t reps, int32_t* chosen, double* us_per_sweep);

/* Select a sweep variant by index (0 .. LES_NUM_SOR_VARIANTS-1); LES_EINVAL
 * for 8-11 with an odd check_every, and for 12-13 (two iterations per
 * launch) when check_every is not a multiple of 4. */
int les_set_sor_variant(les_handle* h, int32_t variant);

/* Step counter (completed steps). */
int les_get_step(const les_handle* h, int64_t* step);

/*
 * Checkpoint.  les_state_size gives the byte size of the opaque blob;
 * les_get_state fills it (u, v, w, p as base + correction, AB2 history,
 * feedback integral, step counter, flags, inflow settings); les_set_state
 * restores it into a handle of the same grid and BC set, so that the runs
 * continue bitwise identically.  LES_EINVAL on a size or grid mismatch.
 */
int les_state_size(const les_handle* h, int64_t* bytes);
int les_get_state(les_handle* h, void* buf, int64_t bytes);
int les_set_state(les_handle* h, const void* buf, int64_t bytes);

/*
 * Ensemble (batched, uneven grids).  An ensemble borrows 1..64 existing
 * handles on one device (not owned: destroy the ensemble before them) with
 * the same check_every and zero_guess = 0; each keeps its own grid,
 * buildings, inflow and parameters.  les_ensemble_step advances every
 * member by nsteps: per step each stage is one launch over an
 * (instance, block) work list, the stage sequences before and after the
 * pressure solve are replayed from HIP graphs, and the pressure solves of
 * all members run together with per-member stopping tests on the device
 * (see les_ensemble_set_mode: batched launches or one persistent
 * cooperative launch).  Results are bitwise identical to stepping
 * each member alone with les_step.  Members' step counters and buffers
 * are updated, so single steps and ensemble steps can be mixed.
 * iters_out (nullable, caller-owned) receives nsteps x n iteration counts
 * (step-major).  Host-synchronous.  Returns LES_NOT_CONVERGED if any solve
 * hit max_iter, LES_ESTATE if a member has no inflow yet or has a learned
 * warm start or a capture set (lesnet.h; those run with les_step only).
 */
typedef struct les_ensemble les_ensemble;
typedef struct {
    int32_t members;
    int32_t steps;
    int64_t cells_total;      /* sum of the members' cells */
    int64_t sor_iters_total;  /* over members and steps */
    int32_t not_converged;    /* member-steps that hit max_iter */
    int32_t pad_;
    double ms_total;          /* host wall time of the call */
} les_ensemble_stats;
int les_ensemble_create(int32_t n, les_handle* const* members, les_ensemble** out);
int les_ensemble_step(les_ensemble* e, int32_t nsteps, les_ensemble_stats* st, int32_t* iters_out);
/* Autotuner for the ensemble: times the batched sweeps over all members
 * for each sweep variant (all members on one variant: with the members'
 * working sets together the cache behaviour differs from each one alone)
 * on the members' scratch pressure systems (the state is not touched),
 * reps pairs of launches each, and uses the fastest from the next step on.
 * les_ensemble_tuning reports the choice and the microseconds per
 * half-sweep of every variant (us_per_sweep[LES_NUM_SOR_VARIANTS]; for
 * 8-11 half a fused iteration, for 12-13 a quarter of a two-iteration
 * launch, 0 where not timed).  The fused variants run only in the batched
 * mode and only as the ensemble's choice (les_ensemble_autotune or
 * les_ensemble_set_variant): 8-11 with an even check_every, 12-13 with a
 * check_every that is a multiple of 4 and every member a uniform grid whose
 * colour arrays span less than 2 GiB; otherwise a member set to one runs
 * its grid's default half-sweep. */
int les_ensemble_autotune(les_ensemble* e, int32_t reps);
/* The sweep variant every member runs (0 .. LES_NUM_SOR_VARIANTS-1), or
 * -1: each member its own; from the next step on.  LES_EINVAL otherwise. */
int les_ensemble_set_variant(les_ensemble* e, int32_t variant);
int les_ensemble_tuning(const les_ensemble* e, int32_t* variant, double* us_per_sweep);
const char* les_ensemble_last_error(const les_ensemble* e);
void les_ensemble_destroy(les_ensemble* e);

/* How the members' pressure solves run (same arithmetic, same results):
 * LES_ENSEMBLE_BATCHED (default): one launch per half-sweep, fused iteration
 * or two fused iterations (and per check phase) over all members' work,
 * check intervals replayed from a HIP graph in batches of 8, per-member stop
 * flags on the device; once members have stopped (seen one batch behind)
 * the sweep launches cover only the members still iterating.
 * LES_ENSEMBLE_PERSISTENT: the whole solve of all members in one
 * cooperative launch with grid barriers between phases. */
enum { LES_ENSEMBLE_BATCHED = 0, LES_ENSEMBLE_PERSISTENT = 1 };
int les_ensemble_set_mode(les_ensemble* e, int32_t mode);

/*
 * Boundary-range mapping of the ghost-refresh launch (section 2.4),
 * exposed for host-side tests; no device work.  les_bc_range gives the
 * launch size for grid g: (ny+2)(nz+2) x-face items + nx(nz+2) y-face items
 * + nx ny z-face items, padded up to whole 256-thread blocks (0 if g is
 * NULL or not >= 1 per axis).  les_bc_map maps an item id to its family
 * (0 = x faces over ghosted (j, k); 1 = y faces over (i, k), i interior;
 * 2 = z faces over interior (i, j)) and the two in-plane ghosted indices
 * (a, b); ids in the padding return family -1 (the guarded tail).
 * LES_EINVAL on NULL pointers or a negative item.
 */
int64_t les_bc_range(const les_grid* g);
int les_bc_map(const les_grid* g, int64_t item, int32_t* family, int32_t* a, int32_t* b);

#ifdef __cplusplus
}
#endif

#endif /* LES_H_ */
