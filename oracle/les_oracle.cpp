// =====================================================================
//  FP64 CPU oracle of one urban-LES time step  --  TEST INFRASTRUCTURE
// =====================================================================
//
//  This file is the checker, not the product.  Only the test-suite, the
//  package smoke test and the CPU-baseline leg of the benchmark may load
//  it.  It shares no source, header, table or helper with the GPU library.
//
//  What it computes follows the paper (Vanderbauwhede 2014, "Model
//  coupling between WRF and the DPRI LES ..."), section 2:
//    * per-step subroutine list (section 2.1): velocity update (velnw),
//      boundary conditions (bondv1), body force (velfg), building effects
//      (feedbf), Smagorinsky viscosity (les), Adams-Bashforth (adam),
//      pressure Poisson by SOR (press);
//    * assembly of the x-momentum tendency from advective (cov) and
//      diffusive (diu) pieces (section 2.5.3, "pre-computing neighbouring
//      points");
//    * the red-black SOR update and its colour order (section 2.6);
//    * boundary work split into the three face families (section 2.4);
//    * per-axis 1-D cell widths (the dx1 / dy1 / dzn arrays of section
//      2.5.3), so every axis may be stretched; a uniform grid is the case
//      of equal widths.
//  Where the paper is silent (staggering, advection formula, SGS model
//  details, feedback law, BC formulas, residual definition) the oracle
//  follows the readings listed in the design notes of this repository;
//  each function below names the reading it implements.
//
//  Everything is float64, plain loops, one function per step.  OpenMP is
//  used only across k inside one colour or one stencil pass, where every
//  cell is independent, so results do not depend on the thread count.
//  Reductions sum per-plane partials serially in k order.
//
//  Index convention (1-based with one ghost layer, as in the Fortran):
//    cells       i = 1..nx, j = 1..ny, k = 1..nz  (ghosts 0 and n+1)
//    u(i,j,k)    east face of cell i   (i = 0: x- boundary face,
//                                        i = nx: x+ boundary face)
//    v(i,j,k)    north face of cell j  (j = 0, ny: y walls)
//    w(i,j,k)    top face of cell k    (k = 0: ground, k = nz: top)
//    p(i,j,k)    cell centre
// =====================================================================
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

enum BcKind { BC_FREESLIP = 0, BC_NOSLIP = 1, BC_INFLOW = 2, BC_OUTFLOW = 3 };
enum Face { XM = 0, XP = 1, YM = 2, YP = 3, ZM = 4, ZP = 5 };

// Mirrors the ctypes structure declared in oracle/__init__.py.
struct OParams {
    double omega;       // SOR relaxation factor
    double tol;         // relative residual target
    int32_t check_every;  // residual checked every K full iterations
    int32_t max_iter;
    double cs;          // Smagorinsky constant
    double nu;          // molecular viscosity [m^2/s]
    double alpha;       // feedback forcing, integral gain [1/s^2]
    double beta;        // feedback forcing, proportional gain [1/s]
    int32_t bc[6];      // x-, x+, y-, y+, z-, z+
    int32_t zero_guess; // 1: SOR starts from p = 0 instead of the previous p
    int32_t pad_;
};

struct OStats {
    int32_t iters;          // SOR iterations of the last solve
    int32_t converged;      // 1 if the last solve reached tol (or rhs == 0)
    double resid;           // final relative residual of the last solve
    double rhs_norm;        // ||rhs||_2 of the last solve
    double reltmp2;         // sum of reltmp^2 over the last SOR iteration
    double div_star;        // ||div u*||_2 before the projection
    double div_new;         // ||div u^{n+1}||_2 after the projection
    double cfl;             // max CFL number of u^{n+1}
    int64_t total_iters;    // summed over the steps of one call
    int32_t not_converged;  // number of solves that hit max_iter
    int32_t pad_;
};

// A field on the ghosted (nx+2) x (ny+2) x (nz+2) box.
struct Box {
    int nx = 0, ny = 0, nz = 0;
    std::vector<double> a;
    void init(int x, int y, int z) {
        nx = x; ny = y; nz = z;
        a.assign((size_t)(nx + 2) * (ny + 2) * (nz + 2), 0.0);
    }
    double& operator()(int i, int j, int k) {
        return a[((size_t)k * (ny + 2) + j) * (nx + 2) + i];
    }
    double operator()(int i, int j, int k) const {
        return a[((size_t)k * (ny + 2) + j) * (nx + 2) + i];
    }
};

// splitmix64 (Steele, Lea & Flood, OOPSLA 2014): one output of the
// generator whose state is x, i.e. advance by the golden gamma, then mix.
uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

struct Oracle {
    int nx, ny, nz;
    double dt;
    OParams prm;
    std::vector<uint8_t> solid;  // cell mask, [k][j][i] 0-based interior
    Box u, v, w, p;              // state u^n (ghosts valid), p^n
    Box us, vs, ws;              // u*, then u^{n+1}
    Box nut;                     // eddy viscosity at centres (+ghost ring)
    Box fu, fv, fw;              // tendency F^n
    Box gu, gv, gw;              // F^{n-1} (AB2 history)
    Box su, sv, sw;              // feedback-forcing time integral
    Box rhs;                     // Poisson right-hand side
    // Grid metrics of one axis (the paper's 1-D spacing arrays, section
    // 2.5.3), indexed 0..n+1; a ghost cell has the width of the interior
    // cell it mirrors.
    //   h[c]   width of cell c
    //   g[f]   distance between the centres of cells f and f+1, i.e. the
    //          width of the control volume of a value on face f (f = 0..n)
    //   lo[f], hi[f]  weights of centres f and f+1 in the linear
    //          interpolation onto face f: lo = h[f+1] / (h[f] + h[f+1]),
    //          hi = h[f] / (h[f] + h[f+1])
    // A uniform axis has g = h and lo = hi = 1/2 exactly.
    struct Axis {
        std::vector<double> h, g, lo, hi;
        void init(const double* widths, int n) {
            h.assign(n + 2, 0.0); g.assign(n + 2, 0.0);
            lo.assign(n + 2, 0.0); hi.assign(n + 2, 0.0);
            for (int c = 1; c <= n; ++c) h[c] = widths[c - 1];
            h[0] = h[1];
            h[n + 1] = h[n];
            for (int f = 0; f <= n; ++f) {
                g[f] = 0.5 * (h[f] + h[f + 1]);
                lo[f] = h[f + 1] / (h[f] + h[f + 1]);
                hi[f] = h[f] / (h[f] + h[f + 1]);
            }
        }
    };
    Axis X, Y, Z;
    // Pressure operator A = D G (section 2.6): weight of the neighbour
    // across each face of a cell, and the diagonal's share per axis.
    std::vector<double> w_east, w_west, w_north, w_south, w_top, w_bottom;
    std::vector<double> d_x, d_y, d_z;
    std::vector<double> prof;        // inflow profile U(k), k = 1..nz
    // Time-interpolated inflow (section 4, coupled time loop): samples U0 =
    // prof at time t0 and U1 = prof1 at time t1, interpolated linearly.
    std::vector<double> prof1;
    bool interp = false;
    double t0 = 0.0, t1 = 1.0;
    double amp = 0.0;
    uint64_t seed = 0;
    bool have_inflow = false;
    bool have_old = false;
    int64_t step = 0;
    OStats st{};

    // short names for the metrics
    double hx(int c) const { return X.h[c]; }
    double hy(int c) const { return Y.h[c]; }
    double hz(int c) const { return Z.h[c]; }
    double gx(int f) const { return X.g[f]; }
    double gy(int f) const { return Y.g[f]; }
    double gz(int f) const { return Z.g[f]; }

    // Only the x+ face can carry the Dirichlet (outflow) pressure condition;
    // without it the operator has the constants as null space.
    bool singular() const { return prm.bc[XP] != BC_OUTFLOW; }

    // ------------------------------------------------------------ mask
    bool cell_solid(int i, int j, int k) const {  // 1-based, clamped
        i = std::min(std::max(i, 1), nx);
        j = std::min(std::max(j, 1), ny);
        k = std::min(std::max(k, 1), nz);
        return solid[((size_t)(k - 1) * ny + (j - 1)) * nx + (i - 1)] != 0;
    }
    // A face is solid when either of the two cells it separates is solid
    // (feedback-forcing reading).  Boundary faces look at their one cell.
    bool u_solid(int i, int j, int k) const { return cell_solid(i, j, k) || cell_solid(i + 1, j, k); }
    bool v_solid(int i, int j, int k) const { return cell_solid(i, j, k) || cell_solid(i, j + 1, k); }
    bool w_solid(int i, int j, int k) const { return cell_solid(i, j, k) || cell_solid(i, j, k + 1); }

    // Sign of a tangential ghost value across a face: mirror for free slip
    // and zero-gradient outflow, anti-mirror for no slip and inflow.
    double tsign(int face) const {
        int b = prm.bc[face];
        return (b == BC_FREESLIP || b == BC_OUTFLOW) ? 1.0 : -1.0;
    }

    // --------------------------------------------------- set-up helpers
    // Poisson operator A = D G on the MAC grid, from the divergence D (face
    // differences over the cell width) and the gradient G (centre
    // differences over the centre distance):
    //   (A p)_c = [(p_{c+1} - p_c) / g_c - (p_c - p_{c-1}) / g_{c-1}] / h_c
    // per axis.  Across a boundary face with a prescribed normal velocity
    // (walls, inflow) the pressure gradient is not used: no neighbour
    // weight, no diagonal share (Neumann).  Across the outflow face p = 0
    // on the face, half a cell away from the centre: gradient -2 p / h,
    // which adds 2 / h^2 to the diagonal.
    void build_coefficients() {
        w_east.assign(nx + 2, 0.0); w_west.assign(nx + 2, 0.0); d_x.assign(nx + 2, 0.0);
        w_north.assign(ny + 2, 0.0); w_south.assign(ny + 2, 0.0); d_y.assign(ny + 2, 0.0);
        w_top.assign(nz + 2, 0.0); w_bottom.assign(nz + 2, 0.0); d_z.assign(nz + 2, 0.0);
        for (int i = 1; i <= nx; ++i) {
            w_west[i] = (i > 1) ? 1.0 / (hx(i) * gx(i - 1)) : 0.0;
            w_east[i] = (i < nx) ? 1.0 / (hx(i) * gx(i)) : 0.0;
            d_x[i] = w_west[i] + w_east[i];
            if (i == nx && prm.bc[XP] == BC_OUTFLOW) d_x[i] += 2.0 / (hx(i) * hx(i));
        }
        for (int j = 1; j <= ny; ++j) {
            w_south[j] = (j > 1) ? 1.0 / (hy(j) * gy(j - 1)) : 0.0;
            w_north[j] = (j < ny) ? 1.0 / (hy(j) * gy(j)) : 0.0;
            d_y[j] = w_south[j] + w_north[j];
        }
        for (int k = 1; k <= nz; ++k) {
            w_bottom[k] = (k > 1) ? 1.0 / (hz(k) * gz(k - 1)) : 0.0;
            w_top[k] = (k < nz) ? 1.0 / (hz(k) * gz(k)) : 0.0;
            d_z[k] = w_bottom[k] + w_top[k];
        }
    }
    double diagonal(int i, int j, int k) const { return d_x[i] + d_y[j] + d_z[k]; }
    // sum over the six neighbours of weight times neighbour value
    double neighbours(const Box& P, int i, int j, int k) const {
        return w_east[i] * P(i + 1, j, k) + w_west[i] * P(i - 1, j, k) +
               w_north[j] * P(i, j + 1, k) + w_south[j] * P(i, j - 1, k) +
               w_top[k] * P(i, j, k + 1) + w_bottom[k] * P(i, j, k - 1);
    }

    // ---------------------------------------------- boundary conditions
    // Ghost refresh (bondv1), done as three face-family passes -- x, then
    // y, then z -- each covering the full ghosted extent of the other two
    // axes, so edge and corner ghosts compose the per-face rules.
    // Owned boundary values (inflow face, wall-normal faces) are not
    // touched here.
    void refresh_ghosts(Box& U, Box& V, Box& W) const {
        const double sxm = tsign(XM), sxp = tsign(XP), sym = tsign(YM), syp = tsign(YP),
                     szm = tsign(ZM), szp = tsign(ZP);
        const bool out_xp = prm.bc[XP] == BC_OUTFLOW;
        for (int k = 0; k <= nz + 1; ++k)
            for (int j = 0; j <= ny + 1; ++j) {
                U(nx + 1, j, k) = out_xp ? U(nx, j, k) : 0.0;
                V(0, j, k) = sxm * V(1, j, k);
                V(nx + 1, j, k) = sxp * V(nx, j, k);
                W(0, j, k) = sxm * W(1, j, k);
                W(nx + 1, j, k) = sxp * W(nx, j, k);
            }
        for (int k = 0; k <= nz + 1; ++k)
            for (int i = 0; i <= nx + 1; ++i) {
                U(i, 0, k) = sym * U(i, 1, k);
                U(i, ny + 1, k) = syp * U(i, ny, k);
                W(i, 0, k) = sym * W(i, 1, k);
                W(i, ny + 1, k) = syp * W(i, ny, k);
                V(i, ny + 1, k) = 0.0;   // beyond the north wall: unused
            }
        for (int j = 0; j <= ny + 1; ++j)
            for (int i = 0; i <= nx + 1; ++i) {
                U(i, j, 0) = szm * U(i, j, 1);
                U(i, j, nz + 1) = szp * U(i, j, nz);
                V(i, j, 0) = szm * V(i, j, 1);
                V(i, j, nz + 1) = szp * V(i, j, nz);
                W(i, j, nz + 1) = 0.0;   // beyond the top wall: unused
            }
    }

    // Wall-normal faces carry zero velocity; walls on x also pin u there.
    void zero_wall_faces(Box& U, Box& V, Box& W) const {
        for (int k = 0; k <= nz + 1; ++k)
            for (int i = 0; i <= nx + 1; ++i) { V(i, 0, k) = 0.0; V(i, ny, k) = 0.0; }
        for (int j = 0; j <= ny + 1; ++j)
            for (int i = 0; i <= nx + 1; ++i) { W(i, j, 0) = 0.0; W(i, j, nz) = 0.0; }
        for (int k = 0; k <= nz + 1; ++k)
            for (int j = 0; j <= ny + 1; ++j) {
                if (prm.bc[XM] != BC_INFLOW) U(0, j, k) = 0.0;
                if (prm.bc[XP] != BC_OUTFLOW) U(nx, j, k) = 0.0;
            }
    }

    // Inflow value on the x- face at step index s (bondv1, inflow part):
    // U(k) (1 + a (2 xi - 1)), xi a counter-based uniform in [0,1) from
    // splitmix64 of seed ^ (s 2^40 + k0 2^20 + j0), 0-based j0, k0.
    double inflow_value(int j, int k, int64_t s) const {
        if (cell_solid(1, j, k)) return 0.0;
        uint64_t ctr = ((uint64_t)s << 40) + ((uint64_t)(k - 1) << 20) + (uint64_t)(j - 1);
        uint64_t r = splitmix64(seed ^ ctr);
        double xi = (double)(r >> 40) * (1.0 / 16777216.0);
        return profile_at(k, s) * (1.0 + amp * (2.0 * xi - 1.0));
    }

    // Profile used by step index s (the step that starts at time (s-1) dt).
    // With a pair of samples: the straight line through (t0, U0(k)) and
    // (t1, U1(k)) evaluated at that time, held at U0 before t0 and at U1
    // after t1 (reading: no extrapolation past the samples).
    double profile_at(int k, int64_t s) const {
        if (!interp) return prof[k];
        const double t = (double)(s - 1) * dt;
        if (t <= t0) return prof[k];
        if (t >= t1) return prof1[k];
        const double w = (t - t0) / (t1 - t0);
        return (1.0 - w) * prof[k] + w * prof1[k];
    }

    // ------------------------------------------------ Smagorinsky (les)
    // Edge-centred strain rates on the MAC grid: each velocity difference
    // across a face is divided by the distance between the two values.
    double e12(const Box& U, const Box& V, int a, int b, int k) const {
        return 0.5 * ((U(a, b + 1, k) - U(a, b, k)) / gy(b) + (V(a + 1, b, k) - V(a, b, k)) / gx(a));
    }
    double e13(const Box& U, const Box& W, int a, int j, int c) const {
        return 0.5 * ((U(a, j, c + 1) - U(a, j, c)) / gz(c) + (W(a + 1, j, c) - W(a, j, c)) / gx(a));
    }
    double e23(const Box& V, const Box& W, int i, int b, int c) const {
        return 0.5 * ((V(i, b, c + 1) - V(i, b, c)) / gz(c) + (W(i, b + 1, c) - W(i, b, c)) / gy(b));
    }

    // nu_t = (Cs Delta)^2 |S|, |S| = sqrt(2 S_ij S_ij), Delta = (hx hy hz)^(1/3)
    // of the cell.  Diagonal S_ii from the two faces of the cell; off-diagonal
    // S_ij as the mean of the four surrounding edge values (the cell centre is
    // the midpoint of those edges on any grid).  The ghost ring copies the
    // nearest interior cell.
    void compute_nut(const Box& U, const Box& V, const Box& W) {
#pragma omp parallel for schedule(static)
        for (int k = 1; k <= nz; ++k)
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) {
                    const double delta = std::cbrt(hx(i) * hy(j) * hz(k));
                    const double c2 = (prm.cs * delta) * (prm.cs * delta);
                    double s11 = (U(i, j, k) - U(i - 1, j, k)) / hx(i);
                    double s22 = (V(i, j, k) - V(i, j - 1, k)) / hy(j);
                    double s33 = (W(i, j, k) - W(i, j, k - 1)) / hz(k);
                    double s12 = 0.25 * (e12(U, V, i - 1, j - 1, k) + e12(U, V, i, j - 1, k) +
                                         e12(U, V, i - 1, j, k) + e12(U, V, i, j, k));
                    double s13 = 0.25 * (e13(U, W, i - 1, j, k - 1) + e13(U, W, i, j, k - 1) +
                                         e13(U, W, i - 1, j, k) + e13(U, W, i, j, k));
                    double s23 = 0.25 * (e23(V, W, i, j - 1, k - 1) + e23(V, W, i, j, k - 1) +
                                         e23(V, W, i, j - 1, k) + e23(V, W, i, j, k));
                    double ss = 2.0 * (s11 * s11 + s22 * s22 + s33 * s33) +
                                4.0 * (s12 * s12 + s13 * s13 + s23 * s23);
                    nut(i, j, k) = c2 * std::sqrt(ss);
                }
        for (int k = 0; k <= nz + 1; ++k)
            for (int j = 0; j <= ny + 1; ++j)
                for (int i = 0; i <= nx + 1; ++i) {
                    if (i >= 1 && i <= nx && j >= 1 && j <= ny && k >= 1 && k <= nz) continue;
                    nut(i, j, k) = nut(std::min(std::max(i, 1), nx), std::min(std::max(j, 1), ny),
                                       std::min(std::max(k, 1), nz));
                }
    }

    // Edge eddy viscosity: mean of the four cells sharing the edge.  (On a
    // stretched axis this is kept rather than a width-weighted
    // interpolation: the model's filter width Delta is itself a property of
    // each cell, so nu_t has no grid-independent value to interpolate.)
    double n12(int a, int b, int k) const {
        return 0.25 * (nut(a, b, k) + nut(a + 1, b, k) + nut(a, b + 1, k) + nut(a + 1, b + 1, k));
    }
    double n13(int a, int j, int c) const {
        return 0.25 * (nut(a, j, c) + nut(a + 1, j, c) + nut(a, j, c + 1) + nut(a + 1, j, c + 1));
    }
    double n23(int i, int b, int c) const {
        return 0.25 * (nut(i, b, c) + nut(i, b + 1, c) + nut(i, b, c + 1) + nut(i, b + 1, c + 1));
    }

    // ------------------------------------------------ body force (velfg)
    // F = -(covx + covy + covz) + nu lap(u) + div(2 nu_t S), assembled on
    // the control volume of each face value (section 2.5.3): for u on face
    // i that volume spans g_i in x and the cell widths h_j, h_k in y and z.
    // Second-order central advective form: a cov piece is the product of
    // the advecting velocity and a one-sided difference of the advected
    // component.  Along the component's own axis the pieces sit at the two
    // neighbouring centres and are interpolated linearly onto the face
    // (weights by the opposite cell widths, the paper's covx1); across it
    // they sit on the two edges, whose midpoint the face is, and are
    // averaged (covy1, covz1).  An advecting velocity is interpolated
    // linearly from its own faces onto the edge.  Diffusion is the
    // difference of the one-sided fluxes (diu) over the control volume.
    double force_u(const Box& U, const Box& V, const Box& W, int i, int j, int k) const {
        auto c1 = [&](int c) {  // at cell centre c
            return 0.5 * (U(c - 1, j, k) + U(c, j, k)) * (U(c, j, k) - U(c - 1, j, k)) / hx(c);
        };
        auto c2 = [&](int b) {  // at the x-y edge on y-face b (between rows b and b+1)
            const double vb = X.lo[i] * V(i, b, k) + X.hi[i] * V(i + 1, b, k);
            return vb * (U(i, b + 1, k) - U(i, b, k)) / gy(b);
        };
        auto c3 = [&](int c) {  // at the x-z edge on z-face c
            const double wc = X.lo[i] * W(i, j, c) + X.hi[i] * W(i + 1, j, c);
            return wc * (U(i, j, c + 1) - U(i, j, c)) / gz(c);
        };
        double covx = X.lo[i] * c1(i) + X.hi[i] * c1(i + 1);
        double covy = 0.5 * (c2(j - 1) + c2(j));
        double covz = 0.5 * (c3(k - 1) + c3(k));
        auto fx = [&](int c) { return (U(c, j, k) - U(c - 1, j, k)) / hx(c); };   // at centre c
        auto fy = [&](int b) { return (U(i, b + 1, k) - U(i, b, k)) / gy(b); };   // on y-face b
        auto fz = [&](int c) { return (U(i, j, c + 1) - U(i, j, c)) / gz(c); };   // on z-face c
        double lap = (fx(i + 1) - fx(i)) / gx(i) + (fy(j) - fy(j - 1)) / hy(j) +
                     (fz(k) - fz(k - 1)) / hz(k);
        double sgs = (2.0 * nut(i + 1, j, k) * fx(i + 1) - 2.0 * nut(i, j, k) * fx(i)) / gx(i) +
                     (2.0 * n12(i, j, k) * e12(U, V, i, j, k) -
                      2.0 * n12(i, j - 1, k) * e12(U, V, i, j - 1, k)) / hy(j) +
                     (2.0 * n13(i, j, k) * e13(U, W, i, j, k) -
                      2.0 * n13(i, j, k - 1) * e13(U, W, i, j, k - 1)) / hz(k);
        return -(covx + covy + covz) + prm.nu * lap + sgs;
    }

    double force_v(const Box& U, const Box& V, const Box& W, int i, int j, int k) const {
        auto c1 = [&](int a) {  // at the x-y edge on x-face a
            const double ua = Y.lo[j] * U(a, j, k) + Y.hi[j] * U(a, j + 1, k);
            return ua * (V(a + 1, j, k) - V(a, j, k)) / gx(a);
        };
        auto c2 = [&](int b) {  // at cell centre b
            return 0.5 * (V(i, b - 1, k) + V(i, b, k)) * (V(i, b, k) - V(i, b - 1, k)) / hy(b);
        };
        auto c3 = [&](int c) {  // at the y-z edge on z-face c
            const double wc = Y.lo[j] * W(i, j, c) + Y.hi[j] * W(i, j + 1, c);
            return wc * (V(i, j, c + 1) - V(i, j, c)) / gz(c);
        };
        double covx = 0.5 * (c1(i - 1) + c1(i));
        double covy = Y.lo[j] * c2(j) + Y.hi[j] * c2(j + 1);
        double covz = 0.5 * (c3(k - 1) + c3(k));
        auto fx = [&](int a) { return (V(a + 1, j, k) - V(a, j, k)) / gx(a); };   // on x-face a
        auto fy = [&](int b) { return (V(i, b, k) - V(i, b - 1, k)) / hy(b); };   // at centre b
        auto fz = [&](int c) { return (V(i, j, c + 1) - V(i, j, c)) / gz(c); };   // on z-face c
        double lap = (fx(i) - fx(i - 1)) / hx(i) + (fy(j + 1) - fy(j)) / gy(j) +
                     (fz(k) - fz(k - 1)) / hz(k);
        double sgs = (2.0 * n12(i, j, k) * e12(U, V, i, j, k) -
                      2.0 * n12(i - 1, j, k) * e12(U, V, i - 1, j, k)) / hx(i) +
                     (2.0 * nut(i, j + 1, k) * fy(j + 1) - 2.0 * nut(i, j, k) * fy(j)) / gy(j) +
                     (2.0 * n23(i, j, k) * e23(V, W, i, j, k) -
                      2.0 * n23(i, j, k - 1) * e23(V, W, i, j, k - 1)) / hz(k);
        return -(covx + covy + covz) + prm.nu * lap + sgs;
    }

    double force_w(const Box& U, const Box& V, const Box& W, int i, int j, int k) const {
        auto c1 = [&](int a) {  // at the x-z edge on x-face a
            const double ua = Z.lo[k] * U(a, j, k) + Z.hi[k] * U(a, j, k + 1);
            return ua * (W(a + 1, j, k) - W(a, j, k)) / gx(a);
        };
        auto c2 = [&](int b) {  // at the y-z edge on y-face b
            const double vb = Z.lo[k] * V(i, b, k) + Z.hi[k] * V(i, b, k + 1);
            return vb * (W(i, b + 1, k) - W(i, b, k)) / gy(b);
        };
        auto c3 = [&](int c) {  // at cell centre c
            return 0.5 * (W(i, j, c - 1) + W(i, j, c)) * (W(i, j, c) - W(i, j, c - 1)) / hz(c);
        };
        double covx = 0.5 * (c1(i - 1) + c1(i));
        double covy = 0.5 * (c2(j - 1) + c2(j));
        double covz = Z.lo[k] * c3(k) + Z.hi[k] * c3(k + 1);
        auto fx = [&](int a) { return (W(a + 1, j, k) - W(a, j, k)) / gx(a); };   // on x-face a
        auto fy = [&](int b) { return (W(i, b + 1, k) - W(i, b, k)) / gy(b); };   // on y-face b
        auto fz = [&](int c) { return (W(i, j, c) - W(i, j, c - 1)) / hz(c); };   // at centre c
        double lap = (fx(i) - fx(i - 1)) / hx(i) + (fy(j) - fy(j - 1)) / hy(j) +
                     (fz(k + 1) - fz(k)) / gz(k);
        double sgs = (2.0 * n13(i, j, k) * e13(U, W, i, j, k) -
                      2.0 * n13(i - 1, j, k) * e13(U, W, i - 1, j, k)) / hx(i) +
                     (2.0 * n23(i, j, k) * e23(V, W, i, j, k) -
                      2.0 * n23(i, j - 1, k) * e23(V, W, i, j - 1, k)) / hy(j) +
                     (2.0 * nut(i, j, k + 1) * fz(k + 1) - 2.0 * nut(i, j, k) * fz(k)) / gz(k);
        return -(covx + covy + covz) + prm.nu * lap + sgs;
    }

    // Faces whose tendency is computed: u on 1..nx-1 (and nx if x+ is an
    // outflow), v on 1..ny-1, w on 1..nz-1.  Others are boundary values.
    int u_last() const { return prm.bc[XP] == BC_OUTFLOW ? nx : nx - 1; }

    void compute_force(const Box& U, const Box& V, const Box& W) {
        const int ul = u_last();
#pragma omp parallel for schedule(static)
        for (int k = 1; k <= nz; ++k)
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) {
                    if (i <= ul) fu(i, j, k) = force_u(U, V, W, i, j, k);
                    if (j <= ny - 1) fv(i, j, k) = force_v(U, V, W, i, j, k);
                    if (k <= nz - 1) fw(i, j, k) = force_w(U, V, W, i, j, k);
                }
    }

    // ------------------------------------------ building effects (feedbf)
    // Feedback forcing on solid faces: usum += dt u; F += alpha usum + beta u.
    void feedback(const Box& U, const Box& V, const Box& W) {
        const int ul = u_last();
        for (int k = 1; k <= nz; ++k)
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) {
                    if (i <= ul && u_solid(i, j, k)) {
                        su(i, j, k) += dt * U(i, j, k);
                        fu(i, j, k) += prm.alpha * su(i, j, k) + prm.beta * U(i, j, k);
                    }
                    if (j <= ny - 1 && v_solid(i, j, k)) {
                        sv(i, j, k) += dt * V(i, j, k);
                        fv(i, j, k) += prm.alpha * sv(i, j, k) + prm.beta * V(i, j, k);
                    }
                    if (k <= nz - 1 && w_solid(i, j, k)) {
                        sw(i, j, k) += dt * W(i, j, k);
                        fw(i, j, k) += prm.alpha * sw(i, j, k) + prm.beta * W(i, j, k);
                    }
                }
    }

    // ----------------------------------------------- Adams-Bashforth (adam)
    // u* = u^n + dt (3/2 F^n - 1/2 F^{n-1}); the first step is forward
    // Euler (F^{n-1} := F^n).  Afterwards F^{n-1} <- F^n.
    void adams_bashforth() {
        const int ul = u_last();
        us = u; vs = v; ws = w;
        for (int k = 1; k <= nz; ++k)
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) {
                    if (i <= ul) {
                        double fo = have_old ? gu(i, j, k) : fu(i, j, k);
                        us(i, j, k) = u(i, j, k) + dt * (1.5 * fu(i, j, k) - 0.5 * fo);
                        gu(i, j, k) = fu(i, j, k);
                    }
                    if (j <= ny - 1) {
                        double fo = have_old ? gv(i, j, k) : fv(i, j, k);
                        vs(i, j, k) = v(i, j, k) + dt * (1.5 * fv(i, j, k) - 0.5 * fo);
                        gv(i, j, k) = fv(i, j, k);
                    }
                    if (k <= nz - 1) {
                        double fo = have_old ? gw(i, j, k) : fw(i, j, k);
                        ws(i, j, k) = w(i, j, k) + dt * (1.5 * fw(i, j, k) - 0.5 * fo);
                        gw(i, j, k) = fw(i, j, k);
                    }
                }
        have_old = true;
    }

    // --------------------------------------------------- divergence, rhs
    double divergence(const Box& U, const Box& V, const Box& W, int i, int j, int k) const {
        return (U(i, j, k) - U(i - 1, j, k)) / hx(i) + (V(i, j, k) - V(i, j - 1, k)) / hy(j) +
               (W(i, j, k) - W(i, j, k - 1)) / hz(k);
    }

    double l2_div(const Box& U, const Box& V, const Box& W) const {
        std::vector<double> part(nz + 2, 0.0);
#pragma omp parallel for schedule(static)
        for (int k = 1; k <= nz; ++k) {
            double s = 0.0;
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) {
                    double d = divergence(U, V, W, i, j, k);
                    s += d * d;
                }
            part[k] = s;
        }
        double t = 0.0;
        for (int k = 1; k <= nz; ++k) t += part[k];
        return std::sqrt(t);
    }

    // rhs = div(u*) / dt; with no Dirichlet face the (volume-weighted) mean
    // is removed.
    void build_rhs() {
#pragma omp parallel for schedule(static)
        for (int k = 1; k <= nz; ++k)
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) rhs(i, j, k) = divergence(us, vs, ws, i, j, k) / dt;
        if (singular()) remove_mean(rhs);
    }

    // Subtract the volume-weighted mean.  With no Dirichlet face, A p = rhs
    // is solvable only when sum V rhs = 0 (V A is symmetric, so the null
    // space of A's transpose is the cell volumes; on a uniform grid this is
    // the plain mean); the same weighted mean fixes the gauge of p.
    void remove_mean(Box& f) const {
        std::vector<double> part(nz + 2, 0.0), vpart(nz + 2, 0.0);
        for (int k = 1; k <= nz; ++k) {
            double s = 0.0, sv = 0.0;
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) {
                    const double vol = hx(i) * hy(j) * hz(k);
                    s += vol * f(i, j, k);
                    sv += vol;
                }
            part[k] = s;
            vpart[k] = sv;
        }
        double t = 0.0, tv = 0.0;
        for (int k = 1; k <= nz; ++k) { t += part[k]; tv += vpart[k]; }
        const double m = t / tv;
        for (int k = 1; k <= nz; ++k)
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) f(i, j, k) -= m;
    }

    // ----------------------------------------------- Poisson, SOR (press)
    // (A p)(i,j,k) = sum of neighbour weights times neighbour p minus the
    // diagonal times p (the discrete Laplacian with folded BCs).
    double apply_A(const Box& P, int i, int j, int k) const {
        return neighbours(P, i, j, k) - diagonal(i, j, k) * P(i, j, k);
    }

    double l2_field(const Box& f) const {
        std::vector<double> part(nz + 2, 0.0);
#pragma omp parallel for schedule(static)
        for (int k = 1; k <= nz; ++k) {
            double s = 0.0;
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) s += f(i, j, k) * f(i, j, k);
            part[k] = s;
        }
        double t = 0.0;
        for (int k = 1; k <= nz; ++k) t += part[k];
        return std::sqrt(t);
    }

    double residual_norm(const Box& P, const Box& R) const {
        std::vector<double> part(nz + 2, 0.0);
#pragma omp parallel for schedule(static)
        for (int k = 1; k <= nz; ++k) {
            double s = 0.0;
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) {
                    double r = R(i, j, k) - apply_A(P, i, j, k);
                    s += r * r;
                }
            part[k] = s;
        }
        double t = 0.0;
        for (int k = 1; k <= nz; ++k) t += part[k];
        return std::sqrt(t);
    }

    // One red-black SOR iteration (section 2.6).  The cells split by the
    // parity of the 0-based index sum i0 + j0 + k0 into colour 0 (even) and
    // colour 1 (odd); every neighbour of a cell has the other colour, so the
    // cells of one colour can be relaxed in any order with the same result.
    // Colour 0 goes first, then colour 1 with the new colour-0 values.  A
    // cell moves from p towards its Gauss-Seidel value
    //   q = (sum of neighbour weights times neighbour p - rhs) / diagonal
    // by the relaxation factor: p <- p + omega (q - p).  Returns the sum of
    // the squared changes over the iteration (the diagnostic the paper
    // accumulates alongside).
    double sor_iteration(Box& P, const Box& R) const {
        double total = 0.0;
        std::vector<double> part(nz + 2, 0.0);
        for (int colour = 0; colour <= 1; ++colour) {
#pragma omp parallel for schedule(static)
            for (int k = 1; k <= nz; ++k) {
                double s = 0.0;
                const int k0 = k - 1;
                for (int j = 1; j <= ny; ++j) {
                    const int j0 = j - 1;
                    // first 0-based i0 of this colour in the row, then every other one
                    for (int i0 = (colour + j0 + k0) & 1; i0 < nx; i0 += 2) {
                        const int i = i0 + 1;
                        const double q = (neighbours(P, i, j, k) - R(i, j, k)) / diagonal(i, j, k);
                        const double change = prm.omega * (q - P(i, j, k));
                        P(i, j, k) += change;
                        s += change * change;
                    }
                }
                part[k] = s;
            }
            for (int k = 1; k <= nz; ++k) total += part[k];
        }
        return total;
    }

    // One iteration of twinned double buffering (section 2.6, the paper's
    // alternative to the red-black scheme on the GPU): with a pair (p_0,
    // p_1) per cell, the first half sets every cell's p_1 from p_0 and the
    // second half p_0 from p_1, each by the relaxation above,
    //   p_dst = p_src + omega (q(p_src) - p_src),
    // so all neighbours come from the previous half: a relaxed Jacobi
    // iteration.  P0 holds the result.
    void twinned_iteration(Box& P0, Box& P1, const Box& R, double omega) const {
        for (int half = 0; half <= 1; ++half) {
            const Box& S = half == 0 ? P0 : P1;
            Box& D = half == 0 ? P1 : P0;
#pragma omp parallel for schedule(static)
            for (int k = 1; k <= nz; ++k)
                for (int j = 1; j <= ny; ++j)
                    for (int i = 1; i <= nx; ++i) {
                        const double q = (neighbours(S, i, j, k) - R(i, j, k)) / diagonal(i, j, k);
                        D(i, j, k) = S(i, j, k) + omega * (q - S(i, j, k));
                    }
        }
    }

    // Iterate to a relative residual ||rhs - A p|| / ||rhs|| <= tol, checked
    // after every check_every iterations and at max_iter.  forced >= 0
    // replays exactly that many iterations instead (no stopping test).
    void solve(Box& P, const Box& R, double tol, int max_iter, int forced) {
        st.rhs_norm = l2_field(R);
        st.reltmp2 = 0.0;
        st.iters = 0;
        st.converged = 1;
        st.resid = 0.0;
        if (forced < 0 && st.rhs_norm == 0.0) return;
        const int K = std::max(1, prm.check_every);
        int m = 0;
        if (forced >= 0) {
            for (m = 0; m < forced; ++m) st.reltmp2 = sor_iteration(P, R);
            st.iters = forced;
            st.resid = st.rhs_norm > 0 ? residual_norm(P, R) / st.rhs_norm : 0.0;
            st.converged = st.resid <= tol ? 1 : 0;
        } else {
            st.converged = 0;
            while (m < max_iter) {
                st.reltmp2 = sor_iteration(P, R);
                ++m;
                if (m % K == 0 || m == max_iter) {
                    st.resid = residual_norm(P, R) / st.rhs_norm;
                    if (st.resid <= tol) { st.converged = 1; break; }
                }
            }
            st.iters = m;
        }
        if (singular()) remove_mean(P);
        st.total_iters += st.iters;
        if (!st.converged) st.not_converged += 1;
    }

    // ------------------------------------------------- projection (velnw)
    // u^{n+1} = u* - dt grad p on faces between two cells (centre difference
    // over the centre distance), plus the outflow face, where p = 0 half a
    // cell from the last centre.
    void project(Box& U, Box& V, Box& W, const Box& P) const {
#pragma omp parallel for schedule(static)
        for (int k = 1; k <= nz; ++k)
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) {
                    if (i <= nx - 1) U(i, j, k) -= dt * (P(i + 1, j, k) - P(i, j, k)) / gx(i);
                    if (j <= ny - 1) V(i, j, k) -= dt * (P(i, j + 1, k) - P(i, j, k)) / gy(j);
                    if (k <= nz - 1) W(i, j, k) -= dt * (P(i, j, k + 1) - P(i, j, k)) / gz(k);
                }
        if (prm.bc[XP] == BC_OUTFLOW)
            for (int k = 1; k <= nz; ++k)
                for (int j = 1; j <= ny; ++j)
                    U(nx, j, k) -= dt * (-2.0 * P(nx, j, k)) / hx(nx);
    }

    double max_cfl(const Box& U, const Box& V, const Box& W) const {
        double c = 0.0;
        for (int k = 1; k <= nz; ++k)
            for (int j = 1; j <= ny; ++j)
                for (int i = 1; i <= nx; ++i) {
                    double uc = 0.5 * std::fabs(U(i, j, k) + U(i - 1, j, k));
                    double vc = 0.5 * std::fabs(V(i, j, k) + V(i, j - 1, k));
                    double wc = 0.5 * std::fabs(W(i, j, k) + W(i, j, k - 1));
                    c = std::max(c, dt * (uc / hx(i) + vc / hy(j) + wc / hz(k)));
                }
        return c;
    }

    // ----------------------------------------------------- one time step
    // Order of work in one step n -> n+1: les, velfg, feedbf, adam, the
    // inflow part of bondv1, press, velnw, the ghost part of bondv1.  This
    // is the paper's cyclic order started at les, so that the step ends
    // with a projected velocity and valid ghosts.
    void time_step(int forced) {
        compute_nut(u, v, w);
        compute_force(u, v, w);
        feedback(u, v, w);
        adams_bashforth();
        if (prm.bc[XM] == BC_INFLOW)
            for (int k = 1; k <= nz; ++k)
                for (int j = 1; j <= ny; ++j) us(0, j, k) = inflow_value(j, k, step + 1);
        build_rhs();
        st.div_star = l2_div(us, vs, ws);
        if (prm.zero_guess) std::fill(p.a.begin(), p.a.end(), 0.0);
        solve(p, rhs, prm.tol, prm.max_iter, forced);
        project(us, vs, ws, p);
        refresh_ghosts(us, vs, ws);
        st.div_new = l2_div(us, vs, ws);
        st.cfl = max_cfl(us, vs, ws);
        std::swap(u.a, us.a);
        std::swap(v.a, vs.a);
        std::swap(w.a, ws.a);
        ++step;
    }
};

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

// =====================================================================
// C interface used by the Python test harness (ctypes).
// Arrays crossing it are float64, C order, i fastest, ghost-free:
//   u [nz][ny][nx+1], v [nz][ny+1][nx], w [nz+1][ny][nx], cell [nz][ny][nx].
// =====================================================================
extern "C" {

// Stretched grid: hx[nx], hy[ny], hz[nz] are the cell widths along each
// axis (the paper's 1-D spacing arrays, section 2.5.3), each > 0 and finite.
void* oracle_create_stretched(int nx, int ny, int nz, const double* hx, const double* hy,
                              const double* hz, double dt, const uint8_t* mask,
                              const OParams* prm) {
    if (nx < 2 || ny < 2 || nz < 2) return nullptr;
    if (!hx || !hy || !hz || !finite_pos(dt) || !prm) return nullptr;
    for (int i = 0; i < nx; ++i) if (!finite_pos(hx[i])) return nullptr;
    for (int j = 0; j < ny; ++j) if (!finite_pos(hy[j])) return nullptr;
    for (int k = 0; k < nz; ++k) if (!finite_pos(hz[k])) return nullptr;
    // x- is inflow or a wall, x+ outflow or a wall, the other faces walls.
    if (prm->bc[XM] == BC_OUTFLOW || prm->bc[XP] == BC_INFLOW) return nullptr;
    for (int f = YM; f <= ZP; ++f)
        if (prm->bc[f] != BC_FREESLIP && prm->bc[f] != BC_NOSLIP) return nullptr;
    Oracle* o = new Oracle();
    o->nx = nx; o->ny = ny; o->nz = nz;
    o->dt = dt;
    o->X.init(hx, nx);
    o->Y.init(hy, ny);
    o->Z.init(hz, nz);
    o->prm = *prm;
    o->solid.assign((size_t)nx * ny * nz, 0);
    if (mask) std::memcpy(o->solid.data(), mask, o->solid.size());
    Box* all[] = {&o->u, &o->v, &o->w, &o->p, &o->us, &o->vs, &o->ws, &o->nut, &o->fu,
                  &o->fv, &o->fw, &o->gu, &o->gv, &o->gw, &o->su, &o->sv, &o->sw, &o->rhs};
    for (Box* b : all) b->init(nx, ny, nz);
    o->prof.assign(nz + 2, 0.0);
    o->build_coefficients();
    return o;
}

// Uniform grid: every cell dx by dy by dz.
void* oracle_create(int nx, int ny, int nz, double dx, double dy, double dz, double dt,
                    const uint8_t* mask, const OParams* prm) {
    if (nx < 2 || ny < 2 || nz < 2) return nullptr;
    if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(dz)) return nullptr;
    std::vector<double> hx(nx, dx), hy(ny, dy), hz(nz, dz);
    return oracle_create_stretched(nx, ny, nz, hx.data(), hy.data(), hz.data(), dt, mask, prm);
}

void oracle_destroy(void* h) { delete static_cast<Oracle*>(h); }

// First call also sets the initial state: u = U(k) on fluid u-faces
// (including the x boundary faces), 0 on solid ones; v = w = p = 0.
int oracle_set_inflow(void* h, const float* profile, double amp, uint64_t seed) {
    Oracle* o = static_cast<Oracle*>(h);
    for (int k = 1; k <= o->nz; ++k) o->prof[k] = (double)profile[k - 1];
    o->amp = amp;
    o->seed = seed;
    o->interp = false;
    if (!o->have_inflow) {
        for (int k = 1; k <= o->nz; ++k)
            for (int j = 1; j <= o->ny; ++j)
                for (int i = 0; i <= o->nx; ++i)
                    o->u(i, j, k) = o->u_solid(i, j, k) ? 0.0 : o->prof[k];
        o->zero_wall_faces(o->u, o->v, o->w);
        o->refresh_ghosts(o->u, o->v, o->w);
        o->have_inflow = true;
    }
    return 0;
}

// Interpolated inflow between (t0, prof0) and (t1, prof1) from the next
// step on; needs oracle_set_inflow first.  Returns -1 on invalid input.
int oracle_set_inflow_pair(void* h, double t0, const float* prof0, double t1, const float* prof1) {
    Oracle* o = static_cast<Oracle*>(h);
    if (!o->have_inflow || !(t1 > t0)) return -1;
    o->prof1.assign(o->nz + 2, 0.0);
    for (int k = 1; k <= o->nz; ++k) {
        o->prof[k] = (double)prof0[k - 1];
        o->prof1[k] = (double)prof1[k - 1];
    }
    o->t0 = t0;
    o->t1 = t1;
    o->interp = true;
    return 0;
}

// Advance n steps.  forced == NULL: SOR to tol; else forced[s] iterations.
int oracle_step(void* h, int n, const int32_t* forced, int32_t* iters_out, OStats* stats) {
    Oracle* o = static_cast<Oracle*>(h);
    o->st.total_iters = 0;
    o->st.not_converged = 0;
    for (int s = 0; s < n; ++s) {
        o->time_step(forced ? forced[s] : -1);
        if (iters_out) iters_out[s] = o->st.iters;
    }
    if (stats) *stats = o->st;
    return o->st.not_converged ? 1 : 0;
}

static void put_owned(Oracle* o, const double* u, const double* v, const double* w) {
    const int nx = o->nx, ny = o->ny, nz = o->nz;
    if (u)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i <= nx; ++i)
                    o->u(i, j + 1, k + 1) = u[((size_t)k * ny + j) * (nx + 1) + i];
    if (v)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i < nx; ++i)
                    o->v(i + 1, j, k + 1) = v[((size_t)k * (ny + 1) + j) * nx + i];
    if (w)
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i)
                    o->w(i + 1, j + 1, k) = w[((size_t)k * ny + j) * nx + i];
}

static void get_cell(const Oracle* o, const Box& b, double* out) {
    const int nx = o->nx, ny = o->ny, nz = o->nz;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) out[((size_t)k * ny + j) * nx + i] = b(i + 1, j + 1, k + 1);
}

static void put_cell(const Oracle* o, Box& b, const double* in) {
    const int nx = o->nx, ny = o->ny, nz = o->nz;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) b(i + 1, j + 1, k + 1) = in[((size_t)k * ny + j) * nx + i];
}

static void get_owned(const Oracle* o, const Box& U, const Box& V, const Box& W, double* u,
                      double* v, double* w) {
    const int nx = o->nx, ny = o->ny, nz = o->nz;
    if (u)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i <= nx; ++i)
                    u[((size_t)k * ny + j) * (nx + 1) + i] = U(i, j + 1, k + 1);
    if (v)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i < nx; ++i)
                    v[((size_t)k * (ny + 1) + j) * nx + i] = V(i + 1, j, k + 1);
    if (w)
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i)
                    w[((size_t)k * ny + j) * nx + i] = W(i + 1, j + 1, k);
}

// Overwrite the state.  Wall-normal faces are forced to zero and ghosts
// refreshed.  The AB2 history is kept unless reset_history is set.
int oracle_set_fields(void* h, const double* u, const double* v, const double* w,
                      const double* p, int reset_history) {
    Oracle* o = static_cast<Oracle*>(h);
    put_owned(o, u, v, w);
    if (p) put_cell(o, o->p, p);
    o->zero_wall_faces(o->u, o->v, o->w);
    o->refresh_ghosts(o->u, o->v, o->w);
    o->have_inflow = true;
    if (reset_history) o->have_old = false;
    return 0;
}

int oracle_get_fields(void* h, double* u, double* v, double* w, double* p) {
    Oracle* o = static_cast<Oracle*>(h);
    get_owned(o, o->u, o->v, o->w, u, v, w);
    if (p) get_cell(o, o->p, p);
    return 0;
}

// Full ghosted boxes of u, v, w ((nz+2)(ny+2)(nx+2) each), for BC tests.
int oracle_get_ghosted(void* h, double* u, double* v, double* w) {
    Oracle* o = static_cast<Oracle*>(h);
    if (u) std::memcpy(u, o->u.a.data(), o->u.a.size() * sizeof(double));
    if (v) std::memcpy(v, o->v.a.data(), o->v.a.size() * sizeof(double));
    if (w) std::memcpy(w, o->w.a.data(), o->w.a.size() * sizeof(double));
    return 0;
}

// Intermediates of the last step: 0 nu_t, 1 rhs (cell arrays);
// 2 F^n, 3 feedback integral usum (u, v, w owned face arrays).
int oracle_get_aux(void* h, int which, double* a, double* b, double* c) {
    Oracle* o = static_cast<Oracle*>(h);
    switch (which) {
        case 0: get_cell(o, o->nut, a); return 0;
        case 1: get_cell(o, o->rhs, a); return 0;
        case 2: get_owned(o, o->gu, o->gv, o->gw, a, b, c); return 0;
        case 3: get_owned(o, o->su, o->sv, o->sw, a, b, c); return 0;
        default: return -1;
    }
}

// ---- stage-level entry points on caller data (used by the pins) ----

// nu_t of the given owned velocity (ghosts from the handle's BCs).
int oracle_nut(void* h, const double* u, const double* v, const double* w, double* nut_out) {
    Oracle* o = static_cast<Oracle*>(h);
    put_owned(o, u, v, w);
    o->refresh_ghosts(o->u, o->v, o->w);
    o->compute_nut(o->u, o->v, o->w);
    get_cell(o, o->nut, nut_out);
    return 0;
}

// Tendency F (advection + diffusion + SGS, no feedback) of the given field.
int oracle_force(void* h, const double* u, const double* v, const double* w, double* fu,
                 double* fv, double* fw) {
    Oracle* o = static_cast<Oracle*>(h);
    put_owned(o, u, v, w);
    o->refresh_ghosts(o->u, o->v, o->w);
    o->compute_nut(o->u, o->v, o->w);
    o->fu.init(o->nx, o->ny, o->nz); o->fv.init(o->nx, o->ny, o->nz); o->fw.init(o->nx, o->ny, o->nz);
    o->compute_force(o->u, o->v, o->w);
    get_owned(o, o->fu, o->fv, o->fw, fu, fv, fw);
    return 0;
}

// Cell divergence of the given owned face velocity.
int oracle_divergence(void* h, const double* u, const double* v, const double* w, double* div) {
    Oracle* o = static_cast<Oracle*>(h);
    Box U, V, W;
    U.init(o->nx, o->ny, o->nz); V.init(o->nx, o->ny, o->nz); W.init(o->nx, o->ny, o->nz);
    std::swap(U.a, o->u.a); std::swap(V.a, o->v.a); std::swap(W.a, o->w.a);
    put_owned(o, u, v, w);
    for (int k = 1; k <= o->nz; ++k)
        for (int j = 1; j <= o->ny; ++j)
            for (int i = 1; i <= o->nx; ++i)
                div[((size_t)(k - 1) * o->ny + (j - 1)) * o->nx + (i - 1)] =
                    o->divergence(o->u, o->v, o->w, i, j, k);
    std::swap(U.a, o->u.a); std::swap(V.a, o->v.a); std::swap(W.a, o->w.a);
    return 0;
}

// Projection u -= dt grad p applied to caller arrays (in place).
int oracle_project(void* h, double* u, double* v, double* w, const double* p) {
    Oracle* o = static_cast<Oracle*>(h);
    Box U, V, W, P;
    U.init(o->nx, o->ny, o->nz); V.init(o->nx, o->ny, o->nz); W.init(o->nx, o->ny, o->nz);
    P.init(o->nx, o->ny, o->nz);
    std::swap(U.a, o->u.a); std::swap(V.a, o->v.a); std::swap(W.a, o->w.a);
    put_owned(o, u, v, w);
    put_cell(o, P, p);
    o->project(o->u, o->v, o->w, P);
    get_owned(o, o->u, o->v, o->w, u, v, w);
    std::swap(U.a, o->u.a); std::swap(V.a, o->v.a); std::swap(W.a, o->w.a);
    return 0;
}

// (A p) on the cell array.
int oracle_apply_A(void* h, const double* p, double* ap) {
    Oracle* o = static_cast<Oracle*>(h);
    Box P;
    P.init(o->nx, o->ny, o->nz);
    put_cell(o, P, p);
    for (int k = 1; k <= o->nz; ++k)
        for (int j = 1; j <= o->ny; ++j)
            for (int i = 1; i <= o->nx; ++i)
                ap[((size_t)(k - 1) * o->ny + (j - 1)) * o->nx + (i - 1)] = o->apply_A(P, i, j, k);
    return 0;
}

// Stand-alone pressure solve with the handle's operator.  p is the initial
// guess on entry and the solution on exit.  forced >= 0 replays that many
// iterations.  A singular operator gets rhs mean removal first.
int oracle_pressure_solve(void* h, const double* rhs, double* p, double tol, int max_iter,
                          int forced, OStats* stats) {
    Oracle* o = static_cast<Oracle*>(h);
    Box R, P;
    R.init(o->nx, o->ny, o->nz);
    P.init(o->nx, o->ny, o->nz);
    put_cell(o, R, rhs);
    put_cell(o, P, p);
    if (o->singular()) o->remove_mean(R);
    o->st.total_iters = 0;
    o->st.not_converged = 0;
    o->solve(P, R, tol, max_iter, forced);
    get_cell(o, P, p);
    if (stats) *stats = o->st;
    return o->st.converged ? 0 : 1;
}

// Exactly n SOR iterations (no stopping test) on caller arrays; returns the
// sum of reltmp^2 of the last iteration.
double oracle_sor_iterations(void* h, const double* rhs, double* p, int n) {
    Oracle* o = static_cast<Oracle*>(h);
    Box R, P;
    R.init(o->nx, o->ny, o->nz);
    P.init(o->nx, o->ny, o->nz);
    put_cell(o, R, rhs);
    put_cell(o, P, p);
    double s = 0.0;
    for (int m = 0; m < n; ++m) s = o->sor_iteration(P, R);
    get_cell(o, P, p);
    return s;
}

// Exactly n twinned double-buffer iterations (relaxation omega) on caller
// arrays; p is the start on entry and p_0 after the last iteration on exit.
int oracle_twinned_iterations(void* h, const double* rhs, double* p, double omega, int n) {
    Oracle* o = static_cast<Oracle*>(h);
    Box R, P0, P1;
    R.init(o->nx, o->ny, o->nz);
    P0.init(o->nx, o->ny, o->nz);
    P1.init(o->nx, o->ny, o->nz);
    put_cell(o, R, rhs);
    put_cell(o, P0, p);
    for (int m = 0; m < n; ++m) o->twinned_iteration(P0, P1, R, omega);
    get_cell(o, P0, p);
    return 0;
}

// Relative residual ||rhs - A p|| / ||rhs|| of caller arrays.
double oracle_residual(void* h, const double* rhs, const double* p) {
    Oracle* o = static_cast<Oracle*>(h);
    Box R, P;
    R.init(o->nx, o->ny, o->nz);
    P.init(o->nx, o->ny, o->nz);
    put_cell(o, R, rhs);
    put_cell(o, P, p);
    double n = o->l2_field(R);
    return n > 0 ? o->residual_norm(P, R) / n : 0.0;
}

uint64_t oracle_splitmix64(uint64_t x) { return splitmix64(x); }

double oracle_inflow_value(void* h, int j, int k, int64_t step) {
    return static_cast<Oracle*>(h)->inflow_value(j, k, step);
}

}  // extern "C"
