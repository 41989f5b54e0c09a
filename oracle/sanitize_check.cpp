// Test infrastructure: a driver for building the oracle with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host (tests/test_sanitize_cpu.py).
// It runs every entry point of the oracle once on small grids -- uniform and
// stretched, with buildings, inflow noise and an outflow face, and on the
// all-wall (singular) operator -- so an out-of-range access or undefined
// arithmetic anywhere in them aborts the run.  Compiled as one translation
// unit with the oracle itself.
#include "les_oracle.cpp"

#include <cstdio>
#include <vector>

static int fail(const char* what) {
    std::fprintf(stderr, "sanitize_check: %s\n", what);
    return 1;
}

static int run_case(bool stretched, bool walls_only) {
    const int nx = 13, ny = 9, nz = 7;
    OParams prm{};
    prm.omega = 1.8;
    prm.tol = 1e-8;
    prm.check_every = 4;
    prm.max_iter = 3000;
    prm.cs = 0.1;
    prm.nu = 1e-5;
    prm.alpha = -10.0;
    prm.beta = -1.0;
    for (int f = 0; f < 6; ++f) prm.bc[f] = BC_NOSLIP;
    if (!walls_only) {
        prm.bc[XM] = BC_INFLOW;
        prm.bc[XP] = BC_OUTFLOW;
        prm.bc[ZP] = BC_FREESLIP;
    }
    std::vector<uint8_t> mask((size_t)nx * ny * nz, 0);
    for (int k = 0; k < 3; ++k)
        for (int j = 3; j < 6; ++j)
            for (int i = 5; i < 8; ++i) mask[((size_t)k * ny + j) * nx + i] = 1;
    void* h;
    if (stretched) {
        std::vector<double> hx(nx), hy(ny), hz(nz);
        for (int i = 0; i < nx; ++i) hx[i] = 2.0 + 0.1 * i;
        for (int j = 0; j < ny; ++j) hy[j] = 2.5 - 0.05 * j;
        for (int k = 0; k < nz; ++k) hz[k] = 1.0 * std::pow(1.1, k);
        h = oracle_create_stretched(nx, ny, nz, hx.data(), hy.data(), hz.data(), 0.05, mask.data(), &prm);
    } else {
        h = oracle_create(nx, ny, nz, 2.0, 2.0, 1.0, 0.05, mask.data(), &prm);
    }
    if (!h) return fail("create");
    std::vector<float> prof(nz);
    for (int k = 0; k < nz; ++k) prof[k] = 1.0f + 0.2f * k;
    if (oracle_set_inflow(h, prof.data(), 0.01, 7) != 0) return fail("set_inflow");
    std::vector<float> prof2(prof);
    for (float& x : prof2) x *= 1.5f;
    if (!walls_only && oracle_set_inflow_pair(h, 0.0, prof.data(), 1.0, prof2.data()) != 0)
        return fail("set_inflow_pair");
    std::vector<int32_t> its(2);
    OStats st{};
    if (oracle_step(h, 2, nullptr, its.data(), &st) < 0) return fail("step");
    const int32_t forced[1] = {5};
    if (oracle_step(h, 1, forced, its.data(), &st) < 0) return fail("forced step");
    const size_t nu = (size_t)(nx + 1) * ny * nz, nv = (size_t)nx * (ny + 1) * nz,
                 nw = (size_t)nx * ny * (nz + 1), nc = (size_t)nx * ny * nz;
    std::vector<double> u(nu), v(nv), w(nw), p(nc), a(nc), b(nc), d(nc);
    if (oracle_get_fields(h, u.data(), v.data(), w.data(), p.data()) != 0) return fail("get_fields");
    const size_t ng = (size_t)(nx + 2) * (ny + 2) * (nz + 2);   // ghosted box of every field
    std::vector<double> gu(ng), gv(ng), gw(ng);
    oracle_get_ghosted(h, gu.data(), gv.data(), gw.data());
    std::vector<double> fu(nu), fv(nv), fw(nw);
    oracle_get_aux(h, 0, a.data(), nullptr, nullptr);
    oracle_get_aux(h, 1, a.data(), nullptr, nullptr);
    oracle_get_aux(h, 2, fu.data(), fv.data(), fw.data());
    oracle_get_aux(h, 3, fu.data(), fv.data(), fw.data());
    if (oracle_set_fields(h, u.data(), v.data(), w.data(), p.data(), 0) != 0) return fail("set_fields");
    if (oracle_step(h, 1, nullptr, its.data(), &st) < 0) return fail("step after set_fields");
    oracle_nut(h, u.data(), v.data(), w.data(), a.data());
    oracle_force(h, u.data(), v.data(), w.data(), fu.data(), fv.data(), fw.data());
    oracle_divergence(h, u.data(), v.data(), w.data(), d.data());
    oracle_project(h, u.data(), v.data(), w.data(), p.data());
    oracle_apply_A(h, p.data(), a.data());
    for (size_t e = 0; e < nc; ++e) b[e] = std::sin(0.3 * (double)e);
    std::vector<double> q(nc, 0.0);
    oracle_pressure_solve(h, b.data(), q.data(), 1e-6, 5000, -1, &st);
    oracle_sor_iterations(h, b.data(), q.data(), 7);
    oracle_twinned_iterations(h, b.data(), q.data(), 1.7, 6);
    const double r = oracle_residual(h, b.data(), q.data());
    if (!std::isfinite(r)) return fail("residual");
    if (!walls_only) (void)oracle_inflow_value(h, 2, 3, 4);
    oracle_destroy(h);
    return 0;
}

int main() {
    int rc = 0;
    rc |= run_case(false, false);
    rc |= run_case(true, false);
    rc |= run_case(false, true);
    if (rc == 0) std::printf("sanitize_check: ok\n");
    return rc;
}
