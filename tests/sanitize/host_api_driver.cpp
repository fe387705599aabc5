// host_api_driver.cpp -- the host side of liblbm (parameter validation, workspace layouts, the
// thermodynamic solvers, error strings) exercised without a GPU, for a build of the library's
// host code under AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
// Every call here returns before the library's first HIP call. Exit status 0 on success.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/lbm.h"

static int failures = 0;
#define EXPECT(cond)                                                      \
    do {                                                                  \
        if (!(cond)) {                                                    \
            ++failures;                                                   \
            std::fprintf(stderr, "FAIL line %d: %s\n", __LINE__, #cond); \
        }                                                                 \
    } while (0)

static lbm_params good(int nx = 64, int ny = 32, int walls = 1) {
    lbm_params p;
    std::memset(&p, 0, sizeof p);
    p.abi_version = LBM_ABI_VERSION;
    p.nx = nx;
    p.ny = ny;
    p.walls = walls;
    p.ghost_psi = walls == LBM_WALLS_MASK ? 0 : 1;
    p.eos = LBM_EOS_CS;
    p.wall_force = LBM_WALL_MODPSI;
    p.a = 0.5; p.b = 4.0; p.R = 1.0; p.T = 0.0244618784;
    p.G = -1.0; p.sigma = 0.11244;
    p.s_rho = 1.0; p.s_e = 0.8; p.s_zeta = 0.8; p.s_j = 1.0; p.s_q = 1.1;
    p.tau_l = 0.6; p.tau_v = 1.0;
    p.rho_l = 0.4450633; p.rho_v = 8.901265e-4;
    return p;
}

int main() {
    // thermodynamics
    double rv, rl, p0, T, r1, r2, pr;
    EXPECT(lbm_cs_temperature(0.5, 4.0, 1.0, 500.0, &T) == LBM_OK);
    EXPECT(lbm_maxwell_cs(0.5, 4.0, 1.0, T, &rv, &rl, &p0) == LBM_OK);
    EXPECT(std::fabs(rl / rv - 500.0) < 1e-6);
    EXPECT(lbm_maxwell_cs(0.5, 4.0, 1.0, 0.05, &rv, &rl, &p0) == LBM_E_INVAL);
    EXPECT(lbm_maxwell_cs(0.5, 4.0, 1.0, T, nullptr, &rl, &p0) == LBM_E_INVAL);
    EXPECT(lbm_piecewise_spinodals(1.0, 500.0, 0.64 / 3, -0.04 / 3, 1.0 / 3, &r1, &r2) == LBM_OK);
    EXPECT(std::fabs(r1 - 1.36) < 0.005 && std::fabs(r2 - 481.04) < 0.005);
    EXPECT(lbm_piecewise_spinodals(1.0, 500.0, 0.64 / 3, 1.0 / 3, 1.0 / 3, &r1, &r2) == LBM_E_INVAL);
    lbm_params q = good();
    EXPECT(lbm_pressure(&q, 0.3, &pr) == LBM_OK && std::isfinite(pr));
    EXPECT(lbm_pressure(&q, -1.0, &pr) == LBM_E_INVAL);

    // workspace sizes of every geometry, and rejected parameter blocks
    size_t n = 0, m = 0;
    for (int walls = 0; walls <= 3; ++walls) {
        lbm_params g = good(100, 50, walls);
        EXPECT(lbm_workspace_size(&g, &n) == LBM_OK && n > 2 * 9 * 100 * 50 * sizeof(double));
    }
    q = good(1024, 512);
    EXPECT(lbm_workspace_size(&q, &m) == LBM_OK && m > n);
    EXPECT(lbm_adjoint_workspace_size(&q, 4000, 200, &n) == LBM_OK && n > 20 * m / 2);
    lbm_params wet = good(64, 32, LBM_WALLS_WET_NODE);
    EXPECT(lbm_adjoint_workspace_size(&wet, 100, 10, &n) == LBM_E_INVAL);
    struct Bad { size_t off; double dv; int iv; bool is_int; int code; };
    const Bad bad[] = {
        {offsetof(lbm_params, abi_version), 0, 99, true, LBM_E_ABI},
        {offsetof(lbm_params, nx), 0, 2, true, LBM_E_INVAL},
        {offsetof(lbm_params, ny), 0, 3, true, LBM_E_INVAL},
        {offsetof(lbm_params, walls), 0, 4, true, LBM_E_INVAL},
        {offsetof(lbm_params, ghost_psi), 0, 7, true, LBM_E_INVAL},
        {offsetof(lbm_params, eos), 0, 5, true, LBM_E_INVAL},
        {offsetof(lbm_params, wall_force), 0, 3, true, LBM_E_INVAL},
        {offsetof(lbm_params, reserved), 0, 1, true, LBM_E_INVAL},
        {offsetof(lbm_params, G), 1.0, 0, false, LBM_E_INVAL},
        {offsetof(lbm_params, sigma), INFINITY, 0, false, LBM_E_INVAL},
        {offsetof(lbm_params, s_q), 2.0, 0, false, LBM_E_INVAL},
        {offsetof(lbm_params, tau_l), 0.5, 0, false, LBM_E_INVAL},
        {offsetof(lbm_params, rho_v), 0.0, 0, false, LBM_E_INVAL},
        {offsetof(lbm_params, T), -1.0, 0, false, LBM_E_INVAL},
    };
    std::vector<double> rho0(64 * 32, 0.3), gw(2 * 64, 0.0);
    for (const Bad& b : bad) {
        lbm_params x = good();
        if (b.is_int) std::memcpy((char*)&x + b.off, &b.iv, sizeof(int32_t));
        else std::memcpy((char*)&x + b.off, &b.dv, sizeof(double));
        EXPECT(lbm_workspace_size(&x, &n) == b.code);
        lbm_ctx* c = nullptr;
        EXPECT(lbm_create(&x, gw.data(), rho0.data(), (void*)256, size_t(1) << 40, nullptr, &c) == b.code);
        EXPECT(c == nullptr);
    }

    // buffers rejected before any HIP call
    q = good();
    EXPECT(lbm_workspace_size(&q, &n) == LBM_OK);
    lbm_ctx* c = nullptr;
    EXPECT(lbm_create(&q, gw.data(), rho0.data(), (void*)256, n - 1, nullptr, &c) == LBM_E_SIZE);
    EXPECT(lbm_create(&q, gw.data(), rho0.data(), (void*)8, n, nullptr, &c) == LBM_E_INVAL);
    EXPECT(lbm_create(&q, nullptr, rho0.data(), (void*)256, n, nullptr, &c) == LBM_E_INVAL);
    std::vector<double> bad_rho = rho0;
    bad_rho[5 * 64 + 5] = 0.0;
    EXPECT(lbm_create(&q, gw.data(), bad_rho.data(), (void*)256, n, nullptr, &c) == LBM_E_INVAL);
    std::vector<double> bad_gw = gw;
    bad_gw[3] = NAN;
    EXPECT(lbm_create(&q, bad_gw.data(), rho0.data(), (void*)256, n, nullptr, &c) == LBM_E_INVAL);
    lbm_params mk = good(64, 32, LBM_WALLS_MASK);
    EXPECT(lbm_create(&mk, gw.data(), rho0.data(), (void*)256, n, nullptr, &c) == LBM_E_INVAL);

    // ensembles: sizes and rejections
    lbm_params ens[3] = {good(128, 64), good(192, 96), good(64, 32)};
    lbm_tune t{1, 0, 0, 2};
    EXPECT(lbm_batch_workspace_size(ens, 3, &t, &n) == LBM_OK);
    lbm_tune tb{7, 0, 0, 2};
    EXPECT(lbm_batch_workspace_size(ens, 3, &tb, &n) == LBM_E_INVAL);
    lbm_tune tw{4, 0, 0, 2};  // the 32 x 4 tile
    EXPECT(lbm_batch_workspace_size(ens, 3, &tw, &n) == LBM_OK);
    tw.tile = 5;
    EXPECT(lbm_batch_workspace_size(ens, 3, &tw, &n) == LBM_E_INVAL);
    EXPECT(lbm_batch_workspace_size(ens, 3, &t, &n) == LBM_OK);
    lbm_params mixed[2] = {good(64, 32), good(64, 32, LBM_WALLS_MASK)};
    EXPECT(lbm_batch_workspace_size(mixed, 2, nullptr, &n) == LBM_E_INVAL);
    lbm_batch* b = nullptr;
    EXPECT(lbm_batch_create(ens, 3, nullptr, nullptr, &t, (void*)256, n, nullptr, &b) == LBM_E_INVAL);

    // null handles and error strings
    EXPECT(lbm_step(nullptr, 1) == LBM_E_INVAL);
    EXPECT(lbm_observables(nullptr, nullptr) == LBM_E_INVAL);
    EXPECT(lbm_destroy(nullptr) == LBM_E_INVAL);
    EXPECT(lbm_batch_destroy(nullptr) == LBM_E_INVAL);
    for (int code = 1; code >= -7; --code) EXPECT(std::strlen(lbm_strerror(code)) > 0);
    EXPECT(lbm_last_error(nullptr) != nullptr);
    std::printf("%s: %d failure(s)\n", failures ? "FAILED" : "passed", failures);
    return failures ? 1 : 0;
}
