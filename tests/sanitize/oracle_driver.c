/*
 * oracle_driver.c -- runs every entry point of the C oracle on small lattices of each geometry,
 * equation of state and adhesion form, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py). Exit status 0 when every call
 * succeeded and every result is finite.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/lbm_oracle.c"

static int failures = 0;

static void expect(int ok, const char *what, int walls, int eos, int form)
{
    if (!ok) {
        ++failures;
        fprintf(stderr, "FAIL %s (walls=%d eos=%d form=%d)\n", what, walls, eos, form);
    }
}

int main(void)
{
    const int nx = 23, ny = 14;
    const size_t N = (size_t)nx * ny;
    double *f = malloc(9 * N * sizeof(double)), *rho0 = malloc(N * sizeof(double));
    double *gw = malloc(N * sizeof(double));
    double *rho = malloc(N * sizeof(double)), *psi = malloc(N * sizeof(double));
    double *Fm = malloc(2 * N * sizeof(double)), *Fa = malloc(2 * N * sizeof(double));
    double *v = malloc(2 * N * sizeof(double));
    uint8_t *solid = calloc(N, 1);
    for (int x = 0; x < nx; ++x) {  /* base and top rows, short pillars */
        solid[x] = solid[(size_t)(ny - 1) * nx + x] = 1;
        if (x % 3 != 2) solid[(size_t)nx + x] = solid[(size_t)2 * nx + x] = 1;
    }
    for (int walls = 0; walls <= 3; ++walls)
        for (int eos = 0; eos <= 1; ++eos)
            for (int form = 0; form <= 2; ++form) {
                orc_params p = {0};
                p.nx = nx; p.ny = ny; p.walls = walls; p.ghost = walls == 3 ? 0 : 1;
                p.eos = eos; p.wall_force = form; p.G = -1.0;
                p.s_rho = 1.0; p.s_e = 0.8; p.s_zeta = 0.8; p.s_j = 1.0; p.s_q = 1.1;
                p.tau_l = 0.6; p.tau_v = 1.0;
                if (eos == 0) {
                    p.a = 0.5; p.b = 4.0; p.R = 1.0; p.T = 0.0244618784; p.sigma = 0.11244;
                    p.rho_v = 8.901265e-4; p.rho_l = 0.4450633;
                } else {
                    p.th_v = 0.64 / 3.0; p.th_m = -0.04 / 3.0; p.th_l = 1.0 / 3.0;
                    p.rho1 = 1.3585916; p.rho2 = 481.04216; p.sigma = 0.084;
                    p.rho_v = 1.0; p.rho_l = 500.0;
                }
                p.solid = walls == 3 ? solid : NULL;
                for (int y = 0; y < ny; ++y)
                    for (int x = 0; x < nx; ++x) {
                        double d = hypot(x - 0.5 * nx, y - (walls == 0 ? 0.5 * ny : 4.0));
                        rho0[(size_t)y * nx + x] =
                            p.rho_v + (p.rho_l - p.rho_v) * 0.5 * (1.0 - tanh((d - 5.0) / 2.0));
                        gw[(size_t)y * nx + x] = 0.01 * ((x + 2 * y) % 5 - 2);
                    }
                expect(orc_init_rest(&p, rho0, f) == 0, "init", walls, eos, form);
                expect(orc_run(&p, gw, f, 12) == 0, "run", walls, eos, form);
                expect(orc_fields(&p, gw, f, rho, psi, Fm, Fa, v) == 0, "fields", walls, eos,
                       form);
                int finite = 1;
                for (size_t i = 0; i < 9 * N; ++i) finite &= isfinite(f[i]) != 0;
                for (size_t i = 0; i < 2 * N; ++i) finite &= isfinite(v[i]) && isfinite(Fm[i]);
                expect(finite, "finite state", walls, eos, form);
                double fin[9], fout[9], Fm2[2] = {1e-3, -2e-3}, F2[2] = {2e-3, -1e-3};
                for (int a = 0; a < 9; ++a) fin[a] = f[a * N + (size_t)(ny / 2) * nx + 3];
                orc_collide_node(&p, fin, 0.3, Fm2, F2, fout);
                for (int a = 0; a < 9; ++a) finite &= isfinite(fout[a]) != 0;
                expect(finite, "collide", walls, eos, form);
                expect(orc_psi(&p, p.rho_l) >= 0.0, "psi", walls, eos, form);
            }
    double M81[81], w9[9];
    int ex9[9], ey9[9], op9[9];
    orc_tables(M81, ex9, ey9, op9, w9);
    /* rejected parameters */
    orc_params bad = {0};
    bad.nx = 2; bad.ny = 10;
    expect(orc_run(&bad, gw, f, 1) == ORC_E_INVAL, "reject nx", 0, 0, 0);
    free(f); free(rho0); free(gw); free(rho); free(psi); free(Fm); free(Fa); free(v); free(solid);
    printf("%s: %d failure(s)\n", failures ? "FAILED" : "passed", failures);
    return failures ? 1 : 0;
}
