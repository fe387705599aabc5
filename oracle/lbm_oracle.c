/*
 * lbm_oracle.c -- FP64 CPU oracle of the D2Q9 MRT pseudopotential lattice Boltzmann step with
 * fluid-solid adhesion (Q. Li, K. H. Luo, Q. J. Kang, Q. Chen, "Contact angles in the
 * pseudopotential lattice Boltzmann modeling of wetting", 2014).
 *
 * TEST INFRASTRUCTURE. This file is a plain, slow, obviously correct reference used only by the
 * tests, the smoke check and the CPU-baseline leg of the benchmark. It shares no code, header,
 * table or constant with the HIP library, and the library never calls it.
 *
 * Layout: populations f[a][y][x] (a = 0..8, x fastest), pre-collision (post-streaming) values,
 * i.e. the f_alpha(x, t) of Eq. (1). With walls, rows y = 0 and y = ny-1 are solid nodes and the
 * fluid occupies 1 <= y <= ny-2; x is periodic. Without walls both directions are periodic.
 * Two wall schemes: halfway bounce-back (walls = 1; the wall plane lies halfway between the solid
 * row and the first fluid row) and the non-slip wet-node scheme of Sec. III.A (walls = 2; rows 1
 * and ny-2 are boundary nodes on the wall plane whose populations arriving from the solid are
 * reconstructed so that the node's velocity, Eq. (6), is zero). With walls = 3 the lattice is
 * periodic in both directions and an arbitrary solid mask (rough surfaces, Sec. III.B) defines the
 * solid nodes: halfway bounce-back on every link from a solid node, psi = 0 on solid nodes (no
 * ghost layer) and G_w given per solid node.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off [-fopenmp] -shared -fPIC. Every per-node loop writes
 * only its own node, so the result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_E_INVAL = -1, ORC_E_PSI = -2, ORC_E_NOMEM = -3 };
enum { ORC_EOS_CS = 0, ORC_EOS_PIECEWISE = 1 };
enum { ORC_WALL_RHO = 0, ORC_WALL_PSI = 1, ORC_WALL_MODPSI = 2 };

typedef struct {
    int32_t nx, ny;
    int32_t walls;       /* 1, 2: solid rows y = 0 and y = ny-1 (1 bounce-back, 2 wet-node);
                            0: periodic in y as well */
    int32_t ghost;       /* 1: Eq. (7) also acts across the wall through mirrored psi rows */
    int32_t eos;         /* ORC_EOS_CS or ORC_EOS_PIECEWISE (Eq. 15) */
    int32_t wall_force;  /* ORC_WALL_RHO (Eq. 10), ORC_WALL_PSI (Eq. 11), ORC_WALL_MODPSI (Eq. 14) */
    double a, b, R, T;   /* Carnahan-Starling constants */
    double rho1, rho2, th_v, th_m, th_l; /* Eq. (15): spinodal densities and slopes */
    double G, sigma;     /* Eq. (7) strength, Eq. (9) tuning parameter */
    double s_rho, s_e, s_zeta, s_j, s_q; /* diagonal of Lambda, Eq. (2) */
    double tau_l, tau_v; /* tau_nu in the liquid and in the vapour */
    double rho_l, rho_v; /* coexistence densities (viscosity interpolation) */
    const uint8_t *solid; /* walls = 3: [ny][nx], 1 = solid node; otherwise unused */
} orc_params;

/* D2Q9 velocities: 0 rest; 1..4 = E, N, W, S; 5..8 = NE, NW, SW, SE (numbering that the paper's
 * wall formulas of Sec. III.A use). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* Orthogonal D2Q9 moment basis of the MRT model the paper cites (Lallemand and Luo):
 * rows m = (rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy). */
static const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

/* Interaction weights of Eq. (7): 1/3 for |e|^2 = 1, 1/12 for |e|^2 = 2. */
static double w_alpha(int a)
{
    int e2 = EX[a] * EX[a] + EY[a] * EY[a];
    return e2 == 1 ? 1.0 / 3.0 : (e2 == 2 ? 1.0 / 12.0 : 0.0);
}

/* Copy-outs so tests can check the tables against the paper's equations. */
void orc_tables(double *M81, int *ex9, int *ey9, int *opp9, double *w9)
{
    for (int k = 0; k < 9; ++k) {
        for (int j = 0; j < 9; ++j) M81[9 * k + j] = MM[k][j];
        ex9[k] = EX[k]; ey9[k] = EY[k]; opp9[k] = OPP[k]; w9[k] = w_alpha(k);
    }
}

/* Equation of state p_EOS(rho): Carnahan-Starling or the piecewise-linear Eq. (15). */
double orc_p_eos(const orc_params *p, double rho)
{
    if (p->eos == ORC_EOS_CS) {
        double eta = p->b * rho / 4.0;
        double num = 1.0 + eta + eta * eta - eta * eta * eta;
        double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
        return rho * p->R * p->T * num / den - p->a * rho * rho;
    }
    if (rho <= p->rho1) return rho * p->th_v;
    if (rho <= p->rho2) return p->rho1 * p->th_v + (rho - p->rho1) * p->th_m;
    return p->rho1 * p->th_v + (p->rho2 - p->rho1) * p->th_m + (rho - p->rho2) * p->th_l;
}

/* psi = sqrt(2 (p_EOS - rho c_s^2) / (G c^2)) with c = 1, c_s^2 = 1/3 (Sec. II.B). Returns -1
 * when the radicand is negative (psi undefined). */
double orc_psi(const orc_params *p, double rho)
{
    double rad = 2.0 * (orc_p_eos(p, rho) - rho / 3.0) / p->G;
    if (!(rad >= 0.0)) return -1.0;
    return sqrt(rad);
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* Geometry: solid rows 0 and ny-1 (walls = 1, 2), the mask (walls = 3, coordinates wrapped), or
 * no solid at all (walls = 0). Rows outside the lattice only arise with walls = 1, 2. */
static int is_solid(const orc_params *p, int x, int y)
{
    if (p->walls == 3) return p->solid[(size_t)wrap(y, p->ny) * p->nx + wrap(x, p->nx)] != 0;
    return (p->walls == 1 || p->walls == 2) && (y == 0 || y == p->ny - 1);
}

/* Row of a neighbour: wrapped where y is periodic (walls = 0, 3). */
static int nb_row(const orc_params *p, int y)
{
    return (p->walls == 0 || p->walls == 3) ? wrap(y, p->ny) : y;
}

/* S1, S2: density and pseudopotential of every fluid node; ghost psi on the solid rows. */
static int density_and_psi(const orc_params *p, const double *f, double *rho, double *psi)
{
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    int bad = 0;
#pragma omp parallel for reduction(| : bad)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            if (is_solid(p, x, y)) { rho[i] = 0.0; psi[i] = 0.0; continue; }
            double s = 0.0;
            for (int a = 0; a < 9; ++a) s += f[a * N + i];        /* Eq. (6) */
            rho[i] = s;
            psi[i] = orc_psi(p, s);
            if (psi[i] < 0.0) bad = 1;
        }
    }
    if (bad) return ORC_E_PSI;
    if (p->walls == 1 || p->walls == 2) {
        /* Eq. (7) applied at the wall: the solid row takes the psi of the fluid row next to it
         * (with bounce-back, the mirror image about the wall plane halfway between them; with
         * the wet-node scheme, the psi of the boundary node on the wall plane). */
        for (int x = 0; x < nx; ++x) {
            psi[x] = p->ghost ? psi[(size_t)nx + x] : 0.0;
            psi[(size_t)(ny - 1) * nx + x] = p->ghost ? psi[(size_t)(ny - 2) * nx + x] : 0.0;
        }
    }
    return ORC_OK;
}

/* S3-S5 at one fluid node: cohesive force Eq. (7), adhesive force Eq. (10)/(11)/(14), total
 * force and velocity Eq. (6). gw: G_w of the solid nodes, [2][nx] for the bottom (row 0) and top
 * (row 1) walls, or [ny][nx] per node with walls = 3. */
static void forces_at(const orc_params *p, const double *gw, const double *f, const double *rho,
                      const double *psi, int x, int y, double Fm[2], double Fads[2], double F[2],
                      double v[2])
{
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    const size_t i = (size_t)y * nx + x;
    const double G = p->G;

    /* Eq. (7): F_m = -G psi(x) sum_a w_a psi(x + e_a) e_a */
    double sx = 0.0, sy = 0.0;
    for (int a = 1; a < 9; ++a) {
        int xn = wrap(x + EX[a], nx);
        int yn = nb_row(p, y + EY[a]);
        double pn = psi[(size_t)yn * nx + xn];
        sx += w_alpha(a) * pn * EX[a];
        sy += w_alpha(a) * pn * EY[a];
    }
    Fm[0] = -G * psi[i] * sx;
    Fm[1] = -G * psi[i] * sy;

    /* Eqs. (10), (11), (14): F_ads = -G_w P(x) sum_a omega_a s(x + e_a) e_a, omega_a = c_s^2 w_a,
     * with pre-sum factor P = rho, psi, or psi * phi with phi = psi. The G_w of the solid node
     * x + e_a sits inside the sum, so a per-node wettability pattern is supported. */
    Fads[0] = Fads[1] = 0.0;
    if (p->walls) {
        double pre;
        if (p->wall_force == ORC_WALL_RHO) pre = rho[i];
        else if (p->wall_force == ORC_WALL_PSI) pre = psi[i];
        else pre = psi[i] * psi[i];
        double ax = 0.0, ay = 0.0;
        for (int a = 1; a < 9; ++a) {
            int yn = nb_row(p, y + EY[a]);
            int xn = wrap(x + EX[a], nx);
            if (!is_solid(p, xn, yn)) continue;
            double g = p->walls == 3 ? gw[(size_t)yn * nx + xn]
                                     : gw[(yn == 0 ? 0 : 1) * (size_t)nx + xn];
            double om = w_alpha(a) / 3.0;
            ax += om * g * EX[a];
            ay += om * g * EY[a];
        }
        Fads[0] = -pre * ax;
        Fads[1] = -pre * ay;
    }
    F[0] = Fm[0] + Fads[0];
    F[1] = Fm[1] + Fads[1];

    /* Eq. (6): rho v = sum_a e_a f_a + F / 2 */
    double jx = 0.0, jy = 0.0;
    for (int a = 0; a < 9; ++a) {
        jx += EX[a] * f[a * N + i];
        jy += EY[a] * f[a * N + i];
    }
    v[0] = (jx + 0.5 * F[0]) / rho[i];
    v[1] = (jy + 0.5 * F[1]) / rho[i];
}

/* Relaxation rate of the shear moments: tau_nu = nu / c_s^2 + 1/2, with the kinematic viscosity
 * interpolated linearly in the phase fraction (rho - rho_v)/(rho_l - rho_v), clamped to [0, 1]. */
static double s_nu_of(const orc_params *p, double rho)
{
    double nu_l = (p->tau_l - 0.5) / 3.0, nu_v = (p->tau_v - 0.5) / 3.0;
    double phi = (rho - p->rho_v) / (p->rho_l - p->rho_v);
    if (phi < 0.0) phi = 0.0;
    if (phi > 1.0) phi = 1.0;
    double nu = nu_v + phi * (nu_l - nu_v);
    return 1.0 / (3.0 * nu + 0.5);
}

/* S6, S7 at one node: m = M f, Eq. (3) equilibria, Eq. (9) forcing, Eq. (4) relaxation,
 * f* = M^-1 m*. M^-1 = M^T diag(1 / |row_k|^2) because the rows of M are orthogonal. */
static void collide_at(const orc_params *p, const double fin[9], double rho, double psi,
                       const double Fm[2], const double F[2], const double v[2], double fout[9])
{
    double m[9], meq[9], S[9], ms[9], s[9];
    for (int k = 0; k < 9; ++k) {
        m[k] = 0.0;
        for (int a = 0; a < 9; ++a) m[k] += MM[k][a] * fin[a];
    }
    const double vx = v[0], vy = v[1], v2 = vx * vx + vy * vy;
    /* Eq. (3) */
    meq[0] = rho;
    meq[1] = rho * (-2.0 + 3.0 * v2);
    meq[2] = rho * (1.0 - 3.0 * v2);
    meq[3] = rho * vx;
    meq[4] = -rho * vx;
    meq[5] = rho * vy;
    meq[6] = -rho * vy;
    meq[7] = rho * (vx * vx - vy * vy);
    meq[8] = rho * vx * vy;
    /* Eq. (2) */
    const double snu = s_nu_of(p, rho);
    s[0] = p->s_rho; s[1] = p->s_e; s[2] = p->s_zeta; s[3] = p->s_j; s[4] = p->s_q;
    s[5] = p->s_j; s[6] = p->s_q; s[7] = snu; s[8] = snu;
    /* Eq. (9), delta_t = 1, tau_e = 1/s_e, tau_zeta = 1/s_zeta */
    const double tau_e = 1.0 / p->s_e, tau_z = 1.0 / p->s_zeta;
    const double Fm2 = Fm[0] * Fm[0] + Fm[1] * Fm[1];
    const double vF = vx * F[0] + vy * F[1];
    S[0] = 0.0;
    S[1] = 6.0 * vF + 12.0 * p->sigma * Fm2 / (psi * psi * (tau_e - 0.5));
    S[2] = -6.0 * vF - 12.0 * p->sigma * Fm2 / (psi * psi * (tau_z - 0.5));
    S[3] = F[0];
    S[4] = -F[0];
    S[5] = F[1];
    S[6] = -F[1];
    S[7] = 2.0 * (vx * F[0] - vy * F[1]);
    S[8] = vx * F[1] + vy * F[0];
    /* Eq. (4) */
    for (int k = 0; k < 9; ++k) ms[k] = m[k] - s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * s[k]) * S[k];
    double n2[9];
    for (int k = 0; k < 9; ++k) {
        n2[k] = 0.0;
        for (int j = 0; j < 9; ++j) n2[k] += MM[k][j] * MM[k][j];
    }
    for (int a = 0; a < 9; ++a) {
        double acc = 0.0;
        for (int k = 0; k < 9; ++k) acc += MM[k][a] * ms[k] / n2[k];
        fout[a] = acc;
    }
}

/* Non-slip wet-node boundary of Sec. III.A at a node of the bottom wall plane (unknowns f2, f5,
 * f6 arrive from the solid) or, rotated by 180 degrees, of the top wall plane (unknowns f4, f7,
 * f8). fn: the node's post-streaming populations with the known ones filled in; F: the total
 * force of the step just taken at this node. The reconstruction makes sum_a e_a f_a + F/2 = 0. */
static void wet_node(int bottom, const double F[2], double fn[9])
{
    const double d13 = fn[1] - fn[3];
    if (bottom) {
        fn[2] = fn[4];
        fn[5] = fn[7] - 0.5 * d13 - 0.25 * (F[0] + F[1]);
        fn[6] = fn[8] + 0.5 * d13 + 0.25 * (F[0] - F[1]);
    } else {
        fn[4] = fn[2];
        fn[7] = fn[5] + 0.5 * d13 + 0.25 * (F[0] + F[1]);
        fn[8] = fn[6] - 0.5 * d13 - 0.25 * (F[0] - F[1]);
    }
}

/* One full time step, f^n -> f^{n+1}, in place. work: 13 * nx * ny doubles (rho, psi, f*, F). */
static int one_step(const orc_params *p, const double *gw, double *f, double *work)
{
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    double *rho = work, *psi = work + N, *fs = work + 2 * N, *Ft = work + 11 * N;
    int rc = density_and_psi(p, f, rho, psi);
    if (rc) return rc;

#pragma omp parallel for
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            if (is_solid(p, x, y)) {
                for (int a = 0; a < 9; ++a) fs[a * N + i] = 0.0;
                continue;
            }
            double Fm[2], Fads[2], F[2], v[2], fin[9], fo[9];
            forces_at(p, gw, f, rho, psi, x, y, Fm, Fads, F, v);
            for (int a = 0; a < 9; ++a) fin[a] = f[a * N + i];
            collide_at(p, fin, rho[i], psi[i], Fm, F, v, fo);
            for (int a = 0; a < 9; ++a) fs[a * N + i] = fo[a];
            Ft[i] = F[0];
            Ft[N + i] = F[1];
        }
    }

    /* S8, Eq. (5): f_a(x, t+1) = f*_a(x - e_a) when x - e_a is fluid. Otherwise, with halfway
     * bounce-back, the population reflected at the wall, f*_opp(a)(x); with the wet-node scheme
     * the populations from the solid are reconstructed from the streamed ones (wet_node). */
#pragma omp parallel for
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            if (is_solid(p, x, y)) {
                for (int a = 0; a < 9; ++a) f[a * N + i] = 0.0;
                continue;
            }
            double fn[9];
            for (int a = 0; a < 9; ++a) {
                int xs = wrap(x - EX[a], nx);
                int ys = nb_row(p, y - EY[a]);
                if (is_solid(p, xs, ys)) fn[a] = p->walls == 2 ? 0.0 : fs[OPP[a] * N + i];
                else fn[a] = fs[a * N + (size_t)ys * nx + xs];
            }
            if (p->walls == 2 && (y == 1 || y == ny - 2)) {
                const double F[2] = {Ft[i], Ft[N + i]};
                if (y == 1) wet_node(1, F, fn);
                if (y == ny - 2) wet_node(0, F, fn);
            }
            for (int a = 0; a < 9; ++a) f[a * N + i] = fn[a];
        }
    }
    return ORC_OK;
}

static int check(const orc_params *p)
{
    if (!p || p->nx < 3 || p->walls < 0 || p->walls > 3) return ORC_E_INVAL;
    if (p->ny < ((p->walls == 1 || p->walls == 2) ? 4 : 3)) return ORC_E_INVAL;
    if (p->walls == 3 && (!p->solid || p->ghost)) return ORC_E_INVAL;
    return ORC_OK;
}

/* Advance f by nsteps steps. */
int orc_run(const orc_params *p, const double *gw, double *f, int64_t nsteps)
{
    int rc = check(p);
    if (rc) return rc;
    const size_t N = (size_t)p->nx * p->ny;
    double *work = (double *)malloc(13 * N * sizeof(double));
    if (!work) return ORC_E_NOMEM;
    for (int64_t n = 0; n < nsteps && rc == ORC_OK; ++n) rc = one_step(p, gw, f, work);
    free(work);
    return rc;
}

/* Rest-state equilibrium f_a = t_a rho with t = 4/9, 1/9, 1/36 (solid rows get 0). */
int orc_init_rest(const orc_params *p, const double *rho0, double *f)
{
    int rc = check(p);
    if (rc) return rc;
    const size_t N = (size_t)p->nx * p->ny;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            size_t i = (size_t)y * p->nx + x;
            for (int a = 0; a < 9; ++a) {
                int e2 = EX[a] * EX[a] + EY[a] * EY[a];
                double t = e2 == 0 ? 4.0 / 9.0 : (e2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
                f[a * N + i] = is_solid(p, x, y) ? 0.0 : t * rho0[i];
            }
        }
    return ORC_OK;
}

/* Macroscopic fields of state f (S1-S5 without collision): rho, psi (with ghost rows), F_m,
 * F_ads and v per node. Solid nodes get rho = 0 and zero force and velocity. */
int orc_fields(const orc_params *p, const double *gw, const double *f, double *rho,
               double *psi, double *Fm_out, double *Fads_out, double *v_out)
{
    int rc = check(p);
    if (rc) return rc;
    const int nx = p->nx, ny = p->ny;
    const size_t N = (size_t)nx * ny;
    rc = density_and_psi(p, f, rho, psi);
    if (rc) return rc;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            double Fm[2] = {0, 0}, Fads[2] = {0, 0}, F[2], v[2] = {0, 0};
            if (!is_solid(p, x, y)) forces_at(p, gw, f, rho, psi, x, y, Fm, Fads, F, v);
            Fm_out[i] = Fm[0]; Fm_out[N + i] = Fm[1];
            Fads_out[i] = Fads[0]; Fads_out[N + i] = Fads[1];
            v_out[i] = v[0]; v_out[N + i] = v[1];
        }
    return ORC_OK;
}

/* One collision at a single node from given inputs (for tests of Eqs. 3, 4, 9 in isolation). */
void orc_collide_node(const orc_params *p, const double fin[9], double psi, const double Fm[2],
                      const double F[2], double fout[9])
{
    double rho = 0.0, jx = 0.0, jy = 0.0, v[2];
    for (int a = 0; a < 9; ++a) { rho += fin[a]; jx += EX[a] * fin[a]; jy += EY[a] * fin[a]; }
    v[0] = (jx + 0.5 * F[0]) / rho;
    v[1] = (jy + 0.5 * F[1]) / rho;
    collide_at(p, fin, rho, psi, Fm, F, v, fout);
}
