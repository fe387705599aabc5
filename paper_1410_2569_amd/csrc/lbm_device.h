// lbm_device.h -- per-node device arithmetic of the wetting pseudopotential LB step (gfx950, FP64).
//
// State layout in HBM: two ping-pong buffers g[2], each 9 population planes of ny rows x pitch
// doubles (x fastest, pitch a multiple of 32 doubles so every row starts on a 256-byte boundary).
// A buffer holds POST-collision populations f*; the pre-collision f^n of a node is pulled from its
// neighbours (streaming, Eq. 5). Rows 0 and ny-1 are solid when walls != 0. Where x - e_a is a
// solid node the population is, with walls = 1, the halfway bounce-back f_a(x) = f*_opp(a)(x);
// with walls = 2 (the non-slip wet-node scheme of Sec. III.A) rows 1 and ny-2 are boundary nodes
// on the wall planes and the populations arriving from the solid are reconstructed from the
// streamed ones and the node's force of the step that wrote the buffer. That force (Fx, Fy) is
// part of the state: planes 0 and 1 of the adjacent solid row hold it, slots no pull reads
// otherwise. With walls = 3 the lattice is periodic in x and y and a solid mask defines the solid
// nodes: links[y][x] bit 0 marks node (x, y) solid and bit a marks x - e_a solid (halfway
// bounce-back on that link); psi is 0 on solid nodes and G_w is given per solid node (gwn).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Kernel-side parameters, computed once on the host (lbm_api.cpp) from lbm_params.
struct KParams {
    int nx, ny, pitch;      // lattice and row pitch (doubles)
    int walls, ghost;       // solid rows 0 and ny-1 (1 bounce-back, 2 wet-node); mirrored psi
    int wet;                // walls == 2
    int mask;               // walls == 3: solid nodes from links, G_w per node in gwn
    int eos, wall_force;    // 0 CS / 1 piecewise; 0 rho / 1 psi / 2 psi^2 pre-sum factor
    int y_lo, y_hi;         // fluid rows [y_lo, y_hi]
    int visc_const;         // 1: tau_l == tau_v, use s_nu_c
    long long plane;        // doubles between consecutive population planes
    // equation of state
    double RT, a, b4;       // Carnahan-Starling: R T, a, b/4
    double rho1, rho2, th_v, th_m, th_l, p1, p2;  // Eq. (15) with p1 = p(rho1), p2 = p(rho2)
    double two_over_G;      // 2/G in psi = sqrt(2 (p - rho/3)/G)
    double negG;            // -G of Eq. (7)
    double c_sig_e, c_sig_z;  // 12 sigma G^2 / (tau - 1/2) for the e and epsilon rows of Eq. (9)
    double s_e, s_z, s_j, s_q;            // relaxation rates (s_rho drops out: rho is conserved)
    double h_e, h_z, h_j, h_q;            // 1 - s/2
    double s_nu_c, nu_v, dnu, rho_v, inv_drho;  // shear rate: constant, or interpolated
    double rho_mid;               // (rho_l + rho_v) / 2, the interface level of the observables
    const unsigned short* links;  // walls = 3: [ny][pitch] solid and bounce-back bits
    const double* gwn;            // walls = 3: [ny][pitch] G_w of solid nodes
};

// Geometry variants compiled into the step kernels. GEO_ROWS: periodic lattice or bounce-back
// rows; GEO_WET: also the wet-node rule where P.wet says so; GEO_MASK: solid mask.
enum { GEO_ROWS = 0, GEO_WET = 1, GEO_MASK = 2 };
// Equation-of-state variants compiled into the step kernels: one EOS only, or the run-time choice
// of P.eos (off the step loop, and ensembles that mix both).
enum { EOS_CS = 0, EOS_PW = 1, EOS_ANY = 2 };

__device__ __forceinline__ int wrap_once(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// x mod nx in [0, nx). Tile halos reach at most a few nodes past either end, so one add or
// subtract suffices except on lattices narrower than a tile.
__device__ __forceinline__ int wrapx(int x, int nx) {
    int r = x < 0 ? x + nx : (x >= nx ? x - nx : x);
    if ((unsigned)r >= (unsigned)nx) {
        r = x % nx;
        r = r < 0 ? r + nx : r;
    }
    return r;
}

// Floating-point contraction is switched off inside the per-node arithmetic and the multiply-adds
// are written as explicit fma(): the rounding of every result is then fixed by the source alone,
// so every kernel that inlines these functions (plain step, every tile shape, ensembles,
// persistent loop, adjoint recomputation) produces the same bits. The reverse-mode functions
// further down follow the same rule, so that every reverse-step tile (interior or not, of any
// shape, single lattice or ensemble) gives the same gradient bits.

// p_EOS(rho) and psi(rho); a negative radicand yields NaN, caught by the observables. EOS selects
// the equation of state compiled in (EOS_ANY: P.eos at run time).
template <int EOS = EOS_ANY>
__device__ __forceinline__ double psi_of_rho(const KParams& P, double rho) {
#pragma clang fp contract(off)
    double p;
    if (EOS == EOS_CS || (EOS == EOS_ANY && P.eos == 0)) {
        const double eta = P.b4 * rho;
        const double om = 1.0 - eta;
        const double num = fma(eta, fma(eta, om, 1.0), 1.0);  // 1 + eta + eta^2 - eta^3
        p = fma(-P.a * rho, rho, (rho * P.RT) * num / (om * om * om));
    } else {
        p = rho <= P.rho1 ? rho * P.th_v
          : (rho <= P.rho2 ? fma(rho - P.rho1, P.th_m, P.p1) : fma(rho - P.rho2, P.th_l, P.p2));
    }
    return sqrt(P.two_over_G * (p - rho * (1.0 / 3.0)));
}

// Non-slip wet-node boundary (Sec. III.A) at a boundary node of the bottom wall plane: the
// populations arriving from the solid (2, 5, 6) follow from the streamed ones and the node's
// force (Fx, Fy) so that sum_a e_a f_a + F/2 = 0. The top wall plane is the same rule rotated by
// 180 degrees (unknowns 4, 7, 8).
__device__ __forceinline__ void wet_node_bottom(double f[9], double Fx, double Fy) {
#pragma clang fp contract(off)
    const double d13 = f[1] - f[3];
    f[2] = f[4];
    f[5] = f[7] - 0.5 * d13 - 0.25 * (Fx + Fy);
    f[6] = f[8] + 0.5 * d13 + 0.25 * (Fx - Fy);
}

__device__ __forceinline__ void wet_node_top(double f[9], double Fx, double Fy) {
#pragma clang fp contract(off)
    const double d13 = f[1] - f[3];
    f[4] = f[2];
    f[7] = f[5] + 0.5 * d13 + 0.25 * (Fx + Fy);
    f[8] = f[6] - 0.5 * d13 - 0.25 * (Fx - Fy);
}

// Pull the 9 pre-collision populations of fluid node (x, y) from post-collision buffer g.
// Plane bases are uniform (scalar registers) and in-plane offsets 32-bit unsigned, so loads use
// scalar-base + 32-bit vector-offset addressing. GEO selects the geometry code compiled in (see
// GEO_ROWS, GEO_WET, GEO_MASK).
template <int GEO>
__device__ __forceinline__ void pull9(const KParams& P, const double* __restrict__ g, int x,
                                      int y, double f[9]);

// Solid-mask geometry: lk = links of (x, y); a set bit a pulls the node's own reflected
// population (halfway bounce-back), otherwise the neighbour's, with x and y periodic.
__device__ __forceinline__ void pull9_mask(const KParams& P, const double* __restrict__ g, int x,
                                           int y, unsigned lk, double f[9]) {
    const unsigned pitch = P.pitch;
    const unsigned xm = x == 0 ? P.nx - 1 : x - 1, xp = x == P.nx - 1 ? 0 : x + 1;
    const unsigned ym = y == 0 ? P.ny - 1 : y - 1, yp = y == P.ny - 1 ? 0 : y + 1;
    const long long pl = P.plane;
    const unsigned r0 = (unsigned)y * pitch, rm = ym * pitch, rp = yp * pitch, i0 = r0 + x;
    f[0] = g[i0];
    f[1] = (lk & 2u) ? (g + 3 * pl)[i0] : (g + 1 * pl)[r0 + xm];
    f[2] = (lk & 4u) ? (g + 4 * pl)[i0] : (g + 2 * pl)[rm + x];
    f[3] = (lk & 8u) ? (g + 1 * pl)[i0] : (g + 3 * pl)[r0 + xp];
    f[4] = (lk & 16u) ? (g + 2 * pl)[i0] : (g + 4 * pl)[rp + x];
    f[5] = (lk & 32u) ? (g + 7 * pl)[i0] : (g + 5 * pl)[rm + xm];
    f[6] = (lk & 64u) ? (g + 8 * pl)[i0] : (g + 6 * pl)[rm + xp];
    f[7] = (lk & 128u) ? (g + 5 * pl)[i0] : (g + 7 * pl)[rp + xp];
    f[8] = (lk & 256u) ? (g + 6 * pl)[i0] : (g + 8 * pl)[rp + xm];
}

template <int GEO>
__device__ __forceinline__ void pull9(const KParams& P, const double* __restrict__ g, int x,
                                      int y, double f[9]) {
    if constexpr (GEO == GEO_MASK) {
        pull9_mask(P, g, x, y, P.links[(unsigned)y * P.pitch + x], f);
        return;
    }
    const unsigned nx = P.nx, pitch = P.pitch;
    const unsigned ux = x;
    const unsigned xm = ux == 0 ? nx - 1 : ux - 1;
    const unsigned xp = ux == nx - 1 ? 0 : ux + 1;
    unsigned ym, yp;
    bool bot, top;
    if (P.walls) {
        ym = y - 1; yp = y + 1;
        bot = (y == 1); top = (y == P.ny - 2);
    } else {
        ym = y == 0 ? P.ny - 1 : y - 1;
        yp = y == P.ny - 1 ? 0 : y + 1;
        bot = top = false;
    }
    const long long pl = P.plane;
    const unsigned r0 = (unsigned)y * pitch, rm = ym * pitch, rp = yp * pitch;
    f[0] = g[r0 + ux];
    f[1] = (g + 1 * pl)[r0 + xm];
    f[3] = (g + 3 * pl)[r0 + xp];
    // populations arriving from below (e_y = +1): reflected at the bottom wall
    f[2] = bot ? (g + 4 * pl)[r0 + ux] : (g + 2 * pl)[rm + ux];
    f[5] = bot ? (g + 7 * pl)[r0 + ux] : (g + 5 * pl)[rm + xm];
    f[6] = bot ? (g + 8 * pl)[r0 + ux] : (g + 6 * pl)[rm + xp];
    // populations arriving from above (e_y = -1): reflected at the top wall
    f[4] = top ? (g + 2 * pl)[r0 + ux] : (g + 4 * pl)[rp + ux];
    f[7] = top ? (g + 5 * pl)[r0 + ux] : (g + 7 * pl)[rp + xp];
    f[8] = top ? (g + 6 * pl)[r0 + ux] : (g + 8 * pl)[rp + xm];
    if (GEO == GEO_WET && P.wet && (bot || top)) {
        // the slots read above for the unknown populations are overwritten by the reconstruction
        if (bot) wet_node_bottom(f, g[rm + ux], (g + pl)[rm + ux]);
        if (top) wet_node_top(f, g[rp + ux], (g + pl)[rp + ux]);
    }
}

// Any geometry, dispatched at run time (for kernels off the time-step loop).
__device__ __forceinline__ void pull9_any(const KParams& P, const double* __restrict__ g, int x,
                                          int y, double f[9]) {
    if (P.mask) pull9<GEO_MASK>(P, g, x, y, f);
    else pull9<GEO_WET>(P, g, x, y, f);
}

__device__ __forceinline__ bool is_solid_node(const KParams& P, int x, int y) {
    return P.mask && (P.links[(unsigned)y * P.pitch + x] & 1u);
}

// The fluid node whose psi a lattice slot (gx, gy) holds: gx wraps (periodic x); a solid row
// takes the adjacent fluid row (mirrored ghost psi) or nothing (psi = 0); rows outside the
// lattice hold nothing; with a solid mask both coordinates wrap and solid nodes hold nothing.
// Returns false when the slot's psi is 0.
__device__ __forceinline__ bool slot_source(const KParams& P, int gx, int gy, int& sx, int& sy) {
    sx = wrapx(gx, P.nx);
    if (P.mask) {
        sy = wrapx(gy, P.ny);
        return (P.links[(unsigned)sy * P.pitch + sx] & 1u) == 0;
    }
    if (P.walls) {
        if (gy < 0 || gy > P.ny - 1) return false;
        if (gy == 0) { sy = 1; return P.ghost != 0; }
        if (gy == P.ny - 1) { sy = P.ny - 2; return P.ghost != 0; }
        sy = gy;
        return true;
    }
    sy = wrapx(gy, P.ny);
    return true;
}

// psi at lattice position (gx, gy) (see slot_source), evaluated from the pulled populations.
template <int GEO, int EOS = EOS_ANY>
__device__ __forceinline__ double psi_at(const KParams& P, const double* __restrict__ g, int gx,
                                         int gy) {
#pragma clang fp contract(off)
    int sx, sy;
    if (!slot_source(P, gx, gy, sx, sy)) return 0.0;
    double f[9];
    pull9<GEO>(P, g, sx, sy, f);
    return psi_of_rho<EOS>(P, ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) +
                                  f[8]);
}

// The pull behind lattice slot (gx, gy) (slot_source; IN: a fluid node reached without wrap)
// into f, without evaluating psi. Returns false when the slot's psi is 0 (nothing pulled);
// fluid: the slot is a fluid node of the lattice (not a ghost row).
template <int GEO, bool IN>
__device__ __forceinline__ bool pull_slot(const KParams& P, const double* __restrict__ g, int gx,
                                          int gy, double f[9], bool& fluid);

__device__ __forceinline__ double sum9(const double f[9]) {
#pragma clang fp contract(off)
    return ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
}

// Adhesion sum A = sum over solid neighbours of omega_a G_w(x + e_a) e_a (omega = w/3) at a fluid
// node next to a flat wall; F_ads = -P A with P = rho, psi or psi^2 (Eqs. 10, 11, 14).
__device__ __forceinline__ void adhesion_sum(const KParams& P, const double* __restrict__ gw,
                                             int x, int y, double& Ax, double& Ay) {
#pragma clang fp contract(off)
    Ax = 0.0; Ay = 0.0;
    if (!P.walls || P.mask) return;
    const int xm = x == 0 ? P.nx - 1 : x - 1;
    const int xp = x == P.nx - 1 ? 0 : x + 1;
    if (y == 1) {  // bottom wall below: e4 (0,-1) w 1/9, e7 (-1,-1) and e8 (1,-1) w 1/36
        const double gc = gw[x], gm = gw[xm], gp = gw[xp];
        Ax += (gp - gm) * (1.0 / 36.0);
        Ay -= fma(gc, 1.0 / 9.0, (gm + gp) * (1.0 / 36.0));
    }
    if (y == P.ny - 2) {  // top wall above: e2 (0,1), e5 (1,1), e6 (-1,1)
        const double* gt = gw + P.pitch;  // rows of the G_w array are pitch apart
        const double gc = gt[x], gm = gt[xm], gp = gt[xp];
        Ax += (gp - gm) * (1.0 / 36.0);
        Ay += fma(gc, 1.0 / 9.0, (gm + gp) * (1.0 / 36.0));
    }
}

// Adhesion sum over the solid neighbours of a solid-mask geometry (lk: links of the node; bit
// opp(a) marks x + e_a solid), in the order a = 1..8.
__device__ __forceinline__ void adhesion_mask(const KParams& P, int x, int y, unsigned lk,
                                              double& Ax, double& Ay) {
#pragma clang fp contract(off)
    Ax = 0.0; Ay = 0.0;
    if ((lk & 0x1FEu) == 0) return;
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const int op[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        if (!((lk >> op[a]) & 1u)) continue;
        const int xs = wrap_once(x + ex[a], P.nx), ys = wrap_once(y + ey[a], P.ny);
        const double om = (a < 5 ? 1.0 / 3.0 : 1.0 / 12.0) * (1.0 / 3.0);
        const double g = P.gwn[(unsigned)ys * P.pitch + xs];
        Ax = fma(om * g, (double)ex[a], Ax);
        Ay = fma(om * g, (double)ey[a], Ay);
    }
}

// Cohesion stencil sum s = sum_a w_a psi(x + e_a) e_a from the 3x3 neighbourhood
// p[dy][dx] (dy, dx in 0..2 for offsets -1..1).
__device__ __forceinline__ void cohesion_sum(double pmm, double p0m, double ppm, double pm0,
                                             double pp0, double pmp, double p0p, double ppp,
                                             double& sx, double& sy) {
#pragma clang fp contract(off)
    // axial w = 1/3, diagonal w = 1/12 (Eq. 7)
    const double dpx = ppp - pmm, dmx = ppm - pmp;  // (+1,+1)-(-1,-1), (+1,-1)-(-1,+1)
    sx = fma(pp0 - pm0, 1.0 / 3.0, (dpx + dmx) * (1.0 / 12.0));
    sy = fma(p0p - p0m, 1.0 / 3.0, (dpx - dmx) * (1.0 / 12.0));
}

// Total force F = F_m + F_ads of one node (Eqs. 7, 10, 11, 14).
__device__ __forceinline__ void total_force(const KParams& P, double rho, double psi_c, double sx,
                                            double sy, double Ax, double Ay, double& Fx,
                                            double& Fy) {
#pragma clang fp contract(off)
    const double pre = P.wall_force == 0 ? rho : (P.wall_force == 1 ? psi_c : psi_c * psi_c);
    Fx = fma(-pre, Ax, P.negG * psi_c * sx);
    Fy = fma(-pre, Ay, P.negG * psi_c * sy);
}

// With the wet-node scheme, a boundary node stores its force of this step in planes 0 and 1 of
// the adjacent solid row of the output buffer (o: the output slot of the node, plane stride pl,
// row stride W). Other nodes store nothing.
template <int GEO>
__device__ __forceinline__ void store_wall_force(const KParams& P, double* out, long long o,
                                                 long long pl, long long W, int y, double rho,
                                                 double psi_c, double sx, double sy, double Ax,
                                                 double Ay) {
    if (GEO != GEO_WET || !P.wet || (y != 1 && y != P.ny - 2)) return;
    double Fx, Fy;
    total_force(P, rho, psi_c, sx, sy, Ax, Ay, Fx, Fy);
    if (y == 1) { out[o - W] = Fx; out[pl + o - W] = Fy; }
    if (y == P.ny - 2) { out[o + W] = Fx; out[pl + o + W] = Fy; }
}

// Forces, velocity and MRT collision of one node (Eqs. 2-4, 6, 7, 9 and 10/11/14):
// in f[9] (pre-collision), rho, psi_c, cohesion sum (sx, sy), adhesion sum (Ax, Ay);
// out f[9] overwritten with f* = M^-1 m*.
__device__ __forceinline__ void collide(const KParams& P, double f[9], double rho, double psi_c,
                                        double sx, double sy, double Ax, double Ay) {
#pragma clang fp contract(off)
    // Eq. (7) cohesion plus the adhesion of Eq. (10)/(11)/(14)
    double Fx, Fy;
    total_force(P, rho, psi_c, sx, sy, Ax, Ay, Fx, Fy);

    // moments m = M f (rows rho, e, epsilon, jx, qx, jy, qy, pxx, pxy)
    const double ax = f[1] + f[3], ay = f[2] + f[4];
    const double sa = ax + ay;                       // axial sum
    const double s57 = f[5] + f[7], s68 = f[6] + f[8];
    const double sd = s57 + s68;                     // diagonal sum
    const double f04 = 4.0 * f[0];
    const double m1 = fma(2.0, sd, -(f04 + sa));
    const double m2 = fma(-2.0, sa, f04 + sd);
    const double d13 = f[1] - f[3], d24 = f[2] - f[4];
    const double d58 = f[5] - f[7], d68 = f[6] - f[8];
    const double ex = d58 - d68, ey = d58 + d68;
    const double jx = d13 + ex, jy = d24 + ey;
    const double m4 = fma(-2.0, d13, ex);
    const double m6 = fma(-2.0, d24, ey);
    const double m7 = ax - ay;
    const double m8 = s57 - s68;

    // Eq. (6): velocity with half the force
    const double ir = 1.0 / rho;
    const double vx = fma(0.5, Fx, jx) * ir, vy = fma(0.5, Fy, jy) * ir;
    const double v2 = fma(vx, vx, vy * vy);

    // shear relaxation rate from the phase-interpolated viscosity
    double snu;
    if (P.visc_const) {
        snu = P.s_nu_c;
    } else {
        double phi = (rho - P.rho_v) * P.inv_drho;
        phi = fmin(fmax(phi, 0.0), 1.0);
        snu = 1.0 / fma(3.0, fma(phi, P.dnu, P.nu_v), 0.5);
    }
    const double hnu = 1.0 - 0.5 * snu;

    // Eq. (9) forcing; |F_m|^2 / psi^2 = G^2 |s|^2
    const double vF = fma(vx, Fx, vy * Fy);
    const double s2 = fma(sx, sx, sy * sy);
    const double S1 = fma(P.c_sig_e, s2, 6.0 * vF);
    const double S2 = fma(-P.c_sig_z, s2, -6.0 * vF);
    const double S7 = 2.0 * fma(vx, Fx, -(vy * Fy));
    const double S8 = fma(vx, Fy, vy * Fx);

    // Eq. (4) with Eq. (3) equilibria; m*_0 = rho
    const double ms1 = fma(P.h_e, S1, fma(-P.s_e, m1 - rho * fma(3.0, v2, -2.0), m1));
    const double ms2 = fma(P.h_z, S2, fma(-P.s_z, m2 - rho * fma(-3.0, v2, 1.0), m2));
    // momentum rows: j - s_j (j - rho v) + (1 - s_j/2) F with rho v = j + F/2 is j + F
    const double ms3 = jx + Fx;
    const double ms4 = fma(-P.h_q, Fx, fma(-P.s_q, fma(rho, vx, m4), m4));
    const double ms5 = jy + Fy;
    const double ms6 = fma(-P.h_q, Fy, fma(-P.s_q, fma(rho, vy, m6), m6));
    const double ms7 = fma(hnu, S7, fma(-snu, fma(-rho, fma(vx, vx, -(vy * vy)), m7), m7));
    const double ms8 = fma(hnu, S8, fma(-snu, fma(-rho, vx * vy, m8), m8));

    // f* = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m*
    const double a0 = rho * (1.0 / 9.0), a1 = ms1 * (1.0 / 36.0), a2 = ms2 * (1.0 / 36.0);
    const double a3 = ms3 * (1.0 / 6.0), a4 = ms4 * (1.0 / 12.0);
    const double a5 = ms5 * (1.0 / 6.0), a6 = ms6 * (1.0 / 12.0);
    const double a7 = ms7 * 0.25, a8 = ms8 * 0.25;
    const double ba = fma(-2.0, a2, a0 - a1), bd = fma(2.0, a1, a0 + a2);
    f[0] = fma(4.0, a2 - a1, a0);
    const double tx = ba + a7, ux = fma(-2.0, a4, a3);  // axial x: ba + a7 +- (a3 - 2 a4)
    const double ty = ba - a7, uy = fma(-2.0, a6, a5);  // axial y: ba - a7 +- (a5 - 2 a6)
    f[1] = tx + ux;
    f[3] = tx - ux;
    f[2] = ty + uy;
    f[4] = ty - uy;
    const double X = a3 + a4, Y = a5 + a6;
    const double sp = X + Y, sm = Y - X;  // diagonals: bd +- a8 +- (X + Y) or (Y - X)
    const double bp = bd + a8, bm = bd - a8;
    f[5] = bp + sp;
    f[7] = bp - sp;
    f[6] = bm + sm;
    f[8] = bm - sm;
}

// Macroscopic velocity of a node (Eq. 6) with the same force as collide().
__device__ __forceinline__ void velocity(const KParams& P, const double f[9], double rho,
                                         double psi_c, double sx, double sy, double Ax,
                                         double Ay, double& vx, double& vy) {
#pragma clang fp contract(off)
    double Fx, Fy;
    total_force(P, rho, psi_c, sx, sy, Ax, Ay, Fx, Fy);
    const double d58 = f[5] - f[7], d68 = f[6] - f[8];
    const double jx = (f[1] - f[3]) + d58 - d68;
    const double jy = (f[2] - f[4]) + d58 + d68;
    const double ir = 1.0 / rho;
    vx = fma(0.5, Fx, jx) * ir;
    vy = fma(0.5, Fy, jy) * ir;
}

// The 9 pre-collision populations of node (x, y): pulled from a post-collision buffer (the
// library's state), or with PRE read in place from an array of pre-collision populations of the
// same [9][ny][pitch] layout.
template <bool PRE>
__device__ __forceinline__ void node_populations(const KParams& P, const double* __restrict__ g,
                                                 int x, int y, double f[9]) {
    if constexpr (PRE) {
        const long long i = (long long)y * P.pitch + x;
#pragma unroll
        for (int a = 0; a < 9; ++a) f[a] = g[a * P.plane + i];
    } else {
        pull9_any(P, g, x, y, f);
    }
}

// Density and pseudopotential of node (x, y) (x < nx, y_lo <= y <= y_hi) into psi_g and, when
// given, rho_out (fields of [ny][pitch] doubles); a solid node of a mask gets 0 in both. With
// ghost rows (Eq. 7 applied at the wall) the solid row next to the node's row receives its psi.
template <bool PRE = false>
__device__ __forceinline__ void psi_node(const KParams& P, const double* __restrict__ gin,
                                         double* __restrict__ psi_g, double* __restrict__ rho_out,
                                         int x, int y) {
    if (is_solid_node(P, x, y)) {
        psi_g[(long long)y * P.pitch + x] = 0.0;
        if (rho_out) rho_out[(long long)y * P.pitch + x] = 0.0;
        return;
    }
    double f[9];
    node_populations<PRE>(P, gin, x, y, f);
    const double rho = sum9(f);
    const double ps = psi_of_rho(P, rho);
    psi_g[(long long)y * P.pitch + x] = ps;
    if (rho_out) rho_out[(long long)y * P.pitch + x] = rho;
    if (P.walls && !P.mask && P.ghost) {
        if (y == 1) psi_g[x] = ps;
        if (y == P.ny - 2) psi_g[(long long)(P.ny - 1) * P.pitch + x] = ps;
    }
}

// Arguments of the observables: contour level, fit window and centring of the sums.
struct ObsArgs {
    double rho_mid;     // (rho_l + rho_v) / 2
    double y_min;       // interface points below this height are not fitted
    double x_lo, x_hi;  // fit window
    double cx, cy;      // coordinates are accumulated relative to this point
};

// Partial quantities of the observables: density extremes, velocity maxima, mass, non-finite
// count, and the sums of the Kasa circle fit over interface points.
enum { O_MIN = 0, O_MAX, O_U, O_UL, O_MASS, O_BAD, O_N, O_SX, O_SY, O_SXX, O_SYY, O_SXY, O_SXR,
       O_SYR, O_SR, O_NQ };

__device__ __forceinline__ double op_combine(int q, double a, double b) {
    if (q == O_MIN) return fmin(a, b);
    if (q == O_MAX || q == O_U || q == O_UL) return fmax(a, b);
    return a + b;
}

__device__ __forceinline__ double op_identity(int q) {
    if (q == O_MIN) return __builtin_huge_val();
    if (q == O_MAX || q == O_U || q == O_UL) return -__builtin_huge_val();
    return 0.0;
}

__device__ __forceinline__ void add_point(double v[O_NQ], double px, double py, double cx,
                                          double cy) {
    const double X = px - cx, Y = py - cy, r2 = X * X + Y * Y;
    v[O_N] += 1.0; v[O_SX] += X; v[O_SY] += Y; v[O_SXX] += X * X; v[O_SYY] += Y * Y;
    v[O_SXY] += X * Y; v[O_SXR] += X * r2; v[O_SYR] += Y * r2; v[O_SR] += r2;
}

// Observables contribution of node (x, y) (x < nx, y_lo <= y <= y_hi) to v[O_NQ]: its density,
// velocity of Eq. (6) (forces from psi_g, the psi field with its ghost rows), and the rho_mid
// crossings on the edges to its right and upper neighbours. rho_f: density of every fluid node.
// Solid nodes of a mask contribute nothing. PRE: gin holds pre-collision populations (see
// node_populations).
template <bool PRE = false>
__device__ __forceinline__ void obs_node(const KParams& P, const double* __restrict__ gin,
                                         const double* __restrict__ rho_f,
                                         const double* __restrict__ psi_g,
                                         const double* __restrict__ gw, const ObsArgs& A, int x,
                                         int y, double v[O_NQ]) {
    if (is_solid_node(P, x, y)) return;
    const long long i = (long long)y * P.pitch + x;
    double f[9];
    node_populations<PRE>(P, gin, x, y, f);
    const double rho = rho_f[i], pc = psi_g[i];
    const int xm = x == 0 ? P.nx - 1 : x - 1, xp = x == P.nx - 1 ? 0 : x + 1;
    int ym = y - 1, yp = y + 1;
    if (!P.walls || P.mask) { ym = wrapx(ym, P.ny); yp = wrapx(yp, P.ny); }
    const double* rm = psi_g + (long long)ym * P.pitch;
    const double* r0 = psi_g + (long long)y * P.pitch;
    const double* rp = psi_g + (long long)yp * P.pitch;
    double sx, sy, Ax = 0.0, Ay = 0.0, vx, vy;
    cohesion_sum(rm[xm], rm[x], rm[xp], r0[xm], r0[xp], rp[xm], rp[x], rp[xp], sx, sy);
    if (P.mask) adhesion_mask(P, x, y, P.links[(unsigned)i], Ax, Ay);
    else adhesion_sum(P, gw, x, y, Ax, Ay);
    velocity(P, f, rho, pc, sx, sy, Ax, Ay, vx, vy);
    const double u = sqrt(vx * vx + vy * vy);
    const bool ok = isfinite(rho) && isfinite(pc) && isfinite(u);
    v[O_BAD] = ok ? 0.0 : 1.0;
    if (ok) {
        v[O_MIN] = rho; v[O_MAX] = rho; v[O_U] = u; v[O_MASS] = rho;
        if (rho >= A.rho_mid) v[O_UL] = u;
    }
    // interface crossings on the edges to the right and upper neighbours
    const bool la = rho >= A.rho_mid;
    if (x + 1 < P.nx && !is_solid_node(P, x + 1, y)) {
        const double rb = rho_f[i + 1];
        if ((rb >= A.rho_mid) != la) {
            const double t = (A.rho_mid - rho) / (rb - rho);
            const double px = x + t, py = (double)y;
            if (py >= A.y_min && px >= A.x_lo && px < A.x_hi) add_point(v, px, py, A.cx, A.cy);
        }
    }
    if (y + 1 <= P.y_hi && !is_solid_node(P, x, y + 1)) {
        const double rb = rho_f[i + P.pitch];
        if ((rb >= A.rho_mid) != la) {
            const double t = (A.rho_mid - rho) / (rb - rho);
            const double px = (double)x, py = y + t;
            if (py >= A.y_min && px >= A.x_lo && px < A.x_hi) add_point(v, px, py, A.cx, A.cy);
        }
    }
}

// XCD-aware tile order: workgroup i runs on XCD i mod 8; give each XCD a contiguous range of
// tiles so neighbouring tiles (which re-read each other's halo) share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int i, int T) {
    const int q = T >> 3, r = T & 7;
    const int k = i & 7, j = i >> 3;
    return k * q + (k < r ? k : r) + j;
}

}  // namespace lbm

namespace lbm {

// One TX x TY tile of the step at origin (x0, y0), executed by a whole workgroup of TX * TY
// threads with the LDS array sp of (TY + 2) * (TX + 2) doubles. FUSED: psi of the tile and its
// halo is evaluated from the pulled populations; otherwise it is staged from psi_g. Contains
// __syncthreads() and no early return, so it can run inside loops over tiles.
template <int TX, int TY, bool FUSED, int GEO, int EOS = EOS_ANY>
__device__ __forceinline__ void step_tile(const KParams& P, const double* __restrict__ gin,
                                          double* __restrict__ gout,
                                          const double* __restrict__ psi_g,
                                          const double* __restrict__ gw, int x0, int y0,
                                          double* sp) {
    constexpr int NT = TX * TY;
    constexpr int LW = TX + 2;
    constexpr int NH = 2 * LW + 2 * TY;  // halo slots of a (TX+2) x (TY+2) tile
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x = x0 + tx, y = y0 + ty;
    unsigned lk = 0;  // solid-mask links of the node
    if (GEO == GEO_MASK && x < P.nx && y <= P.y_hi) lk = P.links[(unsigned)y * P.pitch + x];
    const bool active = x < P.nx && y <= P.y_hi && !(lk & 1u);

    double f[9];
    double rho = 1.0, psi_c = 0.0;
    if (active) {
        if constexpr (GEO == GEO_MASK) pull9_mask(P, gin, x, y, lk, f);
        else pull9<GEO>(P, gin, x, y, f);
        rho = sum9(f);
        if (FUSED) psi_c = psi_of_rho<EOS>(P, rho);
    }
    if (FUSED) {
        // own slot: computed above, or (outside the fluid) the value at that lattice position
        sp[(ty + 1) * LW + tx + 1] = active ? psi_c : psi_at<GEO, EOS>(P, gin, x, y);
        for (int h = threadIdx.x; h < NH; h += NT) {
            int hx, hy;  // tile-local coordinates in [-1, TX] x [-1, TY]
            if (h < LW) { hx = h - 1; hy = -1; }
            else if (h < 2 * LW) { hx = h - LW - 1; hy = TY; }
            else if (h < 2 * LW + TY) { hx = -1; hy = h - 2 * LW; }
            else { hx = TX; hy = h - 2 * LW - TY; }
            sp[(hy + 1) * LW + hx + 1] = psi_at<GEO, EOS>(P, gin, x0 + hx, y0 + hy);
        }
    } else {
        // stage psi (ghost rows already mirrored by the psi pass) with its halo
        for (int s = threadIdx.x; s < (TY + 2) * LW; s += NT) {
            const int gy = y0 - 1 + s / LW;
            const int gx = wrapx(x0 - 1 + s % LW, P.nx);
            double v = 0.0;
            if (P.walls && !P.mask) {
                if (gy >= 0 && gy < P.ny) v = psi_g[(long long)gy * P.pitch + gx];
            } else {
                v = psi_g[(long long)wrapx(gy, P.ny) * P.pitch + gx];
            }
            sp[s] = v;
        }
    }
    __syncthreads();
    if (active) {
        if (!FUSED) psi_c = sp[(ty + 1) * LW + tx + 1];
        const double* c = sp + (ty + 1) * LW + tx + 1;
        double sx, sy;
        cohesion_sum(c[-LW - 1], c[-LW], c[-LW + 1], c[-1], c[1], c[LW - 1], c[LW], c[LW + 1],
                     sx, sy);
        double Ax = 0.0, Ay = 0.0;
        if constexpr (GEO == GEO_MASK) adhesion_mask(P, x, y, lk, Ax, Ay);
        else if (P.walls && (y == 1 || y == P.ny - 2)) adhesion_sum(P, gw, x, y, Ax, Ay);
        store_wall_force<GEO>(P, gout, (long long)y * P.pitch + x, P.plane, P.pitch, y, rho,
                              psi_c, sx, sy, Ax, Ay);
        collide(P, f, rho, psi_c, sx, sy, Ax, Ay);
        const unsigned i = (unsigned)y * P.pitch + x;
#pragma unroll
        for (int a = 0; a < 9; ++a) (gout + a * P.plane)[i] = f[a];
    }
}

}  // namespace lbm

namespace lbm {

// Two time steps per launch (temporal blocking). The workgroup owns a TX x TY tile of the second
// step's output. With Rk the tile grown by k rings:
//   A  psi of step n+1 on R3, from the pulled populations of gin          -> LDS ps1
//   B  step n+1 (forces, collision) on the fluid nodes of R2              -> LDS g1 (9 planes)
//   C  psi of step n+2 on R1, pulling from g1 (bounce-back, ghost rows)   -> LDS ps2
//   D  step n+2 on the tile, pulling from g1                              -> gout
// HBM sees one read and one write of the populations per two steps. Every node's arithmetic is
// that of step_tile, so two launches of k_step and one of k_step2 give identical bits.
template <int GEO>
__device__ __forceinline__ void pull9_lds(const KParams& P, const double* g1, int plane, int W,
                                          int l, int gy, double f[9]) {
    // l: local index of the node in the LDS grid (row stride W); gy: its global row
    const bool bot = P.walls && gy == 1, top = P.walls && gy == P.ny - 2;
    f[0] = g1[l];
    f[1] = g1[1 * plane + l - 1];
    f[3] = g1[3 * plane + l + 1];
    f[2] = bot ? g1[4 * plane + l] : g1[2 * plane + l - W];
    f[5] = bot ? g1[7 * plane + l] : g1[5 * plane + l - W - 1];
    f[6] = bot ? g1[8 * plane + l] : g1[6 * plane + l - W + 1];
    f[4] = top ? g1[2 * plane + l] : g1[4 * plane + l + W];
    f[7] = top ? g1[5 * plane + l] : g1[7 * plane + l + W + 1];
    f[8] = top ? g1[6 * plane + l] : g1[8 * plane + l + W - 1];
    if (GEO == GEO_WET && P.wet && (bot || top)) {
        // the force of the boundary node sits in the solid-row slot below (bottom) or above (top)
        if (bot) wet_node_bottom(f, g1[l - W], g1[plane + l - W]);
        if (top) wet_node_top(f, g1[l + W], g1[plane + l + W]);
    }
}

// Pull of a node whose neighbours are all fluid nodes of the same lattice, reached without the
// periodic wrap: the plain streaming of Eq. (5), the same loads as pull9 makes there.
__device__ __forceinline__ void pull9_in(const KParams& P, const double* __restrict__ g, int x,
                                         int y, double f[9]) {
    const long long pl = P.plane;
    const unsigned r0 = (unsigned)y * P.pitch + x, rm = r0 - P.pitch, rp = r0 + P.pitch;
    f[0] = g[r0];
    f[1] = (g + 1 * pl)[r0 - 1];
    f[3] = (g + 3 * pl)[r0 + 1];
    f[2] = (g + 2 * pl)[rm];
    f[5] = (g + 5 * pl)[rm - 1];
    f[6] = (g + 6 * pl)[rm + 1];
    f[4] = (g + 4 * pl)[rp];
    f[7] = (g + 7 * pl)[rp + 1];
    f[8] = (g + 8 * pl)[rp - 1];
}

template <int GEO, bool IN>
__device__ __forceinline__ bool pull_slot(const KParams& P, const double* __restrict__ g, int gx,
                                          int gy, double f[9], bool& fluid) {
    if constexpr (IN) {
        pull9_in(P, g, gx, gy, f);
        fluid = true;
        return true;
    } else {
        int sx, sy;
        const bool v = slot_source(P, gx, gy, sx, sy);
        fluid = v && (!P.walls || (gy >= 1 && gy <= P.ny - 2));
        if (v) pull9<GEO>(P, g, sx, sy, f);
        return v;
    }
}

// pull9_lds for a node away from the wall rows.
__device__ __forceinline__ void pull9_lds_in(const double* g1, int plane, int W, int l,
                                             double f[9]) {
    f[0] = g1[l];
    f[1] = g1[1 * plane + l - 1];
    f[3] = g1[3 * plane + l + 1];
    f[2] = g1[2 * plane + l - W];
    f[5] = g1[5 * plane + l - W - 1];
    f[6] = g1[6 * plane + l - W + 1];
    f[4] = g1[4 * plane + l + W];
    f[7] = g1[7 * plane + l + W + 1];
    f[8] = g1[8 * plane + l + W - 1];
}

// pull9_lds with a solid mask: lk = links of the node (see pull9_mask).
__device__ __forceinline__ void pull9_lds_mask(const double* g1, int plane, int W, int l,
                                               unsigned lk, double f[9]) {
    f[0] = g1[l];
    f[1] = (lk & 2u) ? g1[3 * plane + l] : g1[1 * plane + l - 1];
    f[2] = (lk & 4u) ? g1[4 * plane + l] : g1[2 * plane + l - W];
    f[3] = (lk & 8u) ? g1[1 * plane + l] : g1[3 * plane + l + 1];
    f[4] = (lk & 16u) ? g1[2 * plane + l] : g1[4 * plane + l + W];
    f[5] = (lk & 32u) ? g1[7 * plane + l] : g1[5 * plane + l - W - 1];
    f[6] = (lk & 64u) ? g1[8 * plane + l] : g1[6 * plane + l - W + 1];
    f[7] = (lk & 128u) ? g1[5 * plane + l] : g1[7 * plane + l + W + 1];
    f[8] = (lk & 256u) ? g1[6 * plane + l] : g1[8 * plane + l + W - 1];
}

// Threads of a two-step workgroup. The LDS of a 64 x 8 tile allows two workgroups per CU; it runs
// 768 threads (12 waves, 6 per SIMD with two workgroups, which step2_waves asks the compiler to
// leave registers for) so that more waves hide each other's latencies and its R2 (816 nodes)
// takes one pass on all but one wave; 832 or more threads leave room for one workgroup per CU
// only. The 64 x 4 tile (three workgroups per CU) runs 512 threads, so that its R2 (544 nodes)
// also takes one pass on all but one wave; the other tiles run one thread per output node.
__host__ __device__ constexpr int step2_threads(int TX, int TY, int GEO) {
    return TX == 64 && TY == 8 ? 768 : (TX == 64 && TY == 4 ? 512 : TX * TY);
}
// Waves per SIMD the two-step kernels must leave registers for (launch bounds): 6 for the tiles
// whose LDS holds two (64 x 8, 12 waves each) or three (64 x 4, 8 waves each) workgroups per CU.
__host__ __device__ constexpr int step2_waves(int TX, int TY, int GEO) {
    return TX == 64 && (TY == 8 || TY == 4) ? 6 : 1;
}
// Threads of a "wide" two-step workgroup, for lattices too small to fill the chip: one R2 slot
// per thread and the outer ring of R3 on waves of its own, so that no wave evaluates more than
// one collision or psi value in a phase and the workgroup's chain of dependent phases is as short
// as the tile allows (64 x 4: 768 threads, 32 x 4: 448).
__host__ __device__ constexpr int step2_wide_threads(int TX, int TY) {
    return ((((TX + 4) * (TY + 4) + 63) / 64 * 64 + 2 * (TX + 6) + 2 * (TY + 4)) + 63) / 64 * 64;
}

// LDS of step2_tile; with a solid mask (GEO_MASK) the link words of R2 are kept too.
template <int TX, int TY, int GEO>
struct Step2Lds {
    static constexpr int W3 = TX + 6, H3 = TY + 6, W2 = TX + 4, H2 = TY + 4, W1 = TX + 2,
                         H1 = TY + 2, PL = W2 * H2;
    double g1[9 * PL];
    double ps1[W3 * H3];
    double ps2[W1 * H1];
    unsigned short lk[GEO == GEO_MASK ? PL : 1];
};

// IN: the tile is interior (step2_interior): every pull of R3 stays inside the lattice, clear of
// the wall rows, solid nodes and the periodic seam, so no node needs a wall, ghost, mask or wrap
// rule. Both variants give the same bits on such a tile. With a solid mask (GEO_MASK) the lattice
// is periodic in x and y, solid nodes hold psi = 0 and are not updated, links select the
// bounce-back of each population and the adhesion sums G_w over the solid neighbours.
// MID: the state after the first of the two steps is also written, to gmid (the tile's nodes;
// without the wet-node force, so not for that wall).
template <int TX, int TY, int GEO, int EOS = EOS_ANY, bool IN = false, bool MID = false,
          bool OPQ = false, int NTH = step2_threads(TX, TY, GEO)>
__device__ __forceinline__ void step2_tile(const KParams& P, const double* __restrict__ gin,
                                           double* __restrict__ gout,
                                           const double* __restrict__ gw, int x0, int y0,
                                           Step2Lds<TX, TY, GEO>& L,
                                           double* __restrict__ gmid = nullptr) {
    // OPQ: the thread index is opaque to the compiler, so nothing derived from it is hoisted
    // out of a loop over tiles around this call (which would hold it in registers throughout)
    int tid = threadIdx.x;
    if constexpr (OPQ) asm volatile("" : "+v"(tid));
    static_assert(!MID || GEO != GEO_WET, "the intermediate state carries no wet-node force");
    constexpr bool MK = GEO == GEO_MASK;
    // NTH threads in the workgroup (the default of the tile shape, or fewer for a caller that
    // needs registers for more waves)
    constexpr int NT = NTH;
    static_assert(NT >= TX * TY, "one thread per output node at least");
    constexpr int W3 = TX + 6, H3 = TY + 6, W2 = TX + 4, H2 = TY + 4, W1 = TX + 2, H1 = TY + 2;
    constexpr int PL = W2 * H2;
    double* g1 = L.g1;
    double* ps1 = L.ps1;
    double* ps2 = L.ps2;

    // A: psi of step n+1 on R3. The R2 slots (up to three per thread) keep their pulled
    // populations and density in registers for B; the outer ring of R3 only needs psi.
    constexpr int NR = (PL + NT - 1) / NT;
    static_assert(NR <= 3, "at most three R2 slots per thread");
    double fk[NR][9], rk[NR];
    bool ok[NR];
    // The ring of R3 outside R2 goes to the waves after those with a slot in the last pass of R2,
    // when they are enough, so that no wave evaluates more than NR psi values.
    constexpr int NRING = 2 * W3 + 2 * H2;
    constexpr int LAST = PL - (NR - 1) * NT;  // threads with a slot in the last pass
    constexpr int RB = (LAST + 63) / 64 * 64;
    constexpr int R0 = RB + NRING <= NT ? RB : 0;
    auto ring_pos = [](int h, int& lx, int& ly) {  // R3-local coordinates of ring slot h
        if (h < W3) { lx = h; ly = 0; }
        else if (h < 2 * W3) { lx = h - W3; ly = H3 - 1; }
        else if (h < 2 * W3 + H2) { lx = 0; ly = h - 2 * W3 + 1; }
        else { lx = W3 - 1; ly = h - 2 * W3 - H2 + 1; }
    };
    if constexpr (!MK && NR == 2 && R0 > 0 && NT < step2_threads(TX, TY, GEO)) {
        // Two passes over R2 and the ring past the second one's threads: a thread holds its first
        // R2 slot and at most one more pull, its second slot or a ring slot, and issues both
        // pulls before it evaluates either psi (one round trip to memory instead of two; the
        // values are those of the loop below). Only for workgroups smaller than the tile's
        // default (the persistent 64 x 8 workgroup of 512 threads, 16 waves per compute unit:
        // 0.337 -> 0.326 ms per step on 8 x 2048x1024); with the default 768 threads the other
        // workgroup of the compute unit hides the second round trip, and issuing both measured
        // 1-3% slower.
        const int s1 = tid + NT, h = tid - R0;
        int l0, l1 = -1;
        bool v0, v1 = false;
        rk[0] = rk[1] = 1.0;
        {
            const int lx = tid % W2, ly = tid / W2;
            l0 = (ly + 1) * W3 + lx + 1;
            v0 = pull_slot<GEO, IN>(P, gin, x0 - 2 + lx, y0 - 2 + ly, fk[0], ok[0]);
        }
        ok[1] = false;
        if (s1 < PL) {
            const int lx = s1 % W2, ly = s1 / W2;
            l1 = (ly + 1) * W3 + lx + 1;
            v1 = pull_slot<GEO, IN>(P, gin, x0 - 2 + lx, y0 - 2 + ly, fk[1], ok[1]);
        } else if (h >= 0 && h < NRING) {
            int lx, ly;
            ring_pos(h, lx, ly);
            l1 = ly * W3 + lx;
            bool fluid;
            v1 = pull_slot<GEO, IN>(P, gin, x0 - 3 + lx, y0 - 3 + ly, fk[1], fluid);
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int l = r ? l1 : l0;
            if (l < 0) continue;
            const bool v = r ? v1 : v0;
            const double rho = v ? sum9(fk[r]) : 1.0;
            rk[r] = ok[r] ? rho : 1.0;
            ps1[l] = v ? psi_of_rho<EOS>(P, rho) : 0.0;
        }
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int s = tid + r * NT;
            ok[r] = false;
            rk[r] = 1.0;
            if (s >= PL) continue;
            const int lx = s % W2, ly = s / W2;
            if constexpr (IN) {
                pull9_in(P, gin, x0 - 2 + lx, y0 - 2 + ly, fk[r]);
                rk[r] = sum9(fk[r]);
                ps1[(ly + 1) * W3 + lx + 1] = psi_of_rho<EOS>(P, rk[r]);
                ok[r] = true;
                continue;
            }
            if constexpr (MK) {
                const int gx = wrapx(x0 - 2 + lx, P.nx), gy = wrapx(y0 - 2 + ly, P.ny);
                const unsigned lk = P.links[(unsigned)gy * P.pitch + gx];
                L.lk[s] = (unsigned short)lk;
                double ps = 0.0;  // solid node
                if (!(lk & 1u)) {
                    pull9_mask(P, gin, gx, gy, lk, fk[r]);
                    rk[r] = sum9(fk[r]);
                    ps = psi_of_rho<EOS>(P, rk[r]);
                    ok[r] = true;
                }
                ps1[(ly + 1) * W3 + lx + 1] = ps;
                continue;
            }
            double ps = 0.0;
            int gy = y0 - 2 + ly;
            bool fluid;
            if (P.walls) fluid = gy >= 1 && gy <= P.ny - 2;
            else { gy = wrapx(gy, P.ny); fluid = true; }
            if (fluid) {
                pull9<GEO>(P, gin, wrapx(x0 - 2 + lx, P.nx), gy, fk[r]);
                rk[r] = sum9(fk[r]);
                ps = psi_of_rho<EOS>(P, rk[r]);
                ok[r] = true;
            } else {
                ps = psi_at<GEO, EOS>(P, gin, x0 - 2 + lx, y0 - 2 + ly);  // solid row: ghost or 0
            }
            ps1[(ly + 1) * W3 + lx + 1] = ps;
        }
        for (int h = tid - R0; h < NRING; h += NT) {
            if (h < 0) continue;
            int lx, ly;
            ring_pos(h, lx, ly);
            if constexpr (IN) {
                double f[9];
                pull9_in(P, gin, x0 - 3 + lx, y0 - 3 + ly, f);
                ps1[ly * W3 + lx] = psi_of_rho<EOS>(P, sum9(f));
            } else {
                ps1[ly * W3 + lx] = psi_at<GEO, EOS>(P, gin, x0 - 3 + lx, y0 - 3 + ly);
            }
        }
    }
    __syncthreads();

    // B: step n+1 on the fluid nodes of R2
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (!ok[r]) continue;
        const int s = tid + r * NT;
        const int lx = s % W2, ly = s / W2;
        const double* c = ps1 + (ly + 1) * W3 + lx + 1;
        double sx, sy;
        cohesion_sum(c[-W3 - 1], c[-W3], c[-W3 + 1], c[-1], c[1], c[W3 - 1], c[W3], c[W3 + 1],
                     sx, sy);
        double Ax = 0.0, Ay = 0.0;
        if constexpr (MK && !IN) {
            adhesion_mask(P, wrapx(x0 - 2 + lx, P.nx), wrapx(y0 - 2 + ly, P.ny), L.lk[s], Ax, Ay);
        } else if constexpr (!IN) {
            const int gx = wrapx(x0 - 2 + lx, P.nx);
            const int gy = P.walls ? y0 - 2 + ly : wrapx(y0 - 2 + ly, P.ny);
            if (P.walls && (gy == 1 || gy == P.ny - 2)) adhesion_sum(P, gw, gx, gy, Ax, Ay);
            // a boundary node's force feeds the reconstruction of step n+2, which only nodes of
            // R1 perform; those have their solid-row slot inside R2
            if (GEO == GEO_WET && P.wet && ly >= 1 && ly <= H2 - 2)
                store_wall_force<GEO>(P, g1, s, PL, W2, gy, rk[r], c[0], sx, sy, Ax, Ay);
        }
        collide(P, fk[r], rk[r], c[0], sx, sy, Ax, Ay);
#pragma unroll
        for (int a = 0; a < 9; ++a) g1[a * PL + s] = fk[r][a];
        if constexpr (MID) {
            // a node of the tile: its state after step n+1
            const int x = x0 - 2 + lx, y = y0 - 2 + ly;
            if (lx >= 2 && lx <= W2 - 3 && ly >= 2 && ly <= H2 - 3 && x < P.nx && y <= P.y_hi) {
                const unsigned i = (unsigned)y * P.pitch + x;
#pragma unroll
                for (int a = 0; a < 9; ++a) (gmid + a * P.plane)[i] = fk[r][a];
            }
        }
    }
    __syncthreads();

    // C: psi of step n+2 on R1 (solid rows take the mirrored fluid row, or 0). A thread first
    // evaluates its own node of the tile, whose pulled populations and density stay in registers
    // for D; the ring of R1 around the tile goes to the threads past the tile's nodes when there
    // are enough of them, otherwise to the first threads after their own node.
    constexpr int NTILE = TX * TY;
    constexpr int NRING1 = 2 * W1 + 2 * TY;  // R1 outside the tile
    const bool own = NT == NTILE || tid < NTILE;
    const int tx = tid % TX, ty = tid / TX;
    const int x = x0 + tx, y = y0 + ty;
    const int l = (ty + 2) * W2 + tx + 2;
    unsigned lk = 0;  // links of the node (solid mask)
    if constexpr (MK && !IN) lk = own ? L.lk[l] : 1u;
    const bool act = own && (IN || (x < P.nx && y <= P.y_hi)) && !(lk & 1u);
    // psi at R1 slot (lx, ly), pulled from the populations in LDS
    auto slot_psi = [&](int lx, int ly) -> double {
        double g[9];
        if constexpr (IN) {
            pull9_lds_in(g1, PL, W2, (ly + 1) * W2 + lx + 1, g);
        } else if constexpr (MK) {
            const int ll = (ly + 1) * W2 + lx + 1;
            const unsigned k = L.lk[ll];
            if (k & 1u) return 0.0;  // solid node
            pull9_lds_mask(g1, PL, W2, ll, k, g);
        } else {
            int sx, sy;
            if (!slot_source(P, x0 - 1 + lx, y0 - 1 + ly, sx, sy)) return 0.0;
            // the source node in the R2 grid: same column, row sy (mirrored rows stay adjacent)
            const int ly2 = P.walls ? sy - (y0 - 2) : ly + 1;
            pull9_lds<GEO>(P, g1, PL, W2, ly2 * W2 + lx + 1, sy, g);
        }
        return psi_of_rho<EOS>(P, sum9(g));
    };
    double f[9], rho = 1.0;
    if (act) {
        if constexpr (IN) pull9_lds_in(g1, PL, W2, l, f);
        else if constexpr (MK) pull9_lds_mask(g1, PL, W2, l, lk, f);
        else pull9_lds<GEO>(P, g1, PL, W2, l, y, f);
        rho = sum9(f);
        ps2[(ty + 1) * W1 + tx + 1] = psi_of_rho<EOS>(P, rho);
    } else if (own) {
        ps2[(ty + 1) * W1 + tx + 1] = slot_psi(tx + 1, ty + 1);  // outside the lattice, or solid
    }
    constexpr int RR0 = NT >= NTILE + NRING1 ? NTILE : 0;
    for (int h = tid - RR0; h < NRING1; h += NT) {
        if (h < 0) continue;
        int lx, ly;  // R1-local coordinates
        if (h < W1) { lx = h; ly = 0; }
        else if (h < 2 * W1) { lx = h - W1; ly = H1 - 1; }
        else if (h < 2 * W1 + TY) { lx = 0; ly = h - 2 * W1 + 1; }
        else { lx = W1 - 1; ly = h - 2 * W1 - TY + 1; }
        ps2[ly * W1 + lx] = slot_psi(lx, ly);
    }
    __syncthreads();

    // D: step n+2 on the tile
    if (act) {
        const double* c = ps2 + (ty + 1) * W1 + tx + 1;
        double sx, sy;
        cohesion_sum(c[-W1 - 1], c[-W1], c[-W1 + 1], c[-1], c[1], c[W1 - 1], c[W1], c[W1 + 1],
                     sx, sy);
        double Ax = 0.0, Ay = 0.0;
        if constexpr (MK && !IN) {
            adhesion_mask(P, x, y, lk, Ax, Ay);
        } else if constexpr (!IN) {
            if (P.walls && (y == 1 || y == P.ny - 2)) adhesion_sum(P, gw, x, y, Ax, Ay);
            store_wall_force<GEO>(P, gout, (long long)y * P.pitch + x, P.plane, P.pitch, y, rho,
                                  c[0], sx, sy, Ax, Ay);
        }
        collide(P, f, rho, c[0], sx, sy, Ax, Ay);
        const unsigned i = (unsigned)y * P.pitch + x;
#pragma unroll
        for (int a = 0; a < 9; ++a) (gout + a * P.plane)[i] = f[a];
    }
}


// True when the pulls of every node of the tile's R3 (see step2_tile) stay inside the lattice
// without the periodic wrap and touch no wall rule: R3 and its pull neighbours lie in columns
// [0, nx) and, with walls, in rows [1, ny-2] (only nodes of rows 1 and ny-2 have solid
// neighbours), otherwise in rows [0, ny). A solid mask also needs no solid node among them: the
// whole workgroup checks the link words of the tile grown by 4 rings (a barrier).
template <int TX, int TY, int GEO, int NTH = step2_threads(TX, TY, GEO)>
__device__ __forceinline__ bool step2_interior(const KParams& P, int x0, int y0) {
    if (x0 - 4 < 0 || x0 + TX + 3 > P.nx - 1) return false;
    if (GEO != GEO_MASK && P.walls) return y0 - 3 >= 2 && y0 + TY + 2 <= P.ny - 3;
    if (y0 - 4 < 0 || y0 + TY + 3 > P.ny - 1) return false;
    if constexpr (GEO == GEO_MASK) {
        constexpr int W4 = TX + 8, N4 = (TX + 8) * (TY + 8);
        int solid = 0;
        for (int s = threadIdx.x; s < N4; s += NTH)
            solid |= P.links[(unsigned)(y0 - 4 + s / W4) * P.pitch + (x0 - 4 + s % W4)] & 1;
        return !__syncthreads_or(solid);
    }
    return true;
}

// step2_tile with the interior variant where it applies (a uniform branch per workgroup).
template <int TX, int TY, int GEO, int EOS, bool MID = false, bool OPQ = false,
          int NTH = step2_threads(TX, TY, GEO)>
__device__ __forceinline__ void step2_tile_any(const KParams& P, const double* __restrict__ gin,
                                               double* __restrict__ gout,
                                               const double* __restrict__ gw, int x0, int y0,
                                               Step2Lds<TX, TY, GEO>& L,
                                               double* __restrict__ gmid = nullptr) {
    if (step2_interior<TX, TY, GEO, NTH>(P, x0, y0))
        step2_tile<TX, TY, GEO, EOS, true, MID, OPQ, NTH>(P, gin, gout, gw, x0, y0, L, gmid);
    else
        step2_tile<TX, TY, GEO, EOS, false, MID, OPQ, NTH>(P, gin, gout, gw, x0, y0, L, gmid);
}

}  // namespace lbm

namespace lbm {

// Contact line on row `row` (dynamic wetting, Sec. III.B): the rho_mid crossings of the row,
// linearly interpolated on the edges (x, x+1) that do not cross the periodic seam. out[0] = the
// leftmost crossing where rho rises through rho_mid, out[1] = the rightmost where it falls; both
// NaN when the row holds no liquid segment. Called by a whole block of 256 threads; min and max
// do not depend on the reduction order.
__device__ __forceinline__ void contact_line_block(const KParams& P, const double* __restrict__ gin,
                                                  int row, double mid, double* __restrict__ out) {
    __shared__ double lo[256], hi[256];
    double l = __builtin_huge_val(), h = -__builtin_huge_val();
    for (int x = threadIdx.x; x + 1 < P.nx; x += 256) {
        if (is_solid_node(P, x, row) || is_solid_node(P, x + 1, row)) continue;
        double f[9];
        pull9_any(P, gin, x, row, f);
        const double ra = sum9(f);
        pull9_any(P, gin, x + 1, row, f);
        const double rb = sum9(f);
        if ((ra >= mid) == (rb >= mid)) continue;
        const double px = x + (mid - ra) / (rb - ra);
        if (rb >= mid) l = fmin(l, px);
        else h = fmax(h, px);
    }
    lo[threadIdx.x] = l;
    hi[threadIdx.x] = h;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + w]);
            hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool ok = lo[0] < hi[0];
        out[0] = ok ? lo[0] : __builtin_nan("");
        out[1] = ok ? hi[0] : __builtin_nan("");
    }
}

}  // namespace lbm

// ================================================================================================
// Adjoint (reverse mode) of the per-node arithmetic
// ================================================================================================
namespace lbm {

// dpsi/drho = (p'(rho) - 1/3) / (G psi), from psi^2 = 2 (p - rho/3)/G.
template <int EOS = EOS_ANY>
__device__ __forceinline__ double dpsi_drho(const KParams& P, double rho, double psi) {
#pragma clang fp contract(off)
    double dp;
    if (EOS == EOS_CS || (EOS == EOS_ANY && P.eos == 0)) {
        const double e = P.b4 * rho, om = 1.0 - e;
        const double om2 = om * om;
        const double D1 = (1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)))) / (om2 * om2);
        dp = P.RT * D1 - 2.0 * P.a * rho;
    } else {
        dp = rho <= P.rho1 ? P.th_v : (rho <= P.rho2 ? P.th_m : P.th_l);
    }
    // 2/G * (dp - 1/3) / (2 psi)
    return 0.5 * P.two_over_G * (dp - 1.0 / 3.0) / psi;
}

// Reverse mode of collide() at one node. In: the forward inputs (f pre-collision, rho = sum f,
// psi_c, cohesion sum s, adhesion sum A) and nu = dL/df* (9). Out: fb = dL/df through every path
// that does not pass through psi (9, including the rho = sum f dependence of v, m_eq, tau_nu and
// a density pre-sum factor), pb = dL/dpsi_c as the node's own pre-factor, (qx, qy) = dL/ds, and
// (rx, ry) = dL/dA.
__device__ __forceinline__ void collide_adj(const KParams& P, const double f[9], double rho,
                                            double psi_c, double sx, double sy, double Ax,
                                            double Ay, const double nu[9], double fb[9],
                                            double& pb, double& qx, double& qy, double& rx,
                                            double& ry) {
#pragma clang fp contract(off)
    // ---- forward recomputation (same expressions as collide) ----
    const double fmx = P.negG * psi_c * sx, fmy = P.negG * psi_c * sy;
    const double pre = P.wall_force == 0 ? rho : (P.wall_force == 1 ? psi_c : psi_c * psi_c);
    const double Fx = fmx - pre * Ax, Fy = fmy - pre * Ay;
    const double ax = f[1] + f[3], ay = f[2] + f[4];
    const double d58 = f[5] - f[7], d68 = f[6] - f[8];
    const double jx = (f[1] - f[3]) + d58 - d68;
    const double jy = (f[2] - f[4]) + d58 + d68;
    const double m7 = ax - ay;
    const double m8 = (f[5] + f[7]) - (f[6] + f[8]);
    const double ir = 1.0 / rho;
    const double vx = (jx + 0.5 * Fx) * ir, vy = (jy + 0.5 * Fy) * ir;
    const double v2 = vx * vx + vy * vy;
    double snu, dsnu_drho = 0.0;
    if (P.visc_const) {
        snu = P.s_nu_c;
    } else {
        const double phr = (rho - P.rho_v) * P.inv_drho;
        const double ph = fmin(fmax(phr, 0.0), 1.0);
        snu = 1.0 / (3.0 * (P.nu_v + ph * P.dnu) + 0.5);
        if (phr > 0.0 && phr < 1.0) dsnu_drho = -snu * snu * 3.0 * P.dnu * P.inv_drho;
    }
    const double hnu = 1.0 - 0.5 * snu;
    const double S7 = 2.0 * (vx * Fx - vy * Fy);
    const double S8 = vx * Fy + vy * Fx;

    // ---- mu = dL/dm* = D (M nu), D = diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) ----
    const double nax = nu[1] + nu[3], nay = nu[2] + nu[4];
    const double nsa = nax + nay, nsd = (nu[5] + nu[7]) + (nu[6] + nu[8]);
    const double n58 = nu[5] - nu[7], n68 = nu[6] - nu[8];
    const double mu0 = (nu[0] + nsa + nsd) * (1.0 / 9.0);
    const double mu1 = (-4.0 * nu[0] - nsa + 2.0 * nsd) * (1.0 / 36.0);
    const double mu2 = (4.0 * nu[0] - 2.0 * nsa + nsd) * (1.0 / 36.0);
    const double mu3 = ((nu[1] - nu[3]) + n58 - n68) * (1.0 / 6.0);
    const double mu4 = (-2.0 * (nu[1] - nu[3]) + n58 - n68) * (1.0 / 12.0);
    const double mu5 = ((nu[2] - nu[4]) + n58 + n68) * (1.0 / 6.0);
    const double mu6 = (-2.0 * (nu[2] - nu[4]) + n58 + n68) * (1.0 / 12.0);
    const double mu7 = (nax - nay) * 0.25;
    const double mu8 = ((nu[5] + nu[7]) - (nu[6] + nu[8])) * 0.25;

    // ---- Eq. (4) relaxation, reversed ----
    double rb = mu0;  // m*_0 = rho
    double vxb = 0.0, vyb = 0.0, v2b = 0.0, Fxb = 0.0, Fyb = 0.0;
    const double m1b = mu1 * (1.0 - P.s_e);
    rb += mu1 * P.s_e * (-2.0 + 3.0 * v2);
    v2b += mu1 * P.s_e * rho * 3.0;
    const double S1b = mu1 * P.h_e;
    const double m2b = mu2 * (1.0 - P.s_z);
    rb += mu2 * P.s_z * (1.0 - 3.0 * v2);
    v2b -= mu2 * P.s_z * rho * 3.0;
    const double S2b = mu2 * P.h_z;
    const double jxb = mu3 * (1.0 - P.s_j);
    rb += mu3 * P.s_j * vx;
    vxb += mu3 * P.s_j * rho;
    Fxb += mu3 * P.h_j;
    const double m4b = mu4 * (1.0 - P.s_q);
    rb -= mu4 * P.s_q * vx;
    vxb -= mu4 * P.s_q * rho;
    Fxb -= mu4 * P.h_q;
    const double jyb = mu5 * (1.0 - P.s_j);
    rb += mu5 * P.s_j * vy;
    vyb += mu5 * P.s_j * rho;
    Fyb += mu5 * P.h_j;
    const double m6b = mu6 * (1.0 - P.s_q);
    rb -= mu6 * P.s_q * vy;
    vyb -= mu6 * P.s_q * rho;
    Fyb -= mu6 * P.h_q;
    const double m7b = mu7 * (1.0 - snu);
    double snub = mu7 * (-(m7 - rho * (vx * vx - vy * vy)) - 0.5 * S7);
    rb += mu7 * snu * (vx * vx - vy * vy);
    vxb += mu7 * snu * rho * 2.0 * vx;
    vyb -= mu7 * snu * rho * 2.0 * vy;
    const double S7b = mu7 * hnu;
    const double m8b = mu8 * (1.0 - snu);
    snub += mu8 * (-(m8 - rho * vx * vy) - 0.5 * S8);
    rb += mu8 * snu * vx * vy;
    vxb += mu8 * snu * rho * vy;
    vyb += mu8 * snu * rho * vx;
    const double S8b = mu8 * hnu;

    // ---- Eq. (9) forcing, reversed ----
    const double vFb = 6.0 * (S1b - S2b);
    const double s2b = P.c_sig_e * S1b - P.c_sig_z * S2b;
    vxb += 2.0 * S7b * Fx + S8b * Fy + vFb * Fx;
    vyb += -2.0 * S7b * Fy + S8b * Fx + vFb * Fy;
    Fxb += 2.0 * S7b * vx + S8b * vy + vFb * vx;
    Fyb += -2.0 * S7b * vy + S8b * vx + vFb * vy;
    double sxb = 2.0 * sx * s2b, syb = 2.0 * sy * s2b;

    // ---- shear rate, |v|^2, velocity (Eq. 6) ----
    rb += snub * dsnu_drho;
    vxb += 2.0 * vx * v2b;
    vyb += 2.0 * vy * v2b;
    const double jxb2 = jxb + vxb * ir, jyb2 = jyb + vyb * ir;
    Fxb += 0.5 * vxb * ir;
    Fyb += 0.5 * vyb * ir;
    rb -= (vxb * vx + vyb * vy) * ir;

    // ---- forces (Eqs. 7, 10, 11, 14) ----
    rx = -pre * Fxb;
    ry = -pre * Fyb;
    const double preb = -(Fxb * Ax + Fyb * Ay);
    pb = P.negG * (sx * Fxb + sy * Fyb);
    if (P.wall_force == 0) rb += preb;
    else if (P.wall_force == 1) pb += preb;
    else pb += 2.0 * psi_c * preb;
    sxb += P.negG * psi_c * Fxb;
    syb += P.negG * psi_c * Fyb;
    qx = sxb;
    qy = syb;

    // ---- m = M f reversed, plus rho = sum f ----
    // fb_a = sum_k M[k][a] mb_k + rb, with mb = (0, m1b, m2b, jxb2, m4b, jyb2, m6b, m7b, m8b)
    const double ba = -m1b - 2.0 * m2b, bd = 2.0 * m1b + m2b;
    const double X = jxb2 + m4b, Y = jyb2 + m6b;
    fb[0] = rb - 4.0 * m1b + 4.0 * m2b;
    fb[1] = rb + ba + jxb2 - 2.0 * m4b + m7b;
    fb[3] = rb + ba - jxb2 + 2.0 * m4b + m7b;
    fb[2] = rb + ba + jyb2 - 2.0 * m6b - m7b;
    fb[4] = rb + ba - jyb2 + 2.0 * m6b - m7b;
    fb[5] = rb + bd + X + Y + m8b;
    fb[6] = rb + bd - X + Y - m8b;
    fb[7] = rb + bd - X - Y + m8b;
    fb[8] = rb + bd + X - Y - m8b;
}

// nu = dL/dg at fluid node (x, y) is the transpose of pull streaming with bounce-back applied to
// lambda = a + c 1 (a: 9 planes, c: one scalar plane): g_b(y) feeds f_b(y + e_b), or f_opp(b)(y)
// when y + e_b is solid. push_gather_a reads the a part from HBM (av[b]); push_add_c adds c from
// an LDS tile (l: the node's slot, W: row stride), the same source node for each b.
__device__ __forceinline__ void push_gather_a(const KParams& P, const double* __restrict__ a,
                                              int x, int y, double av[9]) {
    const unsigned nx = P.nx, pitch = P.pitch;
    const unsigned ux = x;
    const unsigned xm = ux == 0 ? nx - 1 : ux - 1;
    const unsigned xp = ux == nx - 1 ? 0 : ux + 1;
    unsigned ym, yp;
    bool bot, top;
    if (P.walls) {
        ym = y - 1; yp = y + 1;
        bot = (y == 1); top = (y == P.ny - 2);
    } else {
        ym = y == 0 ? P.ny - 1 : y - 1;
        yp = y == P.ny - 1 ? 0 : y + 1;
        bot = top = false;
    }
    const long long pl = P.plane;
    const unsigned r0 = (unsigned)y * pitch, rm = ym * pitch, rp = yp * pitch;
    const unsigned i0 = r0 + ux;
    av[0] = a[i0];
    av[1] = (a + 1 * pl)[r0 + xp];
    av[3] = (a + 3 * pl)[r0 + xm];
    // e_y = +1 populations travel up: reflected at the top wall
    av[2] = top ? (a + 4 * pl)[i0] : (a + 2 * pl)[rp + ux];
    av[5] = top ? (a + 7 * pl)[i0] : (a + 5 * pl)[rp + xp];
    av[6] = top ? (a + 8 * pl)[i0] : (a + 6 * pl)[rp + xm];
    // e_y = -1 populations travel down: reflected at the bottom wall
    av[4] = bot ? (a + 2 * pl)[i0] : (a + 4 * pl)[rm + ux];
    av[7] = bot ? (a + 5 * pl)[i0] : (a + 7 * pl)[rm + xm];
    av[8] = bot ? (a + 6 * pl)[i0] : (a + 8 * pl)[rm + xp];
}

// push_gather_a for a node whose neighbours are all fluid, inside the lattice (no wrap).
__device__ __forceinline__ void push_gather_a_in(const KParams& P, const double* __restrict__ a,
                                                 int x, int y, double av[9]) {
    const long long pl = P.plane;
    const unsigned r0 = (unsigned)y * P.pitch + x, rm = r0 - P.pitch, rp = r0 + P.pitch;
    av[0] = a[r0];
    av[1] = (a + 1 * pl)[r0 + 1];
    av[3] = (a + 3 * pl)[r0 - 1];
    av[2] = (a + 2 * pl)[rp];
    av[5] = (a + 5 * pl)[rp + 1];
    av[6] = (a + 6 * pl)[rp - 1];
    av[4] = (a + 4 * pl)[rm];
    av[7] = (a + 7 * pl)[rm - 1];
    av[8] = (a + 8 * pl)[rm + 1];
}

template <bool IN = false>
__device__ __forceinline__ void push_add_c(const KParams& P, const double av[9], const double* cs,
                                           int W, int l, int y, double nu[9]) {
    const bool top = !IN && P.walls && y == P.ny - 2, bot = !IN && P.walls && y == 1;
    const double c0 = cs[l];
    nu[0] = av[0] + c0;
    nu[1] = av[1] + cs[l + 1];
    nu[3] = av[3] + cs[l - 1];
    nu[2] = av[2] + (top ? c0 : cs[l + W]);
    nu[5] = av[5] + (top ? c0 : cs[l + W + 1]);
    nu[6] = av[6] + (top ? c0 : cs[l + W - 1]);
    nu[4] = av[4] + (bot ? c0 : cs[l - W]);
    nu[7] = av[7] + (bot ? c0 : cs[l - W - 1]);
    nu[8] = av[8] + (bot ? c0 : cs[l - W + 1]);
}

// xi = dL/dpsi of node (x, y) = p0 + sum_a w_a e_a . q(x - e_a) (+ the mirrored ghost rows, whose
// psi is this row's), the transpose of the cohesion stencil of Eq. (7); q from an LDS tile
// (slot l, row stride W; rows outside the fluid hold 0).
template <bool IN = false>
__device__ __forceinline__ double adj_xi(const KParams& P, const double* qx, const double* qy,
                                         int W, int l, int y, double p0) {
#pragma clang fp contract(off)
    double xi = (qx[l - 1] - qx[l + 1] + qy[l - W] - qy[l + W]) * (1.0 / 3.0) +
                ((qx[l - W - 1] + qy[l - W - 1]) + (qy[l - W + 1] - qx[l - W + 1]) -
                 (qx[l + W + 1] + qy[l + W + 1]) + (qx[l + W - 1] - qy[l + W - 1])) *
                    (1.0 / 12.0);
    if (!IN && P.walls && P.ghost) {
        if (y == 1)
            xi += -qy[l] * (1.0 / 3.0) +
                  ((-qx[l + 1] - qy[l + 1]) + (qx[l - 1] - qy[l - 1])) * (1.0 / 12.0);
        if (y == P.ny - 2)
            xi += qy[l] * (1.0 / 3.0) +
                  ((qx[l - 1] + qy[l - 1]) + (qy[l + 1] - qx[l + 1])) * (1.0 / 12.0);
    }
    return xi + p0;
}

// Pointers of one reverse step: the forward state g^{n-1} whose step is reversed, the adjoint
// quantities of the later step (in) and of this one (out), the G_w gradient being accumulated.
struct AdjPtrs {
    const double* gprev;
    const double* a_in;     // 9 planes: dL/df^n along every path except psi
    const double* q_in;     // 2 planes: dL/ds of the cohesion sum
    const double* p0_in;    // dL/dpsi as the node's own pre-factor
    const double* dpsi_in;  // psi'(rho)
    const double* rv_in;    // 4 rows: dL/dA on the wall rows (bottom x, y; top x, y)
    const double* gw;
    double* a_out;
    double* q_out;
    double* p0_out;
    double* dpsi_out;
    double* rv_out;
    double* gwgrad;  // [2][pitch]
};

template <int TX, int TY>
struct AdjLds {
    double sp[(TY + 2) * (TX + 2)];  // psi of g^{n-1} on the tile and one ring
    double qx[(TY + 4) * (TX + 4)];  // q of the later step on the tile and two rings
    double qy[(TY + 4) * (TX + 4)];
    double cs[(TY + 2) * (TX + 2)];  // c = psi' xi of the later step on the tile and one ring
};

// dL/dG_w of the solid node below (bottom wall) or above (top wall) fluid node x of a wall row,
// from the wall vectors r = dL/dA of one step (omega = w/3: 1/9 axial, 1/36 diagonal).
__device__ __forceinline__ void adj_gw_node(const KParams& P, const double* __restrict__ rv,
                                            double* __restrict__ gwgrad, int x, int y) {
#pragma clang fp contract(off)
    const unsigned pitch = P.pitch, ux = x;
    const unsigned xm = ux == 0 ? P.nx - 1 : ux - 1;
    const unsigned xp = ux == (unsigned)P.nx - 1 ? 0 : ux + 1;
    if (y == 1) {
        const double* rX = rv;
        const double* rY = rv + pitch;
        gwgrad[ux] += -rY[ux] * (1.0 / 9.0) + ((-rX[xp] - rY[xp]) + (rX[xm] - rY[xm])) * (1.0 / 36.0);
    }
    if (y == P.ny - 2) {
        const double* rX = rv + 2 * pitch;
        const double* rY = rv + 3 * pitch;
        gwgrad[pitch + ux] +=
            rY[ux] * (1.0 / 9.0) + ((rX[xm] + rY[xm]) + (rY[xp] - rX[xp])) * (1.0 / 36.0);
    }
}

// One reverse step on a TX x TY tile (bounce-back or periodic rows), executed by TX * TY threads:
// lambda^{n-1} = (df^n / df^{n-1})^T lambda^n with lambda = a + c 1, where the scalar part
// c = psi' xi of the later step is formed here, on the tile and one ring, from that step's q, p0
// and psi' (the transpose of the cohesion stencil: each node's psi feeds its 8 neighbours' forces);
// then the forward node is recomputed from g^{n-1} and reverse mode runs through the MRT
// collision, forcing and adhesion (collide_adj). The later step's wall vectors are added to the
// G_w gradient (the last reverse step's by adj_gw_node afterwards).
// NTH threads: one per tile node, or twice as many, the others taking ring work only (more
// waves per compute unit on small lattices). EOS: the equation of state (EOS_ANY: chosen at run
// time). IN: the interior variant (adj_interior), without wall, ghost and wrap rules.
template <int TX, int TY, int NTH, int EOS, bool IN>
__device__ __forceinline__ void adj_tile_impl(const KParams& P, const AdjPtrs& A, int x0, int y0,
                                              AdjLds<TX, TY>& L) {
#pragma clang fp contract(off)
    constexpr int NT = NTH, NTILE = TX * TY;
    static_assert(NTH == NTILE || NTH == 2 * NTILE, "one or two threads per tile node");
    constexpr int LW = TX + 2, QW = TX + 4;
    constexpr int NH = 2 * LW + 2 * TY;
    const bool owner = NTH == NTILE || (int)threadIdx.x < NTILE;
    const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY;
    const int x = x0 + tx, y = y0 + ty;
    const bool active = owner && x < P.nx && y <= P.y_hi;
    // ring work starts at the threads that own no node
    const int rt = NTH == NTILE ? (int)threadIdx.x : ((int)threadIdx.x + NTH - NTILE) % NTH;

    // Every global load is issued before the first barrier: the forward node, psi of the ring,
    // q of two rings, the a part of the transposed streaming, p0 and psi' of the c ring and G_w.
    // forward node and psi on the tile and one ring
    double f[9];
    double rho = 1.0, psi_c = 0.0;
    if (active) {
        if constexpr (IN) pull9_in(P, A.gprev, x, y, f);
        else pull9<GEO_ROWS>(P, A.gprev, x, y, f);
        rho = sum9(f);
        psi_c = psi_of_rho<EOS>(P, rho);
    }
    double av[9];
    if (active) {
        if constexpr (IN) push_gather_a_in(P, A.a_in, x, y, av);
        else push_gather_a(P, A.a_in, x, y, av);
    }
    double Ax = 0.0, Ay = 0.0;
    const bool wall_row = !IN && P.walls && (y == 1 || y == P.ny - 2);
    if (active && wall_row) adhesion_sum(P, A.gw, x, y, Ax, Ay);
    // p0 and psi' of the later step on this thread's slots of the c ring
    constexpr int NC = (TY + 2) * LW, NCR = (NC + NT - 1) / NT;
    double p0v[NCR], dpv[NCR];
    bool flv[NCR];
#pragma unroll
    for (int r = 0; r < NCR; ++r) {
        const int s = rt + r * NT;
        p0v[r] = 0.0;
        dpv[r] = 0.0;
        flv[r] = false;
        if (s >= NC) continue;
        int gx = x0 - 1 + s % LW, gy = y0 - 1 + s / LW;
        if constexpr (!IN) {
            gx = wrapx(gx, P.nx);
            if (P.walls) {
                if (gy < 1 || gy > P.ny - 2) continue;
            } else {
                gy = wrapx(gy, P.ny);
            }
        }
        const unsigned i = (unsigned)gy * P.pitch + gx;
        p0v[r] = A.p0_in[i];
        dpv[r] = A.dpsi_in[i];
        flv[r] = true;
    }
    // psi of the ring: interior tiles pull every ring node directly (all fluid, no wrap)
    auto ring_psi = [&](int gx, int gy) {
        if constexpr (IN) {
            double fr[9];
            pull9_in(P, A.gprev, gx, gy, fr);
            return psi_of_rho<EOS>(P, sum9(fr));
        } else {
            return psi_at<GEO_ROWS, EOS>(P, A.gprev, gx, gy);
        }
    };
    if (owner) L.sp[(ty + 1) * LW + tx + 1] = active ? psi_c : ring_psi(x, y);
    for (int h = rt; h < NH; h += NT) {
        int hx, hy;
        if (h < LW) { hx = h - 1; hy = -1; }
        else if (h < 2 * LW) { hx = h - LW - 1; hy = TY; }
        else if (h < 2 * LW + TY) { hx = -1; hy = h - 2 * LW; }
        else { hx = TX; hy = h - 2 * LW - TY; }
        L.sp[(hy + 1) * LW + hx + 1] = ring_psi(x0 + hx, y0 + hy);
    }
    // q of the later step on the tile and two rings (0 outside the fluid rows)
    for (int s = rt; s < (TY + 4) * QW; s += NT) {
        int gx = x0 - 2 + s % QW, gy = y0 - 2 + s / QW;
        bool fluid = true;
        if constexpr (!IN) {
            gx = wrapx(gx, P.nx);
            if (P.walls) fluid = gy >= 1 && gy <= P.ny - 2;
            else gy = wrapx(gy, P.ny);
        }
        double vx = 0.0, vy = 0.0;
        if (fluid) {
            const unsigned i = (unsigned)gy * P.pitch + gx;
            vx = A.q_in[i];
            vy = (A.q_in + P.plane)[i];
        }
        L.qx[s] = vx;
        L.qy[s] = vy;
    }
    __syncthreads();
    // c of the later step on the tile and one ring (0 on the solid rows)
#pragma unroll
    for (int r = 0; r < NCR; ++r) {
        const int s = rt + r * NT;
        if (s >= NC) continue;
        const int hx = s % LW, hy = s / LW;
        int gy = y0 - 1 + hy;
        if (!IN && !P.walls) gy = wrapx(gy, P.ny);
        L.cs[s] = flv[r] ? dpv[r] * adj_xi<IN>(P, L.qx, L.qy, QW, (hy + 1) * QW + hx + 1, gy,
                                               p0v[r])
                         : 0.0;
    }
    __syncthreads();
    if (!active) return;

    const double* cc = L.sp + (ty + 1) * LW + tx + 1;
    double sx, sy;
    cohesion_sum(cc[-LW - 1], cc[-LW], cc[-LW + 1], cc[-1], cc[1], cc[LW - 1], cc[LW],
                 cc[LW + 1], sx, sy);

    double nu[9], fb[9], pb, qx, qy, rx, ry;
    push_add_c<IN>(P, av, L.cs, LW, (ty + 1) * LW + tx + 1, y, nu);
    collide_adj(P, f, rho, psi_c, sx, sy, Ax, Ay, nu, fb, pb, qx, qy, rx, ry);

    const unsigned i = (unsigned)y * P.pitch + x;
#pragma unroll
    for (int k = 0; k < 9; ++k) (A.a_out + k * P.plane)[i] = fb[k];
    A.q_out[i] = qx;
    (A.q_out + P.plane)[i] = qy;
    A.p0_out[i] = pb;
    A.dpsi_out[i] = dpsi_drho<EOS>(P, rho, psi_c);
    if (wall_row) {
        if (y == 1) { A.rv_out[x] = rx; A.rv_out[P.pitch + x] = ry; }
        if (y == P.ny - 2) { A.rv_out[2 * P.pitch + x] = rx; A.rv_out[3 * P.pitch + x] = ry; }
        adj_gw_node(P, A.rv_in, A.gwgrad, x, y);
    }
}

// A reverse-step tile whose reads (the tile grown by two rings for q, by one for the rest, and
// the pulls of those) stay inside the lattice without wrapping and touch no node next to a wall
// row: no bounce-back, ghost row, wall force or wall vector is involved.
template <int TX, int TY>
__device__ __forceinline__ bool adj_interior(const KParams& P, int x0, int y0) {
    if (x0 - 2 < 0 || x0 + TX + 1 > P.nx - 1) return false;
    if (P.walls) return y0 >= 4 && y0 + TY + 1 <= P.ny - 3;
    return y0 >= 3 && y0 + TY + 2 <= P.ny - 1;
}

// One reverse step on a TX x TY tile: the interior variant where it applies (a uniform branch).
template <int TX, int TY, int NTH = TX * TY, int EOS = EOS_ANY>
__device__ __forceinline__ void adj_tile(const KParams& P, const AdjPtrs& A, int x0, int y0,
                                         AdjLds<TX, TY>& L) {
    if (adj_interior<TX, TY>(P, x0, y0))
        adj_tile_impl<TX, TY, NTH, EOS, true>(P, A, x0, y0, L);
    else
        adj_tile_impl<TX, TY, NTH, EOS, false>(P, A, x0, y0, L);
}

}  // namespace lbm
