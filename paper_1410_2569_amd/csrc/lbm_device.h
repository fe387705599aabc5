// lbm_device.h -- per-node device arithmetic of the wetting pseudopotential LB step (gfx950, FP64).
//
// State layout in HBM: two ping-pong buffers g[2], each 9 population planes of ny rows x pitch
// doubles (x fastest, pitch a multiple of 32 doubles so every row starts on a 256-byte boundary).
// A buffer holds POST-collision populations f*; the pre-collision f^n of a node is pulled from its
// neighbours (streaming, Eq. 5), with halfway bounce-back f_a(x) = f*_opp(a)(x) where x - e_a is
// a solid node. Rows 0 and ny-1 are solid when walls = 1.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Kernel-side parameters, computed once on the host (lbm_api.cpp) from lbm_params.
struct KParams {
    int nx, ny, pitch;      // lattice and row pitch (doubles)
    int walls, ghost;       // solid rows 0 and ny-1; mirrored psi on them
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
};

__device__ __forceinline__ int wrapx(int x, int nx) {
    int r = x % nx;
    return r < 0 ? r + nx : r;
}

// p_EOS(rho) and psi(rho); a negative radicand yields NaN, caught by the observables.
__device__ __forceinline__ double psi_of_rho(const KParams& P, double rho) {
    double p;
    if (P.eos == 0) {
        double eta = P.b4 * rho;
        double om = 1.0 - eta;
        double num = 1.0 + eta * (1.0 + eta * (1.0 - eta));
        p = rho * P.RT * num / (om * om * om) - P.a * rho * rho;
    } else {
        p = rho <= P.rho1 ? rho * P.th_v
          : (rho <= P.rho2 ? P.p1 + (rho - P.rho1) * P.th_m : P.p2 + (rho - P.rho2) * P.th_l);
    }
    return sqrt(P.two_over_G * (p - rho * (1.0 / 3.0)));
}

// Pull the 9 pre-collision populations of fluid node (x, y) from post-collision buffer g.
// Plane bases are uniform (scalar registers) and in-plane offsets 32-bit unsigned, so loads use
// scalar-base + 32-bit vector-offset addressing.
__device__ __forceinline__ void pull9(const KParams& P, const double* __restrict__ g, int x,
                                      int y, double f[9]) {
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
}

// The fluid node whose psi a lattice slot (gx, gy) holds: gx wraps (periodic x); a solid row
// takes the adjacent fluid row (mirrored ghost psi) or nothing (psi = 0); rows outside the
// lattice hold nothing. Returns false when the slot's psi is 0.
__device__ __forceinline__ bool slot_source(const KParams& P, int gx, int gy, int& sx, int& sy) {
    sx = wrapx(gx, P.nx);
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
__device__ __forceinline__ double psi_at(const KParams& P, const double* __restrict__ g, int gx,
                                         int gy) {
    int sx, sy;
    if (!slot_source(P, gx, gy, sx, sy)) return 0.0;
    double f[9];
    pull9(P, g, sx, sy, f);
    return psi_of_rho(P, ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8]);
}

__device__ __forceinline__ double sum9(const double f[9]) {
    return ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
}

// Adhesion sum A = sum over solid neighbours of omega_a G_w(x + e_a) e_a (omega = w/3) at a fluid
// node next to a flat wall; F_ads = -P A with P = rho, psi or psi^2 (Eqs. 10, 11, 14).
__device__ __forceinline__ void adhesion_sum(const KParams& P, const double* __restrict__ gw,
                                             int x, int y, double& Ax, double& Ay) {
    Ax = 0.0; Ay = 0.0;
    if (!P.walls) return;
    const int xm = x == 0 ? P.nx - 1 : x - 1;
    const int xp = x == P.nx - 1 ? 0 : x + 1;
    if (y == 1) {  // bottom wall below: e4 (0,-1) w 1/9, e7 (-1,-1) and e8 (1,-1) w 1/36
        const double gc = gw[x], gm = gw[xm], gp = gw[xp];
        Ax += (gp - gm) * (1.0 / 36.0);
        Ay -= gc * (1.0 / 9.0) + (gm + gp) * (1.0 / 36.0);
    }
    if (y == P.ny - 2) {  // top wall above: e2 (0,1), e5 (1,1), e6 (-1,1)
        const double* gt = gw + P.pitch;  // rows of the G_w array are pitch apart
        const double gc = gt[x], gm = gt[xm], gp = gt[xp];
        Ax += (gp - gm) * (1.0 / 36.0);
        Ay += gc * (1.0 / 9.0) + (gm + gp) * (1.0 / 36.0);
    }
}

// Cohesion stencil sum s = sum_a w_a psi(x + e_a) e_a from the 3x3 neighbourhood
// p[dy][dx] (dy, dx in 0..2 for offsets -1..1).
__device__ __forceinline__ void cohesion_sum(double pmm, double p0m, double ppm, double pm0,
                                             double pp0, double pmp, double p0p, double ppp,
                                             double& sx, double& sy) {
    // axial w = 1/3, diagonal w = 1/12 (Eq. 7)
    const double dpx = ppp - pmm, dmx = ppm - pmp;  // (+1,+1)-(-1,-1), (+1,-1)-(-1,+1)
    sx = (pp0 - pm0) * (1.0 / 3.0) + (dpx + dmx) * (1.0 / 12.0);
    sy = (p0p - p0m) * (1.0 / 3.0) + (dpx - dmx) * (1.0 / 12.0);
}

// Forces, velocity and MRT collision of one node (Eqs. 2-4, 6, 7, 9 and 10/11/14):
// in f[9] (pre-collision), rho, psi_c, cohesion sum (sx, sy), adhesion sum (Ax, Ay);
// out f[9] overwritten with f* = M^-1 m*.
__device__ __forceinline__ void collide(const KParams& P, double f[9], double rho, double psi_c,
                                        double sx, double sy, double Ax, double Ay) {
    // Eq. (7): F_m = -G psi(x) s;  adhesion pre-sum factor
    const double fmx = P.negG * psi_c * sx, fmy = P.negG * psi_c * sy;
    const double pre = P.wall_force == 0 ? rho : (P.wall_force == 1 ? psi_c : psi_c * psi_c);
    const double Fx = fmx - pre * Ax, Fy = fmy - pre * Ay;

    // moments m = M f (rows rho, e, epsilon, jx, qx, jy, qy, pxx, pxy)
    const double ax = f[1] + f[3], ay = f[2] + f[4];
    const double sa = ax + ay;                       // axial sum
    const double sd = (f[5] + f[7]) + (f[6] + f[8]); // diagonal sum
    const double m1 = -4.0 * f[0] - sa + 2.0 * sd;
    const double m2 = 4.0 * f[0] - 2.0 * sa + sd;
    const double d58 = f[5] - f[7], d68 = f[6] - f[8];
    const double jx = (f[1] - f[3]) + d58 - d68;
    const double jy = (f[2] - f[4]) + d58 + d68;
    const double m4 = -2.0 * (f[1] - f[3]) + d58 - d68;
    const double m6 = -2.0 * (f[2] - f[4]) + d58 + d68;
    const double m7 = ax - ay;
    const double m8 = (f[5] + f[7]) - (f[6] + f[8]);

    // Eq. (6): velocity with half the force
    const double ir = 1.0 / rho;
    const double vx = (jx + 0.5 * Fx) * ir, vy = (jy + 0.5 * Fy) * ir;
    const double v2 = vx * vx + vy * vy;

    // shear relaxation rate from the phase-interpolated viscosity
    double snu;
    if (P.visc_const) {
        snu = P.s_nu_c;
    } else {
        double phi = (rho - P.rho_v) * P.inv_drho;
        phi = fmin(fmax(phi, 0.0), 1.0);
        snu = 1.0 / (3.0 * (P.nu_v + phi * P.dnu) + 0.5);
    }
    const double hnu = 1.0 - 0.5 * snu;

    // Eq. (9) forcing; |F_m|^2 / psi^2 = G^2 |s|^2
    const double vF = vx * Fx + vy * Fy;
    const double s2 = sx * sx + sy * sy;
    const double S1 = 6.0 * vF + P.c_sig_e * s2;
    const double S2 = -6.0 * vF - P.c_sig_z * s2;
    const double S7 = 2.0 * (vx * Fx - vy * Fy);
    const double S8 = vx * Fy + vy * Fx;

    // Eq. (4) with Eq. (3) equilibria; m*_0 = rho
    const double ms1 = m1 - P.s_e * (m1 - rho * (-2.0 + 3.0 * v2)) + P.h_e * S1;
    const double ms2 = m2 - P.s_z * (m2 - rho * (1.0 - 3.0 * v2)) + P.h_z * S2;
    const double ms3 = jx - P.s_j * (jx - rho * vx) + P.h_j * Fx;
    const double ms4 = m4 - P.s_q * (m4 + rho * vx) - P.h_q * Fx;
    const double ms5 = jy - P.s_j * (jy - rho * vy) + P.h_j * Fy;
    const double ms6 = m6 - P.s_q * (m6 + rho * vy) - P.h_q * Fy;
    const double ms7 = m7 - snu * (m7 - rho * (vx * vx - vy * vy)) + hnu * S7;
    const double ms8 = m8 - snu * (m8 - rho * vx * vy) + hnu * S8;

    // f* = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m*
    const double a0 = rho * (1.0 / 9.0), a1 = ms1 * (1.0 / 36.0), a2 = ms2 * (1.0 / 36.0);
    const double a3 = ms3 * (1.0 / 6.0), a4 = ms4 * (1.0 / 12.0);
    const double a5 = ms5 * (1.0 / 6.0), a6 = ms6 * (1.0 / 12.0);
    const double a7 = ms7 * 0.25, a8 = ms8 * 0.25;
    const double ba = a0 - a1 - 2.0 * a2, bd = a0 + 2.0 * a1 + a2;
    const double X = a3 + a4, Y = a5 + a6;
    f[0] = a0 - 4.0 * a1 + 4.0 * a2;
    f[1] = ba + a3 - 2.0 * a4 + a7;
    f[3] = ba - a3 + 2.0 * a4 + a7;
    f[2] = ba + a5 - 2.0 * a6 - a7;
    f[4] = ba - a5 + 2.0 * a6 - a7;
    f[5] = bd + X + Y + a8;
    f[6] = bd - X + Y - a8;
    f[7] = bd - X - Y + a8;
    f[8] = bd + X - Y - a8;
}

// Macroscopic velocity of a node (Eq. 6) with the same force as collide().
__device__ __forceinline__ void velocity(const KParams& P, const double f[9], double rho,
                                         double psi_c, double sx, double sy, double Ax,
                                         double Ay, double& vx, double& vy) {
    const double pre = P.wall_force == 0 ? rho : (P.wall_force == 1 ? psi_c : psi_c * psi_c);
    const double Fx = P.negG * psi_c * sx - pre * Ax, Fy = P.negG * psi_c * sy - pre * Ay;
    const double d58 = f[5] - f[7], d68 = f[6] - f[8];
    const double jx = (f[1] - f[3]) + d58 - d68;
    const double jy = (f[2] - f[4]) + d58 + d68;
    const double ir = 1.0 / rho;
    vx = (jx + 0.5 * Fx) * ir;
    vy = (jy + 0.5 * Fy) * ir;
}

// XCD-aware tile order: workgroup i runs on XCD i mod 8; give each XCD a contiguous range of
// tiles so neighbouring tiles (which re-read each other's halo) share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int i, int T) {
    const int q = T >> 3, r = T & 7;
    const int k = i & 7, j = i >> 3;
    return k * q + (k < r ? k : r) + j;
}

}  // namespace lbm
