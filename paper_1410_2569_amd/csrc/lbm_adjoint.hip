// lbm_adjoint.hip -- reverse-mode (adjoint) kernels of the wetting LB step and the wetting
// objective, for gradients with respect to the per-wall-node wettability G_w.
//
// Per time step n (forward: g^n = C(pull(g^{n-1}))), with lambda^n = dL/df^n stored as
// lambda = a + c 1 (a: 9 planes, c: one scalar plane):
//   pass A  (k_adj_local, one thread per fluid node y, tile + halo like the fused forward step):
//           nu = dL/dg^n(y) gathered from (a, c)^{n+1} (transpose of pull streaming and
//           bounce-back), the forward node recomputed from g^{n-1}, then reverse mode through the
//           MRT collision: a^n(y) = dL/df^n(y) along every path except psi, p0 = dL/dpsi(y) as the
//           node's own pre-factor, q = dL/ds for the cohesion sum s = sum w_a psi(y+e_a) e_a,
//           psi'(rho(y)), and r = dL/dA on wall rows.
//   pass B  (k_adj_gather): xi(x) = p0(x) + sum_a w_a e_a . q(x - e_a) (+ the mirrored ghost
//           rows), c^n(x) = psi'(x) xi(x); dL/dG_w(s) += sum_a omega_a e_a . r(s - e_a) on the
//           solid nodes s of both walls.
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

template <int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_adj_local(KParams P, const double* __restrict__ gprev,
                                                      const double* __restrict__ a_in,
                                                      const double* __restrict__ c_in,
                                                      const double* __restrict__ gw,
                                                      double* __restrict__ a_out,
                                                      double* __restrict__ qbuf,
                                                      double* __restrict__ p0buf,
                                                      double* __restrict__ dpsibuf,
                                                      double* __restrict__ rvec) {
    constexpr int NT = TX * TY;
    constexpr int LW = TX + 2;
    constexpr int NH = 2 * LW + 2 * TY;
    __shared__ double sp[(TY + 2) * LW];

    const int ntx = (P.nx + TX - 1) / TX;
    const int nty = (P.y_hi - P.y_lo + TY) / TY;
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    const int x0 = (tile % ntx) * TX;
    const int y0 = P.y_lo + (tile / ntx) * TY;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < P.nx && y <= P.y_hi;

    double f[9];
    double rho = 1.0, psi_c = 0.0;
    if (active) {
        pull9<GEO_ROWS>(P, gprev, x, y, f);
        rho = sum9(f);
        psi_c = psi_of_rho(P, rho);
    }
    sp[(ty + 1) * LW + tx + 1] = active ? psi_c : psi_at<GEO_ROWS>(P, gprev, x, y);
    for (int h = threadIdx.x; h < NH; h += NT) {
        int hx, hy;
        if (h < LW) { hx = h - 1; hy = -1; }
        else if (h < 2 * LW) { hx = h - LW - 1; hy = TY; }
        else if (h < 2 * LW + TY) { hx = -1; hy = h - 2 * LW; }
        else { hx = TX; hy = h - 2 * LW - TY; }
        sp[(hy + 1) * LW + hx + 1] = psi_at<GEO_ROWS>(P, gprev, x0 + hx, y0 + hy);
    }
    __syncthreads();
    if (!active) return;

    const double* cc = sp + (ty + 1) * LW + tx + 1;
    double sx, sy;
    cohesion_sum(cc[-LW - 1], cc[-LW], cc[-LW + 1], cc[-1], cc[1], cc[LW - 1], cc[LW],
                 cc[LW + 1], sx, sy);
    double Ax = 0.0, Ay = 0.0;
    const bool wall_row = P.walls && (y == 1 || y == P.ny - 2);
    if (wall_row) adhesion_sum(P, gw, x, y, Ax, Ay);

    double nu[9], fb[9], pb, qx, qy, rx, ry;
    push_gather(P, a_in, c_in, x, y, nu);
    collide_adj(P, f, rho, psi_c, sx, sy, Ax, Ay, nu, fb, pb, qx, qy, rx, ry);

    const unsigned i = (unsigned)y * P.pitch + x;
#pragma unroll
    for (int k = 0; k < 9; ++k) (a_out + k * P.plane)[i] = fb[k];
    qbuf[i] = qx;
    (qbuf + P.plane)[i] = qy;
    p0buf[i] = pb;
    dpsibuf[i] = dpsi_drho(P, rho, psi_c);
    if (wall_row) {
        if (y == 1) { rvec[x] = rx; rvec[P.pitch + x] = ry; }
        if (y == P.ny - 2) { rvec[2 * P.pitch + x] = rx; rvec[3 * P.pitch + x] = ry; }
    }
}

__global__ __launch_bounds__(256) void k_adj_gather(KParams P, const double* __restrict__ qbuf,
                                                    const double* __restrict__ p0buf,
                                                    const double* __restrict__ dpsibuf,
                                                    const double* __restrict__ rvec,
                                                    double* __restrict__ c_out,
                                                    double* __restrict__ gwgrad) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = P.y_lo + blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= P.nx || y > P.y_hi) return;
    const unsigned pitch = P.pitch;
    const unsigned ux = x;
    const unsigned xm = ux == 0 ? P.nx - 1 : ux - 1;
    const unsigned xp = ux == (unsigned)P.nx - 1 ? 0 : ux + 1;
    unsigned ym, yp;
    if (P.walls) { ym = y - 1; yp = y + 1; }  // solid rows of q hold 0
    else { ym = y == 0 ? P.ny - 1 : y - 1; yp = y == P.ny - 1 ? 0 : y + 1; }
    const double* qx = qbuf;
    const double* qy = qbuf + P.plane;
    const unsigned r0 = (unsigned)y * pitch, rm = ym * pitch, rp = yp * pitch;
    // sum over a of w_a e_a . q(x - e_a)
    double xi = (qx[r0 + xm] - qx[r0 + xp] + qy[rm + ux] - qy[rp + ux]) * (1.0 / 3.0) +
                ((qx[rm + xm] + qy[rm + xm]) + (qy[rm + xp] - qx[rm + xp]) -
                 (qx[rp + xp] + qy[rp + xp]) + (qx[rp + xm] - qy[rp + xm])) * (1.0 / 12.0);
    if (P.walls && P.ghost) {
        // the solid row next to the wall carries this row's psi (mirror ghost)
        if (y == 1)
            xi += -qy[r0 + ux] * (1.0 / 3.0) +
                  ((-qx[r0 + xp] - qy[r0 + xp]) + (qx[r0 + xm] - qy[r0 + xm])) * (1.0 / 12.0);
        if (y == P.ny - 2)
            xi += qy[r0 + ux] * (1.0 / 3.0) +
                  ((qx[r0 + xm] + qy[r0 + xm]) + (qy[r0 + xp] - qx[r0 + xp])) * (1.0 / 12.0);
    }
    xi += p0buf[r0 + ux];
    c_out[r0 + ux] = dpsibuf[r0 + ux] * xi;

    if (P.walls) {
        // dL/dG_w of the solid node beside this fluid node (omega = w/3: 1/9 axial, 1/36 diagonal)
        if (y == 1) {
            const double* rX = rvec;
            const double* rY = rvec + pitch;
            gwgrad[ux] += -rY[ux] * (1.0 / 9.0) +
                          ((-rX[xp] - rY[xp]) + (rX[xm] - rY[xm])) * (1.0 / 36.0);
        }
        if (y == P.ny - 2) {
            const double* rX = rvec + 2 * pitch;
            const double* rY = rvec + 3 * pitch;
            gwgrad[pitch + ux] += rY[ux] * (1.0 / 9.0) +
                                  ((rX[xm] + rY[xm]) + (rY[xp] - rX[xp])) * (1.0 / 36.0);
        }
    }
}

// ------------------------------------------------------------------------------------------------
// Wetting objective: phi = (rho - rho_v)/(rho_l - rho_v); L = w_c y_c + w_w l_w with
// y_c = sum phi (y - 1/2) / sum phi and l_w = sum_x phi(x, 1). Partial sums per block.
// ------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_loss_partial(KParams P, const double* __restrict__ g,
                                                      double* __restrict__ part) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = P.y_lo + blockIdx.y * 4 + (threadIdx.x >> 6);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (x < P.nx && y <= P.y_hi) {
        double f[9];
        pull9<GEO_ROWS>(P, g, x, y, f);
        const double phi = (sum9(f) - P.rho_v) * P.inv_drho;
        s0 = phi;
        s1 = phi * (y - 0.5);
        s2 = y == 1 ? phi : 0.0;
    }
    __shared__ double red[4][3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_xor(s0, off, 64);
        s1 += __shfl_xor(s1, off, 64);
        s2 += __shfl_xor(s2, off, 64);
    }
    if (lane == 0) { red[wv][0] = s0; red[wv][1] = s1; red[wv][2] = s2; }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int q = threadIdx.x;
        part[(long long)(blockIdx.y * gridDim.x + blockIdx.x) * 3 + q] =
            (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    }
}

// Fixed-order sums of nq quantities over nblk partial rows (one block of 256 threads).
__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ part, int nblk,
                                                   int nq, double* __restrict__ out) {
    __shared__ double sh[256];
    for (int q = 0; q < nq; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 256) s += part[(long long)b * nq + q];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = sh[0];
        __syncthreads();
    }
}

// dL/drho^N on every fluid node: the seed of the adjoint (stored as the scalar plane c).
__global__ __launch_bounds__(256) void k_loss_seed(KParams P, double w_c, double w_w, double yc,
                                                   double sum_phi, double* __restrict__ c) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = P.y_lo + blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= P.nx || y > P.y_hi) return;
    const double d = w_c * ((y - 0.5) - yc) / sum_phi + (y == 1 ? w_w : 0.0);
    c[(unsigned)y * P.pitch + x] = P.inv_drho * d;
}

// ------------------------------------------------------------------------------------------------
static dim3 node_grid_adj(const KParams& P) {
    return dim3((P.nx + 63) / 64, (P.y_hi - P.y_lo + 4) / 4);
}

hipError_t launch_adj_step(const KParams& P, const double* gprev, const double* a_in,
                           const double* c_in, const double* gw, double* a_out, double* qbuf,
                           double* p0buf, double* dpsibuf, double* rvec, double* c_out,
                           double* gwgrad, hipStream_t s) {
    constexpr int TX = 64, TY = 4;
    const int ntx = (P.nx + TX - 1) / TX;
    const int nty = (P.y_hi - P.y_lo + TY) / TY;
    hipLaunchKernelGGL((k_adj_local<TX, TY>), dim3(ntx * nty), dim3(TX * TY), 0, s, P, gprev,
                       a_in, c_in, gw, a_out, qbuf, p0buf, dpsibuf, rvec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_gather, node_grid_adj(P), dim3(256), 0, s, P, qbuf, p0buf, dpsibuf,
                       rvec, c_out, gwgrad);
    return hipGetLastError();
}

int loss_blocks(const KParams& P) {
    dim3 g = node_grid_adj(P);
    return (int)(g.x * g.y);
}

hipError_t launch_loss(const KParams& P, const double* g, double* part, double* out,
                       hipStream_t s) {
    dim3 gr = node_grid_adj(P);
    hipLaunchKernelGGL(k_loss_partial, gr, dim3(256), 0, s, P, g, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, part, (int)(gr.x * gr.y), 3, out);
    return hipGetLastError();
}

hipError_t launch_loss_seed(const KParams& P, double w_c, double w_w, double yc, double sum_phi,
                            double* c, hipStream_t s) {
    hipLaunchKernelGGL(k_loss_seed, node_grid_adj(P), dim3(256), 0, s, P, w_c, w_w, yc, sum_phi,
                       c);
    return hipGetLastError();
}

}  // namespace lbm
