// lbm_adjoint.hip -- reverse-mode (adjoint) kernels of the wetting LB step and the wetting
// objective, for gradients with respect to the per-wall-node wettability G_w.
//
// Per time step n (forward: g^n = C(pull(g^{n-1}))), with lambda^n = dL/df^n stored as
// lambda = a + c 1 (a: 9 planes, c: one scalar plane), one launch of k_adj per reverse step
// (adj_tile in lbm_device.h): c of the later step is formed on the tile and one ring from its q,
// p0 and psi' (the transpose of the cohesion stencil), then lambda is gathered through the
// transposed pull streaming and bounce-back and the forward node is recomputed from g^{n-1} for
// the reverse mode of the MRT collision (a^{n-1}, q = dL/ds, p0 = dL/dpsi as the node's own
// pre-factor, psi', and r = dL/dA on the wall rows). dL/dG_w accumulates on the solid nodes of
// both walls from each step's r, the last step's by k_adj_gw.
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

template <int TX, int TY, int NTH, int EOS>
__global__ __launch_bounds__(NTH) void k_adj(KParams P, AdjPtrs A) {
    __shared__ AdjLds<TX, TY> lds;
    const int ntx = (P.nx + TX - 1) / TX;
    const int nty = (P.y_hi - P.y_lo + TY) / TY;
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    adj_tile<TX, TY, NTH, EOS>(P, A, (tile % ntx) * TX, P.y_lo + (tile / ntx) * TY, lds);
}

// dL/dG_w of the wall vectors of the last reverse step.
__global__ __launch_bounds__(256) void k_adj_gw(KParams P, const double* __restrict__ rv,
                                                double* __restrict__ gwgrad) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= P.nx || !P.walls) return;
    adj_gw_node(P, rv, gwgrad, x, 1);
    adj_gw_node(P, rv, gwgrad, x, P.ny - 2);
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

// dL/drho^N on every fluid node, the seed of the adjoint: written as the later step's p0 with
// psi' = 1 (and q = 0), so that the first reverse step forms c = 1 * (0 + seed) = seed exactly.
__global__ __launch_bounds__(256) void k_loss_seed(KParams P, double w_c, double w_w, double yc,
                                                   double sum_phi, double* __restrict__ p0,
                                                   double* __restrict__ dpsi) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = P.y_lo + blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= P.nx || y > P.y_hi) return;
    const double d = w_c * ((y - 0.5) - yc) / sum_phi + (y == 1 ? w_w : 0.0);
    p0[(unsigned)y * P.pitch + x] = P.inv_drho * d;
    dpsi[(unsigned)y * P.pitch + x] = 1.0;
}

// ------------------------------------------------------------------------------------------------
static dim3 node_grid_adj(const KParams& P) {
    return dim3((P.nx + 63) / 64, (P.y_hi - P.y_lo + 4) / 4);
}

template <int TX, int TY, int NTH>
static hipError_t launch_adj_t(const KParams& P, const AdjPtrs& A, hipStream_t s) {
    const int ntx = (P.nx + TX - 1) / TX;
    const int nty = (P.y_hi - P.y_lo + TY) / TY;
    if (P.eos == 0)
        hipLaunchKernelGGL((k_adj<TX, TY, NTH, EOS_CS>), dim3(ntx * nty), dim3(NTH), 0, s, P, A);
    else
        hipLaunchKernelGGL((k_adj<TX, TY, NTH, EOS_PW>), dim3(ntx * nty), dim3(NTH), 0, s, P, A);
    return hipGetLastError();
}

// One reverse step. Tiles of 64 x 4 nodes, or on lattices that would give fewer than 512
// workgroups with those, 32 x 4 tiles with two threads per node (the second half of the
// workgroup takes the ring work): 4 waves per workgroup instead of 2, 256 x 128: 37.1 -> 32.5 ms
// for the loss and backward pass of 4,000 steps.
hipError_t launch_adj(const KParams& P, const AdjPtrs& A, hipStream_t s) {
    const int tiles64 = ((P.nx + 63) / 64) * ((P.y_hi - P.y_lo + 4) / 4);
    if (tiles64 < 512) return launch_adj_t<32, 4, 256>(P, A, s);
    return launch_adj_t<64, 4, 256>(P, A, s);
}

hipError_t launch_adj_gw(const KParams& P, const double* rv, double* gwgrad, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_gw, dim3((P.nx + 255) / 256), dim3(256), 0, s, P, rv, gwgrad);
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
                            double* p0, double* dpsi, hipStream_t s) {
    hipLaunchKernelGGL(k_loss_seed, node_grid_adj(P), dim3(256), 0, s, P, w_c, w_w, yc, sum_phi,
                       p0, dpsi);
    return hipGetLastError();
}

}  // namespace lbm
