// lbm_kernels.hip -- gfx950 kernels of the wetting pseudopotential LB step and its observables.
//
// Step schedules (both call the same per-node arithmetic of lbm_device.h):
//   fused     one kernel per time step. A workgroup owns a TX x TY tile; every thread pulls the
//             9 populations of its node (Eq. 5 with bounce-back), forms rho and psi, and the
//             psi of the one-node tile halo is recomputed from the (L2-resident) populations of
//             the neighbouring tiles. psi lives only in LDS, so HBM sees 72 B read + 72 B
//             written per lattice update.
//   two-pass  psi pass (pull, rho, psi -> psi array with mirrored ghost rows), then the step
//             kernel stages the psi tile plus halo in LDS: 72 + 8 B and 72 + 8 + 72 B per update.
//   two-step  two time steps per launch with the intermediate state in LDS (step2_tile).
// With the wet-node wall scheme the boundary nodes also write their force (16 B) to the solid row,
// which the next pull reads back; that traffic is confined to two rows of the lattice.
#include <algorithm>
#include <type_traits>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

// ------------------------------------------------------------------------------------------------
// Time step
// ------------------------------------------------------------------------------------------------
// GEO, EOS: the geometry and equation-of-state variants compiled in, chosen at launch.
template <int TX, int TY, bool FUSED, int GEO, int EOS>
__global__ __launch_bounds__(TX* TY) void k_step(KParams P, const double* __restrict__ gin,
                                                 double* __restrict__ gout,
                                                 const double* __restrict__ psi_g,
                                                 const double* __restrict__ gw) {
    __shared__ double sp[(TY + 2) * (TX + 2)];
    const int ntx = (P.nx + TX - 1) / TX;
    const int nty = (P.y_hi - P.y_lo + TY) / TY;
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    step_tile<TX, TY, FUSED, GEO, EOS>(P, gin, gout, psi_g, gw, (tile % ntx) * TX,
                                       P.y_lo + (tile / ntx) * TY, sp);
}

// Overlapped tiles: one 64-lane wave spans TXI = 62 interior columns plus the halo column on each
// side, and the workgroup has TYI interior rows plus a halo row above and below. Every thread
// pulls exactly one node and evaluates its psi (one memory round trip per tile, all loads
// coalesced rows); the interior threads then collide and store.
template <int TYI, int GEO, int EOS>
__global__ __launch_bounds__(64 * (TYI + 2)) void k_step_ov(KParams P,
                                                            const double* __restrict__ gin,
                                                            double* __restrict__ gout,
                                                            const double* __restrict__ gw) {
    constexpr int TXI = 62, LW = 64;
    __shared__ double sp[(TYI + 2) * LW];
    const int ntx = (P.nx + TXI - 1) / TXI;
    const int nty = (P.y_hi - P.y_lo + TYI) / TYI;
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    const int x0 = (tile % ntx) * TXI;
    const int y0 = P.y_lo + (tile / ntx) * TYI;
    const int l = threadIdx.x & 63, r = threadIdx.x >> 6;
    const int gx = x0 - 1 + l, gy = y0 - 1 + r;
    const bool interior = l >= 1 && l <= TXI && r >= 1 && r <= TYI && gx < P.nx && gy <= P.y_hi;

    int sx, sy;
    const bool has = slot_source(P, gx, gy, sx, sy);
    double f[9];
    double rho = 1.0, psi_c = 0.0;
    if (has) {
        pull9<GEO>(P, gin, sx, sy, f);
        rho = sum9(f);
        psi_c = psi_of_rho<EOS>(P, rho);
    }
    sp[r * LW + l] = psi_c;
    __syncthreads();
    if (!interior) return;

    const double* c = sp + r * LW + l;
    double sxx, syy;
    cohesion_sum(c[-LW - 1], c[-LW], c[-LW + 1], c[-1], c[1], c[LW - 1], c[LW], c[LW + 1], sxx,
                 syy);
    double Ax = 0.0, Ay = 0.0;
    if (P.walls && (gy == 1 || gy == P.ny - 2)) adhesion_sum(P, gw, gx, gy, Ax, Ay);
    store_wall_force<GEO>(P, gout, (long long)gy * P.pitch + gx, P.plane, P.pitch, gy, rho, psi_c,
                          sxx, syy, Ax, Ay);
    collide(P, f, rho, psi_c, sxx, syy, Ax, Ay);
    const unsigned i = (unsigned)gy * P.pitch + gx;
#pragma unroll
    for (int a = 0; a < 9; ++a) (gout + a * P.plane)[i] = f[a];
}

// Two steps per launch over TX x TY output tiles (step2_tile) with NTH threads; MID: the state
// after the first step is written to gmid as well.
template <int TX, int TY, int GEO, int EOS, bool MID, int NTH = step2_threads(TX, TY, GEO)>
__global__ __launch_bounds__(NTH, NTH == step2_threads(TX, TY, GEO)
                                      ? step2_waves(TX, TY, GEO)
                                      : (NTH / 64 + 3) / 4) void k_step2(
    KParams P, const double* __restrict__ gin, double* __restrict__ gout,
    const double* __restrict__ gw, double* __restrict__ gmid) {
    __shared__ Step2Lds<TX, TY, GEO> lds;
    const int ntx = (P.nx + TX - 1) / TX;
    const int nty = (P.y_hi - P.y_lo + TY) / TY;
    const int tile = xcd_tile(blockIdx.x, ntx * nty);
    step2_tile_any<TX, TY, GEO, EOS, MID, false, NTH>(P, gin, gout, gw, (tile % ntx) * TX,
                                                      P.y_lo + (tile / ntx) * TY, lds, gmid);
}

// psi pass of the two-pass schedule; also writes the mirrored ghost rows. PRE: gin holds
// pre-collision populations.
template <bool PRE = false>
__global__ __launch_bounds__(256) void k_psi(KParams P, const double* __restrict__ gin,
                                             double* __restrict__ psi_g,
                                             double* __restrict__ rho_out) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = P.y_lo + blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= P.nx || y > P.y_hi) return;
    psi_node<PRE>(P, gin, psi_g, rho_out, x, y);
}

// ------------------------------------------------------------------------------------------------
// State set-up and read-out
// ------------------------------------------------------------------------------------------------

// Inverse of streaming + bounce-back: writes g so that the first pull yields f_a = t_a rho0.
// Every post-collision slot of a fluid node is the source of exactly one pulled population.
__global__ __launch_bounds__(256) void k_init(KParams P, const double* __restrict__ rho0,
                                              double* __restrict__ g) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = P.y_lo + blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= P.nx || y > P.y_hi) return;
    if (is_solid_node(P, x, y)) return;
    const double r = rho0[(long long)y * P.pitch + x];
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    const int op[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    const unsigned lk = P.mask ? P.links[(unsigned)y * P.pitch + x] : 0u;
    for (int a = 0; a < 9; ++a) {
        const double t = a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        int sx = wrapx(x - ex[a], P.nx);
        int sy = y - ey[a];
        bool solid = false;
        if (P.mask) { solid = (lk >> a) & 1u; sy = wrapx(sy, P.ny); }
        else if (P.walls) solid = (sy == 0 || sy == P.ny - 1);
        else sy = wrapx(sy, P.ny);
        if (solid) g[op[a] * P.plane + (long long)y * P.pitch + x] = t * r;
        else g[a * P.plane + (long long)sy * P.pitch + sx] = t * r;
    }
}

// Pre-collision populations f^n (pulled) into a [9][ny][pitch] buffer, or with `dense` a
// [9][ny][nx] one.
__global__ __launch_bounds__(256) void k_pull(KParams P, const double* __restrict__ gin,
                                              double* __restrict__ fout, int dense) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = P.y_lo + blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= P.nx || y > P.y_hi || is_solid_node(P, x, y)) return;
    double f[9];
    pull9_any(P, gin, x, y, f);
    const long long pl = dense ? (long long)P.nx * P.ny : P.plane;
    const long long i = dense ? (long long)y * P.nx + x : (long long)y * P.pitch + x;
    for (int a = 0; a < 9; ++a) fout[a * pl + i] = f[a];
}

// Copy of `planes` planes of ny rows of nx doubles between two layouts in device memory: rows
// src_pitch doubles apart (planes src_plane apart) to rows dst_pitch apart (planes dst_plane
// apart). Host data enter and leave the library densely packed through it, so that every copy
// between host and device memory is one contiguous transfer.
__global__ __launch_bounds__(256) void k_repack(const double* __restrict__ src, long long src_plane,
                                                int src_pitch, double* __restrict__ dst,
                                                long long dst_plane, int dst_pitch, int nx,
                                                int ny, int planes) {
    const long long per = (long long)ny * nx, n = per * planes;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (long long)gridDim.x * 256) {
        const long long a = i / per, r = i - a * per;
        const long long y = r / nx, x = r - y * nx;
        dst[a * dst_plane + y * dst_pitch + x] = src[a * src_plane + y * src_pitch + x];
    }
}

// ------------------------------------------------------------------------------------------------
// Observables: per-block partials (wave-level shuffles, then LDS across waves), fixed-order final
// reduction. No floating-point atomics, so results are bitwise reproducible.
// ------------------------------------------------------------------------------------------------
// Block of 256 threads over a 64 x 4 patch. rho_f: rho of every fluid node (from k_psi);
// psi_g: psi with ghost rows. Writes O_NQ partials per block. PRE: gin holds pre-collision
// populations.
template <bool PRE = false>
__global__ __launch_bounds__(256) void k_obs(KParams P, const double* __restrict__ gin,
                                             const double* __restrict__ rho_f,
                                             const double* __restrict__ psi_g,
                                             const double* __restrict__ gw, ObsArgs A,
                                             double* __restrict__ part) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = P.y_lo + blockIdx.y * 4 + (threadIdx.x >> 6);
    double v[O_NQ];
    for (int q = 0; q < O_NQ; ++q) v[q] = op_identity(q);
    if (x < P.nx && y <= P.y_hi) obs_node<PRE>(P, gin, rho_f, psi_g, gw, A, x, y, v);
    // wave-level tree (xor shuffles), then across the 4 waves of the block
    __shared__ double red[4][O_NQ];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q = 0; q < O_NQ; ++q) {
        double s = v[q];
        for (int off = 32; off > 0; off >>= 1) s = op_combine(q, s, __shfl_xor(s, off, 64));
        if (lane == 0) red[wv][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < O_NQ) {
        const int q = threadIdx.x;
        double s = op_combine(q, op_combine(q, red[0][q], red[1][q]),
                              op_combine(q, red[2][q], red[3][q]));
        part[(long long)(blockIdx.y * gridDim.x + blockIdx.x) * O_NQ + q] = s;
    }
}

// One block of 256 threads: for every quantity, thread t combines partials t, t+256, ... in
// order, then a fixed tree; all quantities advance together (one pass over the partial rows).
__global__ __launch_bounds__(256) void k_obs_final(const double* __restrict__ part, int nblk,
                                                   double* __restrict__ out) {
    __shared__ double sh[O_NQ][256];
    double s[O_NQ];
#pragma unroll
    for (int q = 0; q < O_NQ; ++q) s[q] = op_identity(q);
    for (int b = threadIdx.x; b < nblk; b += 256) {
        const double* r = part + (long long)b * O_NQ;
#pragma unroll
        for (int q = 0; q < O_NQ; ++q) s[q] = op_combine(q, s[q], r[q]);
    }
#pragma unroll
    for (int q = 0; q < O_NQ; ++q) sh[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < O_NQ; ++q)
                sh[q][threadIdx.x] = op_combine(q, sh[q][threadIdx.x], sh[q][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < O_NQ) out[threadIdx.x] = sh[threadIdx.x][0];
}

// Contact line of one lattice (contact_line_block).
__global__ __launch_bounds__(256) void k_contact_line(KParams P, const double* __restrict__ gin,
                                                      int row, double mid,
                                                      double* __restrict__ out) {
    contact_line_block(P, gin, row, mid, out);
}

// Zero fill of n 8-byte words (grid-stride). The library clears its buffers with this kernel
// rather than a runtime memset, so the clear is ordered like every other kernel of the stream.
__global__ __launch_bounds__(256) void k_zero(unsigned long long* __restrict__ p, size_t n) {
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

// ------------------------------------------------------------------------------------------------
// Host-side launchers
// ------------------------------------------------------------------------------------------------
static dim3 node_grid(const KParams& P) {
    return dim3((P.nx + 63) / 64, (P.y_hi - P.y_lo + 4) / 4);
}

// Calls f(geo, eos) with the geometry and equation of state of P as compile-time constants.
template <class F>
static hipError_t dispatch(const KParams& P, F&& f) {
    auto with_eos = [&](auto geo) {
        if (P.eos == 0) return f(geo, std::integral_constant<int, EOS_CS>{});
        return f(geo, std::integral_constant<int, EOS_PW>{});
    };
    if (P.mask) return with_eos(std::integral_constant<int, GEO_MASK>{});
    if (P.wet) return with_eos(std::integral_constant<int, GEO_WET>{});
    return with_eos(std::integral_constant<int, GEO_ROWS>{});
}

template <int TX, int TY, bool FUSED>
static hipError_t launch_step_t(const KParams& P, const double* gin, double* gout,
                                const double* psi, const double* gw, hipStream_t s) {
    const int ntx = (P.nx + TX - 1) / TX;
    const int nty = (P.y_hi - P.y_lo + TY) / TY;
    return dispatch(P, [&](auto geo, auto eos) {
        hipLaunchKernelGGL((k_step<TX, TY, FUSED, decltype(geo)::value, decltype(eos)::value>),
                           dim3(ntx * nty), dim3(TX * TY), 0, s, P, gin, gout, psi, gw);
        return hipGetLastError();
    });
}

// The overlapped tiles have no solid-mask variant (the API rejects those schedules for a
// mask).
template <int TYI>
static hipError_t launch_step_ov(const KParams& P, const double* gin, double* gout,
                                 const double* gw, hipStream_t s) {
    const int ntx = (P.nx + 61) / 62;
    const int nty = (P.y_hi - P.y_lo + TYI) / TYI;
    return dispatch(P, [&](auto geo, auto eos) {
        if constexpr (decltype(geo)::value == GEO_MASK) {
            return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((k_step_ov<TYI, decltype(geo)::value, decltype(eos)::value>),
                               dim3(ntx * nty), dim3(64 * (TYI + 2)), 0, s, P, gin, gout, gw);
            return hipGetLastError();
        }
    });
}

template <int TX, int TY, bool WIDE = false>
static hipError_t launch_step2_t(const KParams& P, const double* gin, double* gout,
                                 const double* gw, double* gmid, hipStream_t s) {
    const int ntx = (P.nx + TX - 1) / TX;
    const int nty = (P.y_hi - P.y_lo + TY) / TY;
    return dispatch(P, [&](auto geo, auto eos) {
        constexpr int G = decltype(geo)::value;
        constexpr int E = decltype(eos)::value;
        constexpr int NT = WIDE ? step2_wide_threads(TX, TY) : step2_threads(TX, TY, G);
        if (!gmid) {
            hipLaunchKernelGGL((k_step2<TX, TY, G, E, false, NT>), dim3(ntx * nty), dim3(NT), 0,
                               s, P, gin, gout, gw, (double*)nullptr);
            return hipGetLastError();
        }
        if constexpr (G == GEO_ROWS) {
            hipLaunchKernelGGL((k_step2<TX, TY, G, E, true, NT>), dim3(ntx * nty), dim3(NT), 0,
                               s, P, gin, gout, gw, gmid);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;  // intermediate states: bounce-back or periodic rows only
        }
    });
}

// Two steps in one launch; tile2 selects the output tile: 0 64x8, 1 64x4, 2 128x4, 3 64x16,
// 4 32x8, 5 32x4 (the narrow tiles for lattices too small to fill the chip with the others), 6
// 64x4 and 7 32x4 with wide workgroups (step2_wide_threads).
// gmid (optional): receives the state after the first step.
hipError_t launch_step2(const KParams& P, int tile2, const double* gin, double* gout,
                        const double* gw, hipStream_t s, double* gmid) {
    switch (tile2) {
        case 1: return launch_step2_t<64, 4>(P, gin, gout, gw, gmid, s);
        case 2: return launch_step2_t<128, 4>(P, gin, gout, gw, gmid, s);
        case 3: return launch_step2_t<64, 16>(P, gin, gout, gw, gmid, s);
        case 4: return launch_step2_t<32, 8>(P, gin, gout, gw, gmid, s);
        case 5: return launch_step2_t<32, 4>(P, gin, gout, gw, gmid, s);
        case 6: return launch_step2_t<64, 4, true>(P, gin, gout, gw, gmid, s);
        case 7: return launch_step2_t<32, 4, true>(P, gin, gout, gw, gmid, s);
        default: return launch_step2_t<64, 8>(P, gin, gout, gw, gmid, s);
    }
}

// Fused tile shapes: 0-3 halo-recompute tiles TX x TY; 4-7 overlapped tiles 62 x TYI.
static const int kTiles[8][3] = {{64, 4, 0}, {64, 8, 0}, {64, 16, 0}, {128, 4, 0},
                                 {62, 4, 1}, {62, 6, 1}, {62, 8, 1}, {62, 14, 1}};

int n_tiles() { return 8; }

void tile_shape(int tile, int* tx, int* ty) {
    if (tile < 0 || tile >= 8) tile = 0;
    *tx = kTiles[tile][0];
    *ty = kTiles[tile][1];
}

hipError_t launch_step(const KParams& P, int schedule, int tile, const double* gin, double* gout,
                       double* psi, const double* gw, hipStream_t s) {
    if (schedule == 1) {
        hipLaunchKernelGGL(k_psi<false>, node_grid(P), dim3(256), 0, s, P, gin, psi,
                           (double*)nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_step_t<64, 4, false>(P, gin, gout, psi, gw, s);
    }
    switch (tile) {
        case 1: return launch_step_t<64, 8, true>(P, gin, gout, psi, gw, s);
        case 2: return launch_step_t<64, 16, true>(P, gin, gout, psi, gw, s);
        case 3: return launch_step_t<128, 4, true>(P, gin, gout, psi, gw, s);
        case 4: return launch_step_ov<4>(P, gin, gout, gw, s);
        case 5: return launch_step_ov<6>(P, gin, gout, gw, s);
        case 6: return launch_step_ov<8>(P, gin, gout, gw, s);
        case 7: return launch_step_ov<14>(P, gin, gout, gw, s);
        default: return launch_step_t<64, 4, true>(P, gin, gout, psi, gw, s);
    }
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes % 8 || ((uintptr_t)p) % 8) return hipErrorInvalidValue;
    const size_t n = bytes / 8;
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, (unsigned long long*)p, n);
    return hipGetLastError();
}

// SplitMix64 (S. Vigna's public-domain mixer): add the golden-ratio increment, then two
// xor-shift-multiply rounds and a final xor-shift, all modulo 2^64.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Initial density of liquid droplets in their vapour on every node of the lattice (pitched
// rows): the largest of the droplets' tanh profiles, times 1 + jitter (2u - 1) with u the
// node's uniform of the seeded counter stream; 0 on solid rows.
__global__ __launch_bounds__(256) void k_droplets(KParams P, DropletArgs D, double* __restrict__ rho) {
#pragma clang fp contract(off)
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= P.nx || y >= P.ny) return;
    double v = 0.0;
    if (y >= P.y_lo && y <= P.y_hi) {
        v = -INFINITY;
        for (int k = 0; k < D.count; ++k) {
            const double dx = x - D.x0[k], dy = y - D.y0[k];
            const double d = sqrt(dx * dx + dy * dy);
            const double rk = D.mid - D.half * tanh(2.0 * (d - D.r[k]) / D.width);
            v = fmax(v, rk);
        }
        if (D.jitter != 0.0) {
            const unsigned long long z =
                splitmix64(D.base + (unsigned long long)y * (unsigned long long)P.nx + x);
            const double u = (double)(z >> 11) * 0x1.0p-53;
            v = v * (1.0 + D.jitter * (2.0 * u - 1.0));
        }
    }
    rho[(long long)y * P.pitch + x] = v;
}

hipError_t launch_droplets(const KParams& P, const DropletArgs& D, double* rho, hipStream_t s) {
    hipLaunchKernelGGL(k_droplets, dim3((P.nx + 63) / 64, (P.ny + 3) / 4), dim3(256), 0, s, P, D,
                       rho);
    return hipGetLastError();
}

// The device's FP64 square root and division as the step kernels compile them: sq = sqrt(a),
// quot = a / b, element-wise.
__global__ __launch_bounds__(256) void k_fp64_probe(const double* __restrict__ a,
                                                    const double* __restrict__ b,
                                                    double* __restrict__ sq,
                                                    double* __restrict__ quot, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    sq[i] = sqrt(a[i]);
    quot[i] = a[i] / b[i];
}

hipError_t launch_fp64_probe(const double* a, const double* b, double* sq, double* quot,
                             long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fp64_probe, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b,
                       sq, quot, n);
    return hipGetLastError();
}

hipError_t launch_init(const KParams& P, const double* rho0, double* g, hipStream_t s) {
    hipLaunchKernelGGL(k_init, node_grid(P), dim3(256), 0, s, P, rho0, g);
    return hipGetLastError();
}

hipError_t launch_pull(const KParams& P, const double* gin, double* fout, hipStream_t s,
                       bool dense) {
    hipLaunchKernelGGL(k_pull, node_grid(P), dim3(256), 0, s, P, gin, fout, dense ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_repack(const double* src, long long src_plane, int src_pitch, double* dst,
                         long long dst_plane, int dst_pitch, int nx, int ny, int planes,
                         hipStream_t s) {
    const long long n = (long long)planes * ny * nx;
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_repack, dim3(blocks), dim3(256), 0, s, src, src_plane, src_pitch, dst,
                       dst_plane, dst_pitch, nx, ny, planes);
    return hipGetLastError();
}

hipError_t launch_rho_psi(const KParams& P, const double* gin, double* psi, double* rho,
                          hipStream_t s, bool pre) {
    if (pre) hipLaunchKernelGGL(k_psi<true>, node_grid(P), dim3(256), 0, s, P, gin, psi, rho);
    else hipLaunchKernelGGL(k_psi<false>, node_grid(P), dim3(256), 0, s, P, gin, psi, rho);
    return hipGetLastError();
}

hipError_t launch_contact_line(const KParams& P, const double* gin, int row, double mid,
                               double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_contact_line, dim3(1), dim3(256), 0, s, P, gin, row, mid, out);
    return hipGetLastError();
}

int obs_blocks(const KParams& P) {
    dim3 g = node_grid(P);
    return (int)(g.x * g.y);
}

hipError_t launch_obs(const KParams& P, const double* gin, const double* rho, const double* psi,
                      const double* gw, const ObsArgs& A, double* part, double* out,
                      hipStream_t s, bool pre) {
    dim3 g = node_grid(P);
    if (pre) hipLaunchKernelGGL(k_obs<true>, g, dim3(256), 0, s, P, gin, rho, psi, gw, A, part);
    else hipLaunchKernelGGL(k_obs<false>, g, dim3(256), 0, s, P, gin, rho, psi, gw, A, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(256), 0, s, part, (int)(g.x * g.y), out);
    return hipGetLastError();
}

}  // namespace lbm
