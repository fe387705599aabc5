// lbm_batch.hip -- ensembles of uneven lattices advanced together.
//
// The tiles of every instance form one flattened work-list. Two schedules run the same per-tile
// device function as the single-instance step (so results are bitwise identical to it):
//   per-step   one launch per time step over the whole work-list (replayed from a hipGraph);
//   persistent one launch for n steps: an occupancy-sized grid whose workgroups take the tiles
//              of their XCD's share of the work-list from a ticket counter and advance each
//              tile two steps (step2_tile), with a grid barrier between the two-step passes
//              (an odd last step is one per-step launch after it). The barrier publishes the
//              pass's stores at agent scope (release), waits for every workgroup, then
//              acquires, through one leader per XCD after the first pass; its 64-bit counters
//              cannot wrap, and its waits are bounded and raise an abort flag on timeout so
//              every workgroup always exits.
#include <algorithm>
#include <type_traits>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

// A pointer read from an instance descriptor, known to address global memory: loads and stores
// through it compile to global (not flat) instructions, which do not share the LDS wait counter.
template <class T>
__device__ __forceinline__ T* gptr(T* p) {
    return (T*)(__attribute__((address_space(1))) T*)(unsigned long long)p;
}

__device__ __forceinline__ void batch_tile_origin(const InstDesc* D, int t, int TX, int TY,
                                                  int& x0, int& y0) {
    const int lt = t - D->tile0;
    x0 = (lt % D->ntx) * TX;
    y0 = D->P.y_lo + (lt / D->ntx) * TY;
}

// GEO: GEO_MASK for an ensemble of solid masks, GEO_WET when some instance uses the wet-node
// wall, else GEO_ROWS; EOS: the equation of state shared by every instance, or EOS_ANY (chosen at
// launch).
template <int TX, int TY, int GEO, int EOS>
__global__ __launch_bounds__(TX* TY) void k_batch_step(const InstDesc* __restrict__ inst,
                                                       const int* __restrict__ tile_inst,
                                                       int ntiles, int cur) {
    __shared__ double sp[(TY + 2) * (TX + 2)];
    const int t = xcd_tile(blockIdx.x, ntiles);
    const InstDesc* D = inst + tile_inst[t];
    int x0, y0;
    batch_tile_origin(D, t, TX, TY, x0, y0);
    step_tile<TX, TY, true, GEO, EOS>(D->P, D->g[cur], D->g[cur ^ 1], nullptr, D->gw, x0, y0, sp);
}

// Two steps per launch over the work-list (the tiles are the output tiles of step2_tile), NTH
// threads per workgroup.
template <int TX, int TY, int GEO, int EOS, int NTH = step2_threads(TX, TY, GEO)>
__global__ __launch_bounds__(NTH, NTH == step2_threads(TX, TY, GEO) ? step2_waves(TX, TY, GEO)
                                                                    : (NTH / 64 + 3) / 4) void
k_batch_step2(
    const InstDesc* __restrict__ inst, const int* __restrict__ tile_inst, int ntiles, int cur) {
    __shared__ Step2Lds<TX, TY, GEO> lds;
    const int t = xcd_tile(blockIdx.x, ntiles);
    const InstDesc* D = inst + tile_inst[t];
    int x0, y0;
    batch_tile_origin(D, t, TX, TY, x0, y0);
    step2_tile_any<TX, TY, GEO, EOS, false, false, NTH>(D->P, gptr(D->g[cur]), gptr(D->g[cur ^ 1]),
                                                        gptr(D->gw), x0, y0, lds);
}

// Bounded wait (thread 0 of a workgroup) until *ctr >= target. Returns 0 when the run was
// aborted: by another workgroup's flag, or here after spin_limit polls, raising the flag.
__device__ __forceinline__ int spin_until(unsigned long long* ctr, unsigned long long target,
                                          int* flag, int spin_limit) {
    for (int n = 0;; ++n) {
        if (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) return 1;
        if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return 0;
        if (n >= spin_limit) {
            __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return 0;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Grid-wide barrier number `target / gridDim.x` on a 64-bit arrival counter: every workgroup
// releases and acquires at agent scope itself. Returns false when the run was aborted.
// Every wave waits for its own global stores of the pass to reach the L2 before the workgroup
// barrier: the barrier alone orders them for the workgroup's waves (which share the compute
// unit's write-through L1), not for a release that thread 0 then makes for all of them.
__device__ __forceinline__ void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ bool grid_barrier(unsigned long long* bar, unsigned long long target,
                                             int* flag, int spin_limit, int* go_on) {
    stores_done();
    __syncthreads();  // every wave's stores of this pass have reached the L2
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int ok = spin_until(bar, target, flag, spin_limit);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *go_on = ok;
    }
    // The other threads acquire through the workgroup barrier: thread 0's agent-scope acquire
    // happens before it, and it invalidated the caches that the workgroup's waves share.
    __syncthreads();
    return *go_on != 0;
}

// The XCD that runs the calling wave (the hardware's own register, 0 ... 7 on this device).
__device__ __forceinline__ int xcc_id() {
    unsigned v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return (int)(v & 0xfu);
}

// Grid barrier number k (k >= 1) through one leader per XCD. The workgroups of an XCD share its
// L2, so one write-back of that L2 serves all of them: each workgroup arrives at its XCD's
// counter once its stores have reached the L2; the last to arrive (the leader) writes the L2
// back (agent-scope release), arrives at the global counter, waits for every XCD's leader,
// acquires and opens its XCD's gate; the others wait at the gate and then acquire at agent
// scope themselves (their compute unit's L1 may hold lines that other compute units have since
// rewritten). nx: workgroups on this XCD; ng: XCDs with workgroups; g0: the global count after
// the first (grid_barrier) pass. A per-workgroup release and acquire (grid_barrier) cost 28 us
// per pass on 512 workgroups, most of it in serialised L2 write-backs and invalidations.
__device__ __forceinline__ bool xcd_barrier(unsigned long long* bar, int xcc, unsigned long long nx,
                                            unsigned long long ng, unsigned long long g0,
                                            unsigned long long k, int* flag, int spin_limit,
                                            int* go_on) {
    stores_done();
    __syncthreads();  // every wave's stores of this pass have reached the L2
    if (threadIdx.x == 0) {
        unsigned long long* xarr = bar + kXcdArrSlot + xcc;
        unsigned long long* xgate = bar + kXcdGateSlot + xcc;
        int ok;
        const unsigned long long old =
            __hip_atomic_fetch_add(xarr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == k * nx) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = spin_until(bar, g0 + k * ng, flag, spin_limit);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            // the gate opens only after the invalidation has completed
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __hip_atomic_store(xgate, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = spin_until(xgate, k, flag, spin_limit);
            // agent-scope acquire: a workgroup-scope invalidation does not reach the compute
            // unit's L1 outside thread-group-split mode, and stale L1 lines were read here
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        *go_on = ok;
    }
    __syncthreads();
    return *go_on != 0;
}

// npairs two-step passes over the work-list in one launch (the tiles are the output tiles of
// step2_tile, as in k_batch_step2). The work-list is dealt to the XCDs in contiguous shares, as
// xcd_tile deals it to separate launches (workgroup b runs on XCD b mod 8), and the workgroups of
// one XCD take the tiles of its share in order from a ticket counter of their own, so a
// workgroup that finishes early takes the next tile, as the hardware dispatcher balances
// separate launches. Tickets are never reset within a launch: ticket T of an XCD with a share of
// S tiles is tile c0 + T mod S of pass T / S. A workgroup claims its next ticket when it starts a
// tile (the atomic's latency hides behind the tile) and publishes it to its threads through a
// double-buffered LDS slot at the barrier that ends the tile; a ticket of a later pass is held
// until that pass. Against a fixed walk (tiles L, L + G, ...) the tickets cut the 8 x 2048x1024
// ensemble from 0.42 to 0.35 ms per step. The tile function sees an opaque thread index, so that
// its per-thread index arithmetic is not hoisted out of the loops (held across them it would need
// more registers than the two-step tile leaves free).
// Threads of a persistent workgroup: those of the two-step launches, except 512 for 64 x 8 tiles:
// two workgroups per CU then leave 128 VGPRs per thread (4 waves per SIMD) where 768 threads leave
// 80, which the loop state around the tile function overflows.
// The 32 x 4 tile runs its wide workgroup (step2_wide_threads) in every schedule.
__host__ __device__ constexpr int persist_threads(int TX, int TY, int GEO) {
    return TX == 64 && TY == 8 ? 512
                               : (TX == 32 && TY == 4 ? step2_wide_threads(32, 4)
                                                      : step2_threads(TX, TY, GEO));
}
__host__ __device__ constexpr int persist_waves(int TX, int TY, int GEO) {
    return TX == 64 && TY == 8 ? 4
                               : (TX == 32 && TY == 4 ? (step2_wide_threads(32, 4) / 64 + 3) / 4
                                                      : step2_waves(TX, TY, GEO));
}

template <int TX, int TY, int GEO, int EOS>
__global__ __launch_bounds__(persist_threads(TX, TY, GEO), persist_waves(TX, TY, GEO)) void
k_batch_persistent(const InstDesc* __restrict__ inst, const int* __restrict__ tile_inst,
                   int ntiles, int npairs, int cur0, unsigned long long* bar, int* flag,
                   int spin_limit) {
    __shared__ Step2Lds<TX, TY, GEO> lds;
    __shared__ int go_on;
    __shared__ unsigned long long next[2];
    const int G = gridDim.x;
    // this XCD's share of the work-list: [c0, c0 + S)
    const int groups = G < kXcds ? G : kXcds;
    const int xg = (int)blockIdx.x % groups;
    const int q = ntiles / groups, rem = ntiles % groups;
    const int c0 = xg * q + (xg < rem ? xg : rem);
    const unsigned long long S = (unsigned long long)(q + (xg < rem ? 1 : 0));
    unsigned long long* tk = bar + kTicketSlot + xg;
    auto claim = [&]() {
        return S ? __hip_atomic_fetch_add(tk, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                 : ~0ull;
    };
    // registration: workgroups per XCD, complete once the first (grid-wide) barrier has passed
    const int xcc = xcc_id();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar + kXcdRegSlot + (xcc < kXcds ? xcc : 0), 1ull,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (xcc >= kXcds) __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        next[0] = claim();
    }
    __syncthreads();
    unsigned long long T = next[0];
    int slot = 1;
    unsigned long long nx = 0, ng = 0;
    // each pass reads g[cur0] and writes g[cur0 ^ 1] (two steps), then the two swap roles
    for (int k = 0; k < npairs; ++k) {
        const unsigned long long base = (unsigned long long)k * S, end = base + S;
        while (T < end) {  // T >= base: a held ticket is never of an earlier pass
            unsigned long long Tn = 0;
            if (threadIdx.x == 0) Tn = claim();
            const int t = c0 + (int)(T - base);
            const InstDesc* D = inst + tile_inst[t];
            int x0, y0;
            batch_tile_origin(D, t, TX, TY, x0, y0);
            step2_tile_any<TX, TY, GEO, EOS, false, true, persist_threads(TX, TY, GEO)>(
                D->P, gptr(D->g[cur0]), gptr(D->g[cur0 ^ 1]), gptr(D->gw), x0, y0, lds);
            if (threadIdx.x == 0) next[slot] = Tn;
            __syncthreads();  // the LDS tile is reused by the next tile; the ticket is published
            T = next[slot];
            slot ^= 1;
        }
        if (k + 1 == npairs) break;  // the launch's end orders the last pass before what follows
        if (k == 0) {
            if (!grid_barrier(bar, (unsigned long long)G, flag, spin_limit, &go_on)) return;
            if (threadIdx.x == 0) {
                unsigned long long n = 0, c = 0;
                for (int x = 0; x < kXcds; ++x) {
                    c = __hip_atomic_load(bar + kXcdRegSlot + x, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                    n += c != 0;
                    if (x == xcc) next[0] = c;
                }
                next[1] = n;
                // an XCD id beyond the control block raised the flag at registration
                go_on = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
            }
            __syncthreads();
            nx = next[0];
            ng = next[1];
            const bool go = go_on != 0;
            __syncthreads();  // next[] serves the tickets again
            if (!go) return;
        } else if (!xcd_barrier(bar, xcc, nx, ng, (unsigned long long)G, (unsigned long long)k,
                                flag, spin_limit, &go_on)) {
            return;
        }
        cur0 ^= 1;
    }
}

// Contact lines of every instance (one block per instance): out[2i], out[2i+1] on rows[i].
__global__ __launch_bounds__(256) void k_batch_contact_line(const InstDesc* __restrict__ inst,
                                                            const int* __restrict__ rows, int cur,
                                                            double* __restrict__ out) {
    const InstDesc* D = inst + blockIdx.x;
    contact_line_block(D->P, D->g[cur], rows[blockIdx.x], D->P.rho_mid, out + 2 * blockIdx.x);
}

// ---- ensemble adjoint ---------------------------------------------------------------------------

__device__ __forceinline__ void adj_tile_origin(const AdjInst* D, int t, int& x0, int& y0) {
    const int lt = t - D->tile0;
    x0 = (lt % D->ntx) * 64;
    y0 = D->P.y_lo + (lt / D->ntx) * 4;
}

// Segment states i -> i+1, i+2 of every instance (two steps per launch, the first written too),
// over a work-list of 64 x 8 output tiles (the recomputation work-list).
template <int EOS>
__global__ __launch_bounds__(step2_threads(64, 8, GEO_ROWS), step2_waves(64, 8, GEO_ROWS)) void
k_batch_seg_step2(const AdjInst* __restrict__ inst, const int* __restrict__ tile_inst, int ntiles,
                  int i) {
    __shared__ Step2Lds<64, 8, GEO_ROWS> lds;
    const int t = xcd_tile(blockIdx.x, ntiles);
    const AdjInst* D = inst + tile_inst[t];
    const int lt = t - D->tile0_8;
    const int x0 = (lt % D->ntx) * 64;
    const int y0 = D->P.y_lo + (lt / D->ntx) * 8;
    double* s0 = gptr(D->seg) + (long long)i * D->fstride;
    step2_tile_any<64, 8, GEO_ROWS, EOS, true>(D->P, s0, s0 + 2 * D->fstride, gptr(D->gw), x0, y0,
                                               lds, s0 + D->fstride);
}

// Segment state i -> i+1 of every instance (one fused step).
template <int EOS>
__global__ __launch_bounds__(256) void k_batch_seg_step(const AdjInst* __restrict__ inst,
                                                        const int* __restrict__ tile_inst,
                                                        int ntiles, int i) {
    __shared__ double sp[6 * 66];
    const int t = xcd_tile(blockIdx.x, ntiles);
    const AdjInst* D = inst + tile_inst[t];
    int x0, y0;
    adj_tile_origin(D, t, x0, y0);
    double* s0 = gptr(D->seg) + (long long)i * D->fstride;
    step_tile<64, 4, true, GEO_ROWS, EOS>(D->P, s0, s0 + D->fstride, nullptr, gptr(D->gw), x0, y0,
                                          sp);
}

// One reverse step of every instance: segment state i, later-step buffers of parity k.
template <int EOS>
__global__ __launch_bounds__(256) void k_batch_adj(const AdjInst* __restrict__ inst,
                                                   const int* __restrict__ tile_inst, int ntiles,
                                                   int i, int k) {
    __shared__ AdjLds<64, 4> lds;
    const int t = xcd_tile(blockIdx.x, ntiles);
    const AdjInst* D = inst + tile_inst[t];
    int x0, y0;
    adj_tile_origin(D, t, x0, y0);
    const AdjPtrs A{gptr(D->seg) + (long long)i * D->fstride,
                    gptr(D->a[k]),     gptr(D->q[k]),     gptr(D->p0[k]),     gptr(D->dpsi[k]),
                    gptr(D->rv[k]),    gptr(D->gw),       gptr(D->a[k ^ 1]),  gptr(D->q[k ^ 1]),
                    gptr(D->p0[k ^ 1]), gptr(D->dpsi[k ^ 1]), gptr(D->rv[k ^ 1]), gptr(D->gg)};
    adj_tile<64, 4, 256, EOS>(D->P, A, x0, y0, lds);
}

// dL/dG_w of the last reverse step's wall vectors (instance blockIdx.y).
__global__ __launch_bounds__(256) void k_batch_adj_gw(const AdjInst* __restrict__ inst, int k) {
    const AdjInst* D = inst + blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= D->P.nx || !D->P.walls) return;
    adj_gw_node(D->P, D->rv[k], D->gg, x, 1);
    adj_gw_node(D->P, D->rv[k], D->gg, x, D->P.ny - 2);
}

// Clears the barrier counter, the abort flag, the ticket counters and the per-XCD barrier
// counters (a kernel rather than a memset node, so the pair can sit in a hipGraph).
__global__ void k_batch_reset(unsigned long long* bar, int* flag) {
    static_assert(kControlWords <= 64, "one thread per control word");
    if (threadIdx.x == 0) {
        *bar = 0ull;
        *flag = 0;
    }
    if (threadIdx.x >= kTicketSlot && threadIdx.x < kControlWords) bar[threadIdx.x] = 0ull;
}

// ------------------------------------------------------------------------------------------------
// Calls f(geo, eos) with the ensemble's geometry and equation-of-state variants as compile-time
// constants.
template <class F>
static hipError_t dispatch(int geo, int eos, F&& f) {
    auto with_eos = [&](auto g) {
        if (eos == EOS_CS) return f(g, std::integral_constant<int, EOS_CS>{});
        if (eos == EOS_PW) return f(g, std::integral_constant<int, EOS_PW>{});
        return f(g, std::integral_constant<int, EOS_ANY>{});
    };
    if (geo == GEO_MASK) return with_eos(std::integral_constant<int, GEO_MASK>{});
    if (geo == GEO_WET) return with_eos(std::integral_constant<int, GEO_WET>{});
    return with_eos(std::integral_constant<int, GEO_ROWS>{});
}

template <int TX, int TY>
static hipError_t launch_batch_t(int geo, int eos, const InstDesc* inst, const int* tile_inst,
                                 int ntiles, int cur, hipStream_t s) {
    return dispatch(geo, eos, [&](auto g, auto e) {
        hipLaunchKernelGGL((k_batch_step<TX, TY, decltype(g)::value, decltype(e)::value>),
                           dim3(ntiles), dim3(TX * TY), 0, s, inst, tile_inst, ntiles, cur);
        return hipGetLastError();
    });
}

template <int TX, int TY>
static hipError_t launch_persist_t(int geo, int eos, int grid, const InstDesc* inst,
                                   const int* tile_inst, int ntiles, int npairs, int cur,
                                   unsigned long long* bar, int* flag, int spin_limit,
                                   hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, bar, flag);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
    return dispatch(geo, eos, [&](auto g, auto e) {
        constexpr int G = decltype(g)::value;
        hipLaunchKernelGGL((k_batch_persistent<TX, TY, G, decltype(e)::value>), dim3(grid),
                           dim3(persist_threads(TX, TY, G)), 0, s, inst, tile_inst, ntiles, npairs,
                           cur, bar, flag, spin_limit);
        return hipGetLastError();
    });
}

// Resident workgroups per CU of the persistent kernel: the smallest over its variants, so a grid
// sized by it fits whichever is launched.
template <int TX, int TY>
static int occupancy_t() {
    int lo = 1 << 30;
    for (int geo : {GEO_ROWS, GEO_WET, GEO_MASK})
        for (int eos : {EOS_CS, EOS_PW, EOS_ANY}) {
            int n = 0;
            hipError_t r = dispatch(geo, eos, [&](auto g, auto e) {
                constexpr int G = decltype(g)::value;
                return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &n, k_batch_persistent<TX, TY, G, decltype(e)::value>,
                    persist_threads(TX, TY, G), 0);
            });
            if (r != hipSuccess) return 0;
            lo = std::min(lo, n);
        }
    return lo;
}

int batch_tiles(int tile) { return tile >= 0 && tile < 4; }

template <int TX, int TY>
static hipError_t launch_batch2_t(int geo, int eos, const InstDesc* inst, const int* tile_inst,
                                  int ntiles, int cur, hipStream_t s) {
    return dispatch(geo, eos, [&](auto g, auto e) {
        constexpr int G = decltype(g)::value;
        constexpr int NT = TX == 32 && TY == 4 ? step2_wide_threads(32, 4)
                                               : step2_threads(TX, TY, G);
        hipLaunchKernelGGL((k_batch_step2<TX, TY, G, decltype(e)::value, NT>), dim3(ntiles),
                           dim3(NT), 0, s, inst, tile_inst, ntiles, cur);
        return hipGetLastError();
    });
}

// Tile shapes of an ensemble's work-list: 0 64x4, 1 64x8, 2 64x16, 3 128x4, 4 32x4 (whose
// two-step workgroups are the wide ones: for ensembles too small to fill the chip).
void batch_tile_shape(int tile, int* tx, int* ty) {
    static const int k[5][2] = {{64, 4}, {64, 8}, {64, 16}, {128, 4}, {32, 4}};
    if (tile < 0 || tile > 4) tile = 0;
    *tx = k[tile][0];
    *ty = k[tile][1];
}

// Two steps per launch (schedule 2) with the output tiles of the work-list's tile shape.
hipError_t launch_batch_step2(int tile, int geo, int eos, const InstDesc* inst,
                              const int* tile_inst, int ntiles, int cur, hipStream_t s) {
    switch (tile) {
        case 4: return launch_batch2_t<32, 4>(geo, eos, inst, tile_inst, ntiles, cur, s);
        case 1: return launch_batch2_t<64, 8>(geo, eos, inst, tile_inst, ntiles, cur, s);
        case 2: return launch_batch2_t<64, 16>(geo, eos, inst, tile_inst, ntiles, cur, s);
        case 3: return launch_batch2_t<128, 4>(geo, eos, inst, tile_inst, ntiles, cur, s);
        default: return launch_batch2_t<64, 4>(geo, eos, inst, tile_inst, ntiles, cur, s);
    }
}

hipError_t launch_batch_step(int tile, int geo, int eos, const InstDesc* inst,
                             const int* tile_inst, int ntiles, int cur, hipStream_t s) {
    switch (tile) {
        case 4: return launch_batch_t<32, 4>(geo, eos, inst, tile_inst, ntiles, cur, s);
        case 1: return launch_batch_t<64, 8>(geo, eos, inst, tile_inst, ntiles, cur, s);
        case 2: return launch_batch_t<64, 16>(geo, eos, inst, tile_inst, ntiles, cur, s);
        case 3: return launch_batch_t<128, 4>(geo, eos, inst, tile_inst, ntiles, cur, s);
        default: return launch_batch_t<64, 4>(geo, eos, inst, tile_inst, ntiles, cur, s);
    }
}

hipError_t launch_batch_persistent(int tile, int geo, int eos, int grid, const InstDesc* inst,
                                   const int* tile_inst, int ntiles, int npairs, int cur,
                                   unsigned long long* bar, int* flag, int spin_limit,
                                   hipStream_t s) {
    switch (tile) {
        case 4: return launch_persist_t<32, 4>(geo, eos, grid, inst, tile_inst, ntiles, npairs,
                                               cur, bar, flag, spin_limit, s);
        case 1: return launch_persist_t<64, 8>(geo, eos, grid, inst, tile_inst, ntiles, npairs,
                                               cur, bar, flag, spin_limit, s);
        case 2: return launch_persist_t<64, 16>(geo, eos, grid, inst, tile_inst, ntiles, npairs,
                                                cur, bar, flag, spin_limit, s);
        case 3: return launch_persist_t<128, 4>(geo, eos, grid, inst, tile_inst, ntiles, npairs,
                                                cur, bar, flag, spin_limit, s);
        default: return launch_persist_t<64, 4>(geo, eos, grid, inst, tile_inst, ntiles, npairs,
                                                cur, bar, flag, spin_limit, s);
    }
}

int batch_persistent_occupancy(int tile) {
    switch (tile) {
        case 4: return occupancy_t<32, 4>();
        case 1: return occupancy_t<64, 8>();
        case 2: return occupancy_t<64, 16>();
        case 3: return occupancy_t<128, 4>();
        default: return occupancy_t<64, 4>();
    }
}

template <class F>
static hipError_t with_eos(int eos, F&& f) {
    if (eos == EOS_CS) return f(std::integral_constant<int, EOS_CS>{});
    if (eos == EOS_PW) return f(std::integral_constant<int, EOS_PW>{});
    return f(std::integral_constant<int, EOS_ANY>{});
}

hipError_t launch_batch_seg_step2(int eos, const AdjInst* inst, const int* tile_inst, int ntiles,
                                  int i, hipStream_t s) {
    return with_eos(eos, [&](auto e) {
        hipLaunchKernelGGL((k_batch_seg_step2<decltype(e)::value>), dim3(ntiles),
                           dim3(step2_threads(64, 8, GEO_ROWS)), 0, s, inst, tile_inst, ntiles, i);
        return hipGetLastError();
    });
}

hipError_t launch_batch_seg_step(int eos, const AdjInst* inst, const int* tile_inst, int ntiles,
                                 int i, hipStream_t s) {
    return with_eos(eos, [&](auto e) {
        hipLaunchKernelGGL((k_batch_seg_step<decltype(e)::value>), dim3(ntiles), dim3(256), 0, s,
                           inst, tile_inst, ntiles, i);
        return hipGetLastError();
    });
}

hipError_t launch_batch_adj(int eos, const AdjInst* inst, const int* tile_inst, int ntiles, int i,
                            int k, hipStream_t s) {
    return with_eos(eos, [&](auto e) {
        hipLaunchKernelGGL((k_batch_adj<decltype(e)::value>), dim3(ntiles), dim3(256), 0, s, inst,
                           tile_inst, ntiles, i, k);
        return hipGetLastError();
    });
}

hipError_t launch_batch_adj_gw(const AdjInst* inst, int count, int max_nx, int k,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_batch_adj_gw, dim3((max_nx + 255) / 256, count), dim3(256), 0, s, inst,
                       k);
    return hipGetLastError();
}

hipError_t launch_batch_contact_line(const InstDesc* inst, const int* rows, int count, int cur,
                                     double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_contact_line, dim3(count), dim3(256), 0, s, inst, rows, cur, out);
    return hipGetLastError();
}

}  // namespace lbm
