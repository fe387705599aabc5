// lbm_internal.h -- launchers shared between the kernels and the C-ABI layer (not installed).
#pragma once
#include <hip/hip_runtime.h>

#include "lbm_device.h"

namespace lbm {

enum { OBS_NQ = 15 };

// One instance of an ensemble, as the batch kernels see it (device memory).
struct InstDesc {
    KParams P;
    double* g[2];  // population buffers (post-collision), ping-pong
    double* gw;    // [2][pitch] G_w
    int tile0;     // first tile of this instance in the flattened work-list
    int ntx, nty;  // tiles in x and y
    int pad;
};

// One instance of an ensemble's adjoint run (device memory): its segment of recomputed states
// and the adjoint quantities of two consecutive reverse steps (see AdjPtrs).
struct AdjInst {
    KParams P;
    double* seg;       // the segment's states, fstride doubles apart
    long long fstride;
    double* a[2];
    double* q[2];
    double* p0[2];
    double* dpsi[2];
    double* rv[2];
    const double* gw;
    double* gg;  // [2][pitch] dL/dG_w
    int tile0;   // first 64 x 4 tile of this instance in the adjoint work-list
    int ntx, nty;
    int tile0_8;  // first 64 x 8 tile in the recomputation work-list (ntx columns as above)
    int nty8;
    int pad;
};

int n_tiles();
void tile_shape(int tile, int* tx, int* ty);
// Tile shape of an ensemble's work-list (tune.tile 0..4).
void batch_tile_shape(int tile, int* tx, int* ty);
hipError_t launch_step(const KParams& P, int schedule, int tile, const double* gin, double* gout,
                       double* psi, const double* gw, hipStream_t s);
// gmid (optional, bounce-back or periodic rows): also receives the state after the first step
hipError_t launch_step2(const KParams& P, int tile2, const double* gin, double* gout,
                        const double* gw, hipStream_t s, double* gmid = nullptr);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);  // bytes and p 8-byte aligned
hipError_t launch_init(const KParams& P, const double* rho0, double* g, hipStream_t s);
// droplets of the initial state (lbm_create_droplets): up to kMaxDroplets tanh profiles
constexpr int kMaxDroplets = 64;
struct DropletArgs {
    int count;
    double x0[kMaxDroplets], y0[kMaxDroplets], r[kMaxDroplets];
    double mid, half;            // (rho_l + rho_v) / 2, (rho_l - rho_v) / 2
    double width, jitter;
    unsigned long long base;     // splitmix64(seed)
};
hipError_t launch_droplets(const KParams& P, const DropletArgs& D, double* rho, hipStream_t s);
hipError_t launch_fp64_probe(const double* a, const double* b, double* sq, double* quot,
                             long long n, hipStream_t s);
// dense: fout is [9][ny][nx] (otherwise [9][ny][pitch])
hipError_t launch_pull(const KParams& P, const double* gin, double* fout, hipStream_t s,
                       bool dense = false);
// `planes` planes of ny x nx doubles from one row/plane layout to another (device memory)
hipError_t launch_repack(const double* src, long long src_plane, int src_pitch, double* dst,
                         long long dst_plane, int dst_pitch, int nx, int ny, int planes,
                         hipStream_t s);
// pre: gin holds pre-collision populations (otherwise the post-collision state, pulled)
hipError_t launch_rho_psi(const KParams& P, const double* gin, double* psi, double* rho,
                          hipStream_t s, bool pre = false);
hipError_t launch_contact_line(const KParams& P, const double* gin, int row, double mid,
                               double* out, hipStream_t s);
int obs_blocks(const KParams& P);
hipError_t launch_obs(const KParams& P, const double* gin, const double* rho, const double* psi,
                      const double* gw, const ObsArgs& A, double* part, double* out,
                      hipStream_t s, bool pre = false);

// adjoint
hipError_t launch_adj(const KParams& P, const AdjPtrs& A, hipStream_t s);
hipError_t launch_adj_gw(const KParams& P, const double* rv, double* gwgrad, hipStream_t s);
int loss_blocks(const KParams& P);
hipError_t launch_loss(const KParams& P, const double* g, double* part, double* out,
                       hipStream_t s);
hipError_t launch_loss_seed(const KParams& P, double w_c, double w_w, double yc, double sum_phi,
                            double* p0, double* dpsi, hipStream_t s);

// batch
int batch_tiles(int tile);
// geo: GEO_ROWS, GEO_WET (some instance uses the wet-node wall) or GEO_MASK (every instance has
// a solid mask); eos: EOS_CS or EOS_PW when every instance uses it, else EOS_ANY. They select the
// kernels compiled for that variant.
hipError_t launch_batch_step(int tile, int geo, int eos, const InstDesc* inst,
                             const int* tile_inst, int ntiles, int cur, hipStream_t s);
hipError_t launch_batch_step2(int tile, int geo, int eos, const InstDesc* inst,
                              const int* tile_inst, int ntiles, int cur, hipStream_t s);
// The persistent schedule's control block (kControlWords 8-byte words of the ensemble
// workspace): the grid barrier's arrival counter (word 0), the abort flag (an int at byte 64),
// and per XCD a tile-ticket counter, a barrier arrival counter, a barrier gate and a count of
// its workgroups (kXcds words each from kTicketSlot, kXcdArrSlot, kXcdGateSlot, kXcdRegSlot).
constexpr int kXcds = 8;
constexpr int kTicketSlot = 16;
constexpr int kXcdArrSlot = kTicketSlot + kXcds;
constexpr int kXcdGateSlot = kXcdArrSlot + kXcds;
constexpr int kXcdRegSlot = kXcdGateSlot + kXcds;
constexpr int kControlWords = kXcdRegSlot + kXcds;
// npairs two-step passes in one launch (after a reset of the control block)
hipError_t launch_batch_persistent(int tile, int geo, int eos, int grid, const InstDesc* inst,
                                   const int* tile_inst, int ntiles, int npairs, int cur,
                                   unsigned long long* bar, int* flag, int spin_limit,
                                   hipStream_t s);
hipError_t launch_batch_contact_line(const InstDesc* inst, const int* rows, int count, int cur,
                                     double* out, hipStream_t s);
int batch_persistent_occupancy(int tile);
// ensemble adjoint, over work-lists of the tiles of every instance (bounce-back walls):
// recomputation of segment states i -> i+1, i+2 (two steps, 64 x 8 output tiles) or i -> i+1 (one
// step, 64 x 4), one reverse step of segment state i (64 x 4; k: parity of the later step's
// buffers), and the last step's G_w gradient
hipError_t launch_batch_seg_step2(int eos, const AdjInst* inst, const int* tile_inst, int ntiles,
                                  int i, hipStream_t s);
hipError_t launch_batch_seg_step(int eos, const AdjInst* inst, const int* tile_inst, int ntiles,
                                 int i, hipStream_t s);
hipError_t launch_batch_adj(int eos, const AdjInst* inst, const int* tile_inst, int ntiles, int i,
                            int k, hipStream_t s);
hipError_t launch_batch_adj_gw(const AdjInst* inst, int count, int max_nx, int k,
                               hipStream_t s);

}  // namespace lbm
