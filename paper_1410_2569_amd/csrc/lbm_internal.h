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

int n_tiles();
void tile_shape(int tile, int* tx, int* ty);
hipError_t launch_step(const KParams& P, int schedule, int tile, const double* gin, double* gout,
                       double* psi, const double* gw, hipStream_t s);
hipError_t launch_step2(const KParams& P, int tile2, const double* gin, double* gout,
                        const double* gw, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);  // bytes and p 8-byte aligned
hipError_t launch_init(const KParams& P, const double* rho0, double* g, hipStream_t s);
hipError_t launch_pull(const KParams& P, const double* gin, double* fout, hipStream_t s);
hipError_t launch_rho_psi(const KParams& P, const double* gin, double* psi, double* rho,
                          hipStream_t s);
hipError_t launch_contact_line(const KParams& P, const double* gin, int row, double mid,
                               double* out, hipStream_t s);
int obs_blocks(const KParams& P);
hipError_t launch_obs(const KParams& P, const double* gin, const double* rho, const double* psi,
                      const double* gw, const ObsArgs& A, double* part, double* out,
                      hipStream_t s);

// adjoint
hipError_t launch_adj_step(const KParams& P, const double* gprev, const double* a_in,
                           const double* c_in, const double* gw, double* a_out, double* qbuf,
                           double* p0buf, double* dpsibuf, double* rvec, double* c_out,
                           double* gwgrad, hipStream_t s);
int loss_blocks(const KParams& P);
hipError_t launch_loss(const KParams& P, const double* g, double* part, double* out,
                       hipStream_t s);
hipError_t launch_loss_seed(const KParams& P, double w_c, double w_w, double yc, double sum_phi,
                            double* c, hipStream_t s);

// batch
int batch_tiles(int tile);
// geo: GEO_ROWS, GEO_WET (some instance uses the wet-node wall) or GEO_MASK (every instance has
// a solid mask); eos: EOS_CS or EOS_PW when every instance uses it, else EOS_ANY. They select the
// kernels compiled for that variant.
hipError_t launch_batch_step(int tile, int geo, int eos, const InstDesc* inst,
                             const int* tile_inst, int ntiles, int cur, hipStream_t s);
hipError_t launch_batch_step2(int tile, int geo, int eos, const InstDesc* inst,
                              const int* tile_inst, int ntiles, int cur, hipStream_t s);
hipError_t launch_batch_persistent(int tile, int geo, int eos, int grid, const InstDesc* inst,
                                   const int* tile_inst, int ntiles, int nsteps, int cur,
                                   unsigned* bar, int* flag, int spin_limit, hipStream_t s);
hipError_t launch_batch_contact_line(const InstDesc* inst, const int* rows, int count, int cur,
                                     double* out, hipStream_t s);
int batch_persistent_occupancy(int tile);

}  // namespace lbm
