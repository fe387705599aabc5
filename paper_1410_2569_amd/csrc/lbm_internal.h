// lbm_internal.h -- launchers shared between the kernels and the C-ABI layer (not installed).
#pragma once
#include <hip/hip_runtime.h>

#include "lbm_device.h"

namespace lbm {

// Arguments of the observables kernel: contour level, fit window and centring of the sums.
struct ObsArgs {
    double rho_mid;     // (rho_l + rho_v) / 2
    double y_min;       // interface points below this height are not fitted
    double x_lo, x_hi;  // fit window
    double cx, cy;      // coordinates are accumulated relative to this point
};

enum { OBS_NQ = 15 };

int n_tiles();
void tile_shape(int tile, int* tx, int* ty);
hipError_t launch_step(const KParams& P, int schedule, int tile, const double* gin, double* gout,
                       double* psi, const double* gw, hipStream_t s);
hipError_t launch_init(const KParams& P, const double* rho0, double* g, hipStream_t s);
hipError_t launch_pull(const KParams& P, const double* gin, double* fout, hipStream_t s);
hipError_t launch_rho_psi(const KParams& P, const double* gin, double* psi, double* rho,
                          hipStream_t s);
int obs_blocks(const KParams& P);
hipError_t launch_obs(const KParams& P, const double* gin, const double* rho, const double* psi,
                      const double* gw, const ObsArgs& A, double* part, double* out,
                      hipStream_t s);

}  // namespace lbm
