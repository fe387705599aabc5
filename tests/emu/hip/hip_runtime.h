// Host stand-in for the few HIP device facilities the library's per-node and per-tile device
// functions use, so that those functions compile for the CPU and run inside an emulated
// workgroup (one host thread per device thread). Test infrastructure only.
#pragma once
#include <cmath>
#include <cstdint>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static

struct EmuIdx {
    unsigned x = 0, y = 0, z = 0;
};
extern thread_local EmuIdx threadIdx;

// Workgroup barrier and barrier-with-or of the emulated workgroup.
void __syncthreads();
int __syncthreads_or(int v);

using std::fma;
using std::fmax;
using std::fmin;
using std::isfinite;
using std::sqrt;
