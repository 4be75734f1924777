// bodex_launch.h -- launchers of the kernels, one translation unit per kernel
// family so that they compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

namespace bodex {
struct KArgs;
hipError_t launch_admm(int mm, int occ, const KArgs& a, int grid, size_t lds, hipStream_t st);
hipError_t launch_finalize(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st);
hipError_t launch_backward(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st);
hipError_t launch_reset(int* q, int n, hipStream_t st);
}  // namespace bodex
