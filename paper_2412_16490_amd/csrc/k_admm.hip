// Launcher of the admm kernel for the compiled contact counts.
#include "bodex_kernels.h"
#include "bodex_launch.h"

namespace bodex {

// Reset of the persistent-launch tile counters (a kernel rather than a memset
// so that it can sit inside a captured graph).
__global__ void reset_counter_kernel(int* q, int n) {
    if (int(threadIdx.x) < n) q[threadIdx.x] = 0;
}

hipError_t launch_admm(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    switch (mm) {
        case 4: hipLaunchKernelGGL(admm_kernel<4>, dim3(grid), dim3(64), lds, st, a); break;
        case 5: hipLaunchKernelGGL(admm_kernel<5>, dim3(grid), dim3(64), lds, st, a); break;
#ifdef BODEX_WITH_MM8
        case 8: hipLaunchKernelGGL(admm_kernel<8>, dim3(grid), dim3(64), lds, st, a); break;
#endif
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reset(int* q, int n, hipStream_t st) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, q, n);
    return hipGetLastError();
}

}  // namespace bodex
