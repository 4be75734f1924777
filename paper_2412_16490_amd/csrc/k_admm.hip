// Launcher of the admm kernel for the compiled contact counts.
#include "bodex_kernels.h"
#include "bodex_launch.h"

namespace bodex {

// Reset of the persistent-launch tile counters (a kernel rather than a memset
// so that it can sit inside a captured graph).
__global__ void reset_counter_kernel(int* q, int n) {
    if (int(threadIdx.x) < n) q[threadIdx.x] = 0;
}

template <int MM>
static hipError_t launch_admm_mm(int occ, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    switch (occ) {
        case 1: hipLaunchKernelGGL((admm_kernel<MM, 1, false>), dim3(grid), dim3(64), lds, st, a); break;
        case 2: hipLaunchKernelGGL((admm_kernel<MM, 2, false>), dim3(grid), dim3(64), lds, st, a); break;
        case 3: hipLaunchKernelGGL((admm_kernel<MM, 3, false>), dim3(grid), dim3(64), lds, st, a); break;
        case 4: hipLaunchKernelGGL((admm_kernel<MM, 4, false>), dim3(grid), dim3(64), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_admm(int mm, int occ, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    if (a.cone) return launch_admm_cone(mm, occ, a, grid, lds, st);
    switch (mm) {
        case 4: return launch_admm_mm<4>(occ, a, grid, lds, st);
        case 5: return launch_admm_mm<5>(occ, a, grid, lds, st);
        case 6: return launch_admm_mm<6>(occ, a, grid, lds, st);
        case 7: return launch_admm_mm<7>(occ, a, grid, lds, st);
        case 8: return launch_admm_mm<8>(occ, a, grid, lds, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reset(int* q, int n, hipStream_t st) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, q, n);
    return hipGetLastError();
}

}  // namespace bodex
