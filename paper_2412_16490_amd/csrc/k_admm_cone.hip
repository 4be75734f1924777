// Launcher of the admm kernel for the circular-cone form.
#include "bodex_kernels.h"
#include "bodex_launch.h"

namespace bodex {

template <int MM>
static hipError_t launch_admm_cone_mm(int occ, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    switch (occ) {
        case 1: hipLaunchKernelGGL((admm_kernel<MM, 1, true>), dim3(grid), dim3(64), lds, st, a); break;
        case 2: hipLaunchKernelGGL((admm_kernel<MM, 2, true>), dim3(grid), dim3(64), lds, st, a); break;
        case 3: hipLaunchKernelGGL((admm_kernel<MM, 3, true>), dim3(grid), dim3(64), lds, st, a); break;
        case 4: hipLaunchKernelGGL((admm_kernel<MM, 4, true>), dim3(grid), dim3(64), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_admm_cone(int mm, int occ, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    switch (mm) {
        case 4: return launch_admm_cone_mm<4>(occ, a, grid, lds, st);
        case 5: return launch_admm_cone_mm<5>(occ, a, grid, lds, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bodex
