// Launcher of the backward kernel for the circular-cone form.
#include "bodex_kernels.h"
#include "bodex_launch.h"

namespace bodex {

hipError_t launch_backward_cone(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    switch (mm) {
        case 4: hipLaunchKernelGGL((backward_kernel<4, false, true>), dim3(grid), dim3(64), lds, st, a); break;
        case 5: hipLaunchKernelGGL((backward_kernel<5, false, true>), dim3(grid), dim3(64), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bodex
