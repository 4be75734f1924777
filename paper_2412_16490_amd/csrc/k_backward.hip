// Launcher of the backward kernel for the compiled contact counts (gamma = 0).
#include "bodex_kernels.h"
#include "bodex_launch.h"

namespace bodex {

hipError_t launch_backward_sum(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st);

hipError_t launch_backward(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    if (a.gamma > 0.f) return launch_backward_sum(mm, a, grid, lds, st);
    switch (mm) {
        case 4: hipLaunchKernelGGL((backward_kernel<4, false, false>), dim3(grid), dim3(64), lds, st, a); break;
        case 5: hipLaunchKernelGGL((backward_kernel<5, false, false>), dim3(grid), dim3(64), lds, st, a); break;
        case 6: hipLaunchKernelGGL((backward_kernel<6, false, false>), dim3(grid), dim3(64), lds, st, a); break;
        case 7: hipLaunchKernelGGL((backward_kernel<7, false, false>), dim3(grid), dim3(64), lds, st, a); break;
        case 8: hipLaunchKernelGGL((backward_kernel<8, false, false>), dim3(grid), dim3(64), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bodex
