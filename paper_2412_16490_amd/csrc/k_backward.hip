// Launcher of the backward kernel for the compiled contact counts.
#include "bodex_kernels.h"
#include "bodex_launch.h"

namespace bodex {

hipError_t launch_backward(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    switch (mm) {
        case 4: hipLaunchKernelGGL(backward_kernel<4>, dim3(grid), dim3(64), lds, st, a); break;
        case 5: hipLaunchKernelGGL(backward_kernel<5>, dim3(grid), dim3(64), lds, st, a); break;
#ifdef BODEX_WITH_MM8
        case 8: hipLaunchKernelGGL(backward_kernel<8>, dim3(grid), dim3(64), lds, st, a); break;
#endif
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bodex
