// Launcher of the finalize kernel for the compiled contact counts, with the normal-sum row (gamma > 0).
#include "bodex_kernels.h"
#include "bodex_launch.h"

namespace bodex {

hipError_t launch_finalize_sum(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    switch (mm) {
        case 4: hipLaunchKernelGGL((finalize_kernel<4, true, 0>), dim3(grid), dim3(64), lds, st, a); break;
        case 5: hipLaunchKernelGGL((finalize_kernel<5, true, 0>), dim3(grid), dim3(64), lds, st, a); break;
        case 6: hipLaunchKernelGGL((finalize_kernel<6, true, 0>), dim3(grid), dim3(64), lds, st, a); break;
        case 7: hipLaunchKernelGGL((finalize_kernel<7, true, 0>), dim3(grid), dim3(64), lds, st, a); break;
        case 8: hipLaunchKernelGGL((finalize_kernel<8, true, 0>), dim3(grid), dim3(64), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bodex
