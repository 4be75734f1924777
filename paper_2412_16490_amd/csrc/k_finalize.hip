// Launcher of the finalize kernel for the compiled contact counts (gamma = 0).
#include "bodex_kernels.h"
#include "bodex_launch.h"

namespace bodex {

hipError_t launch_finalize_sum(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st);
hipError_t launch_finalize_chunk(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st);

hipError_t launch_finalize(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    if (a.gamma > 0.f) return launch_finalize_sum(mm, a, grid, lds, st);
    if (a.fin_mode != 0) return launch_finalize_chunk(mm, a, grid, lds, st);
    switch (mm) {
        case 4: hipLaunchKernelGGL((finalize_kernel<4, false, 0>), dim3(grid), dim3(64), lds, st, a); break;
        case 5: hipLaunchKernelGGL((finalize_kernel<5, false, 0>), dim3(grid), dim3(64), lds, st, a); break;
        case 6: hipLaunchKernelGGL((finalize_kernel<6, false, 0>), dim3(grid), dim3(64), lds, st, a); break;
        case 7: hipLaunchKernelGGL((finalize_kernel<7, false, 0>), dim3(grid), dim3(64), lds, st, a); break;
        case 8: hipLaunchKernelGGL((finalize_kernel<8, false, 0>), dim3(grid), dim3(64), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bodex
