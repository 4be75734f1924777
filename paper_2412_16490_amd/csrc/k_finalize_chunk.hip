// Launcher of the two finalize passes around the contact-parallel polish
// (KArgs::fin_mode 1: budgeted one-lane polish that hands unfinished QPs on;
// 2: outputs of the QPs it handed on), gamma = 0.
#include "bodex_kernels.h"
#include "bodex_launch.h"

namespace bodex {

template <int MODE>
hipError_t launch_finalize_mode(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    switch (mm) {
        case 4: hipLaunchKernelGGL((finalize_kernel<4, false, MODE>), dim3(grid), dim3(64), lds, st, a); break;
        case 5: hipLaunchKernelGGL((finalize_kernel<5, false, MODE>), dim3(grid), dim3(64), lds, st, a); break;
        case 6: hipLaunchKernelGGL((finalize_kernel<6, false, MODE>), dim3(grid), dim3(64), lds, st, a); break;
        case 7: hipLaunchKernelGGL((finalize_kernel<7, false, MODE>), dim3(grid), dim3(64), lds, st, a); break;
        case 8: hipLaunchKernelGGL((finalize_kernel<8, false, MODE>), dim3(grid), dim3(64), lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_finalize_chunk(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    if (a.fin_mode == 1) return launch_finalize_mode<1>(mm, a, grid, lds, st);
    if (a.fin_mode == 2) return launch_finalize_mode<2>(mm, a, grid, lds, st);
    return hipErrorInvalidValue;
}

}  // namespace bodex
