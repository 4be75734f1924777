// Launcher of the contact-parallel polish for the compiled contact counts
// (one lane per contact: groups of 4 lanes up to 4 contacts, 8 up to 8).
#include "bodex_kernels.h"
#include "bodex_launch.h"

namespace bodex {

int gpolish_group(int mm) { return mm <= 4 ? 4 : 8; }

hipError_t launch_gpolish(int mm, const KArgs& a, int grid, hipStream_t st) {
    switch (mm) {
        case 4: hipLaunchKernelGGL((gpolish_kernel<4, 4>), dim3(grid), dim3(64), 0, st, a); break;
        case 5: hipLaunchKernelGGL((gpolish_kernel<5, 8>), dim3(grid), dim3(64), 0, st, a); break;
        case 6: hipLaunchKernelGGL((gpolish_kernel<6, 8>), dim3(grid), dim3(64), 0, st, a); break;
        case 7: hipLaunchKernelGGL((gpolish_kernel<7, 8>), dim3(grid), dim3(64), 0, st, a); break;
        case 8: hipLaunchKernelGGL((gpolish_kernel<8, 8>), dim3(grid), dim3(64), 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bodex
