// Launcher of the finalize kernel for the circular-cone form.
#include "bodex_kernels.h"
#include "bodex_launch.h"

namespace bodex {

hipError_t launch_finalize_cone(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st) {
    const bool gam = a.gamma > 0.f;
    switch (mm) {
        case 4:
            if (gam)
                hipLaunchKernelGGL((cone_finalize_kernel<4, true>), dim3(grid), dim3(64), lds, st, a);
            else
                hipLaunchKernelGGL((cone_finalize_kernel<4, false>), dim3(grid), dim3(64), lds, st, a);
            break;
        case 5:
            if (gam)
                hipLaunchKernelGGL((cone_finalize_kernel<5, true>), dim3(grid), dim3(64), lds, st, a);
            else
                hipLaunchKernelGGL((cone_finalize_kernel<5, false>), dim3(grid), dim3(64), lds, st, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t cone_fin_lds(int mm, int slots, bool gam) {
    switch (mm) {
        case 4: return ConeFinLds<4>::bytes(slots, gam);
        case 5: return ConeFinLds<5>::bytes(slots, gam);
    }
    return 0;
}

}  // namespace bodex
