// bodex_launch.h -- launchers of the kernels, one translation unit per kernel
// family so that they compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

namespace bodex {
struct KArgs;
hipError_t launch_admm(int mm, int occ, const KArgs& a, int grid, size_t lds, hipStream_t st);
hipError_t launch_finalize(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st);
hipError_t launch_backward(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st);
hipError_t launch_reset(int* q, int n, hipStream_t st);
// Circular-cone form (KArgs::cone set).
hipError_t launch_admm_cone(int mm, int occ, const KArgs& a, int grid, size_t lds, hipStream_t st);
hipError_t launch_finalize_cone(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st);
size_t cone_fin_lds(int mm, int slots, bool gam);
hipError_t launch_backward_cone(int mm, const KArgs& a, int grid, size_t lds, hipStream_t st);

// Fine-stage surrogate energies (Detach trick): arrays [G][M][...], row-major
// 3x3 link matrices; counts, wq, we may be null (all M contacts, zero
// weights); dR and dT are both null (no gradient) or both set.
struct DetachArgs {
    int G, M;
    const int* counts;
    const float *R, *T, *cw, *pf, *pc;
    const float *wq, *we;
    float *Qp, *Ed;
    float *dR, *dT;
    int accumulate;
};
hipError_t launch_detach(const DetachArgs& a, hipStream_t st);
int detach_blocks(int G, int M);
}  // namespace bodex
