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
// Contact-parallel polish of the records the first finalize pass handed on
// (KArgs::spill); group size (lanes per QP) for a kernel size.
hipError_t launch_gpolish(int mm, const KArgs& a, int grid, hipStream_t st);
int gpolish_group(int mm);
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

// Floating hand over an analytic object (coarse stage): arrays [G][M][...];
// counts may be null (all M).  The query writes points, normals (and dist if
// set).  The step kernel reads dLdp / dLdn (either may be null), writes the
// optional e_dist, dLdrot, dLdtrans and trace (= w_qp e_qp + w_dist E^c_d,
// e_qp may be null), updates rot / trans when `step` is set, and then, when
// `requery` is set, writes the contacts of the (new) pose like the query.
struct HandArgs {
    int G, M;
    const int* counts;
    const float *tip, *axes;
    float *rot, *trans;
    float *points, *normals, *dist;
    const float *dLdp, *dLdn, *e_qp;
    float w_qp, w_dist, radius, offset;
    float *e_dist, *dLdrot, *dLdtrans, *trace;
    float step_rot, step_trans;
    int step, requery;
    int signed_dist;  // E^c_d with the signed distance d_i instead of |c_i - p_i|
};
hipError_t launch_hand_query(const HandArgs& a, hipStream_t st);
hipError_t launch_hand_step(const HandArgs& a, hipStream_t st);
hipError_t launch_fill(float* p, int n, float v, hipStream_t st);
int hand_blocks(int G, int M);
}  // namespace bodex
