// k_hand.hip -- the step before the QP on analytic objects (arXiv 2412.16490,
// Sec. IV-B and the coarse stage of Sec. IV-C) for a floating hand whose
// fingertips share the root transform (R, T):
//
//   c_i   = R c_{i,l} + T                                   fingertip centre
//   p_i, n_i, d_i = nearest point of the ellipsoid surface sum (x_k/a_k)^2 = 1,
//                   its inward unit normal and the signed distance (> 0 outside)
//   E^c_d = sum_i (|c_i - p_i| - alpha - delta)^2           coarse distance energy
//   g_i   = (dp/dc)^T dL/dp_i + (dn/dc)^T dL/dn_i + 2 w_dist (|d_i| - alpha - delta) sgn(d_i) (dd/dc)^T
//   (|c_i - p_i| = |d_i|; sgn(0) = +1.  With signed_dist, d_i replaces |d_i|
//   and sgn is dropped, so that a fingertip inside is pushed out.)
//   dL/dT = sum_i g_i,   dL/domega = sum_i (R c_{i,l}) x g_i     (R(omega) = Exp(omega) R)
//   T <- T - eta_T dL/dT,   R <- Exp(-eta_R dL/domega) R        (descent step)
//
// Nearest point.  With D = diag(a_k^2) the nearest point is p = D (D + tI)^{-1} c
// for the root t > -a0^2 (a0 the smallest semi-axis) of
// sum_k a_k^2 c_k^2 / (a_k^2 + t)^2 = 1.  In the shifted variable u = t + a0^2
// (so that the smallest denominator carries no cancellation) the function
// h(u) = S(u)^{-1/2}, S(u) = sum_k (a_k c_k / (a_k^2 - a0^2 + u))^2, is a
// weighted power mean with exponent -2 of functions linear in u, hence concave
// and increasing: Newton's method started where h <= 1 (u = a0 |c_0|, where
// the axis-0 term alone is 1) climbs monotonically to the root without
// overshooting, and is exact in one step when one term dominates.  A point
// with c_0 = 0 inside the object may lie on the medial ridge (h >= 1 already
// at u = 0): the nearest point then has p_k = a_k^2 c_k / (a_k^2 - a0^2) off
// axis 0 and p_0 >= 0 on the surface; the exact centre returns p = a0 e_0.
// Neither has a derivative (zero Jacobians there).
//
// Jacobians (implicit function theorem on the root equation), M = (D + tI)^{-1}:
//   w = D M^2 c,  s = c^T D M^3 c,  dt/dc = w / s,
//   dp/dc = D M - w w^T / s  (symmetric),   g = M c,   dg/dc = M - M^2 c (dt/dc)^T,
//   n = -g / |g|,   dn/dc = -(I - g^ g^^T) dg/dc / |g|,   dd/dc = g^^T = -n^T.
// Everything runs in FP64 from the FP32 inputs; outputs are FP32.
//
// One thread per fingertip, whole grasps per 256-thread block; the gradient
// kernel reduces a grasp's fingertips in LDS, takes the step and re-queries
// the new pose's contacts in the same launch.
#include <hip/hip_runtime.h>

#include <cmath>

#include "bodex_hand.h"
#include "bodex_launch.h"

namespace bodex {

namespace {

constexpr int kThreads = 256;

struct Slot {
    int g, i, lg;
    bool valid;  // the thread holds a fingertip slot of the layout
    bool live;   // ... of a fingertip the grasp uses
};

__device__ inline Slot slot_of(const HandArgs& a) {
    const int gpb = kThreads / a.M;
    Slot s;
    s.lg = threadIdx.x / a.M;
    s.i = threadIdx.x - s.lg * a.M;
    s.g = blockIdx.x * gpb + s.lg;
    s.valid = s.lg < gpb && s.g < a.G;
    s.live = s.valid && s.i < (a.counts ? a.counts[s.g] : a.M);
    return s;
}

// Fingertip centre c = R c_l + T in FP64; also R c_l.
__device__ inline void tip_centre(const float* R, const float* T, const float* cl, double c[3], double rc[3]) {
    for (int r = 0; r < 3; ++r) {
        rc[r] = double(R[3 * r]) * cl[0] + double(R[3 * r + 1]) * cl[1] + double(R[3 * r + 2]) * cl[2];
        c[r] = rc[r] + double(T[r]);
    }
}

__device__ inline void store_contact(const HandArgs& a, const Slot& s, const Near* q) {
    const size_t idx = size_t(s.g) * a.M + s.i;
    for (int k = 0; k < 3; ++k) {
        a.points[idx * 3 + k] = q ? float(q->p[k]) : 0.0f;
        a.normals[idx * 3 + k] = q ? float(q->n[k]) : 0.0f;
    }
    if (a.dist) a.dist[idx] = q ? float(q->d) : 0.0f;
}

__device__ inline void load_axes(const HandArgs& a, int g, double ax[3]) {
    for (int k = 0; k < 3; ++k) ax[k] = a.axes[size_t(g) * 3 + k];
}

__global__ __launch_bounds__(kThreads) void hand_query_kernel(HandArgs a) {
    const Slot s = slot_of(a);
    if (!s.valid) return;
    if (!s.live) {
        store_contact(a, s, nullptr);
        return;
    }
    double c[3], rc[3], ax[3];
    tip_centre(a.rot + size_t(s.g) * 9, a.trans + size_t(s.g) * 3, a.tip + (size_t(s.g) * a.M + s.i) * 3, c, rc);
    load_axes(a, s.g, ax);
    Near q;
    nearest(c, ax, q);
    store_contact(a, s, &q);
}

__global__ __launch_bounds__(kThreads) void hand_step_kernel(HandArgs a) {
    __shared__ double red[kThreads][7];
    __shared__ float pose[kThreads][12];
    const Slot s = slot_of(a);
    const int tid = threadIdx.x;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    if (s.live) {
        const size_t idx = size_t(s.g) * a.M + s.i;
        double c[3], rc[3], ax[3];
        tip_centre(a.rot + size_t(s.g) * 9, a.trans + size_t(s.g) * 3, a.tip + idx * 3, c, rc);
        load_axes(a, s.g, ax);
        Near q;
        nearest(c, ax, q);
        // |c - p| = |d| (the paper's form), or the signed distance itself
        const double sg = (a.signed_dist || q.d >= 0.0) ? 1.0 : -1.0;
        const double r = sg * q.d - double(a.radius) - double(a.offset);
        double gi[3] = {0.0, 0.0, 0.0};
        if (q.jac) {
            double vp[3], vn[3];
            if (a.dLdp)
                for (int k = 0; k < 3; ++k) vp[k] = a.dLdp[idx * 3 + k];
            if (a.dLdn)
                for (int k = 0; k < 3; ++k) vn[k] = a.dLdn[idx * 3 + k];
            chain(c, ax, q, a.dLdp ? vp : nullptr, a.dLdn ? vn : nullptr, gi);
            for (int k = 0; k < 3; ++k) gi[k] += 2.0 * double(a.w_dist) * r * sg * q.gh[k];
        }
        acc[0] = gi[0];
        acc[1] = gi[1];
        acc[2] = gi[2];
        acc[3] = rc[1] * gi[2] - rc[2] * gi[1];
        acc[4] = rc[2] * gi[0] - rc[0] * gi[2];
        acc[5] = rc[0] * gi[1] - rc[1] * gi[0];
        acc[6] = r * r;
    }
    for (int k = 0; k < 7; ++k) red[tid][k] = acc[k];
    __syncthreads();
    if (s.valid && s.i == 0) {
        double sum[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int j = 0; j < a.M; ++j)
            for (int k = 0; k < 7; ++k) sum[k] += red[tid + j][k];
        const int g = s.g;
        if (a.e_dist) a.e_dist[g] = float(sum[6]);
        if (a.dLdtrans)
            for (int k = 0; k < 3; ++k) a.dLdtrans[size_t(g) * 3 + k] = float(sum[k]);
        if (a.dLdrot)
            for (int k = 0; k < 3; ++k) a.dLdrot[size_t(g) * 3 + k] = float(sum[3 + k]);
        if (a.trace) {
            const double eq = a.e_qp ? double(a.e_qp[g]) : 0.0;
            a.trace[g] = float(double(a.w_qp) * eq + double(a.w_dist) * sum[6]);
        }
        if (a.step) {
            double w[3], E[9];
            for (int k = 0; k < 3; ++k) w[k] = -double(a.step_rot) * sum[3 + k];
            rodrigues(w, E);
            const float* R = a.rot + size_t(g) * 9;
            float Rn[9], Tn[3];
            for (int r = 0; r < 3; ++r)
                for (int col = 0; col < 3; ++col)
                    Rn[3 * r + col] = float(E[3 * r] * R[col] + E[3 * r + 1] * R[3 + col] + E[3 * r + 2] * R[6 + col]);
            for (int k = 0; k < 3; ++k)
                Tn[k] = float(double(a.trans[size_t(g) * 3 + k]) - double(a.step_trans) * sum[k]);
            for (int k = 0; k < 9; ++k) {
                a.rot[size_t(g) * 9 + k] = Rn[k];
                pose[s.lg][k] = Rn[k];
            }
            for (int k = 0; k < 3; ++k) {
                a.trans[size_t(g) * 3 + k] = Tn[k];
                pose[s.lg][9 + k] = Tn[k];
            }
        }
    }
    if (!a.requery) return;
    __syncthreads();
    if (!s.valid) return;
    if (!s.live) {
        store_contact(a, s, nullptr);
        return;
    }
    // the stored (rounded) pose, so that the contacts are those of the pose in memory
    const float* R = a.step ? pose[s.lg] : a.rot + size_t(s.g) * 9;
    const float* T = a.step ? pose[s.lg] + 9 : a.trans + size_t(s.g) * 3;
    double c[3], rc[3], ax[3];
    tip_centre(R, T, a.tip + (size_t(s.g) * a.M + s.i) * 3, c, rc);
    load_axes(a, s.g, ax);
    Near q;
    nearest(c, ax, q);
    store_contact(a, s, &q);
}

__global__ void fill_kernel(float* p, int n, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

int hand_blocks(int G, int M) {
    const int gpb = kThreads / M;
    return (G + gpb - 1) / gpb;
}

hipError_t launch_hand_query(const HandArgs& a, hipStream_t st) {
    const int grid = hand_blocks(a.G, a.M);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(hand_query_kernel, dim3(grid), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_hand_step(const HandArgs& a, hipStream_t st) {
    const int grid = hand_blocks(a.G, a.M);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(hand_step_kernel, dim3(grid), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, int n, float v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace bodex
