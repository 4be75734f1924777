// k_detach.hip -- the fine-stage surrogate energies with the Detach trick
// (arXiv 2412.16490, Sec. IV-C, Eq. 10-11).
//
// Per contact i of grasp g, with the link transform (R, T) of its fingertip:
//   c_l = R^{-1} (c^f_w - T)            the fingertip point in the link frame
//   c'  = R c_l + T                     (c_l held constant: Detach)
//   Q'  += |c' - p^c|^2,   E^f_d += |c' - p^f|^2
//   g   = 2 w_q (c' - p^c) + 2 w_e (c' - p^f)
//   dL/dR = g c_l^T,  dL/dT = g.
//
// The kernel streams every array once (HBM-bound: 84 bytes read and 48
// written per contact with gradients).  A block takes a run of whole grasps
// whose contacts are contiguous in every array, so each array slab is loaded
// into LDS with consecutive lanes on consecutive float4s (coalesced; scalar
// words when an array is not 16-byte aligned) and each lane then reads its
// own contact from LDS; the gradient slabs go back the same way.
#include <hip/hip_runtime.h>

#include "bodex_launch.h"

namespace bodex {

namespace {

constexpr int kThreads = 256;

__device__ inline void inverse_apply(const float* R, const float* v, float* out) {
    // R^{-1} v = adj(R) v / det(R)
    const float a00 = R[4] * R[8] - R[5] * R[7];
    const float a01 = R[2] * R[7] - R[1] * R[8];
    const float a02 = R[1] * R[5] - R[2] * R[4];
    const float a10 = R[5] * R[6] - R[3] * R[8];
    const float a11 = R[0] * R[8] - R[2] * R[6];
    const float a12 = R[2] * R[3] - R[0] * R[5];
    const float a20 = R[3] * R[7] - R[4] * R[6];
    const float a21 = R[1] * R[6] - R[0] * R[7];
    const float a22 = R[0] * R[4] - R[1] * R[3];
    const float det = R[0] * a00 + R[1] * a10 + R[2] * a20;
    const float id = 1.0f / det;
    out[0] = (a00 * v[0] + a01 * v[1] + a02 * v[2]) * id;
    out[1] = (a10 * v[0] + a11 * v[1] + a12 * v[2]) * id;
    out[2] = (a20 * v[0] + a21 * v[1] + a22 * v[2]) * id;
}

// Streaming accesses: every word is read or written once, so the slabs are
// loaded and stored non-temporally.  With the default policy the counters
// showed 1.25x the algorithmic bytes read and 1.7x written (0.196 ms per
// 2^20-grasp launch); non-temporal accesses bring both to the algorithmic
// figures (0.123 ms).
__device__ inline float4 stream_load(const float4* p) {
    float4 v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    v.z = __builtin_nontemporal_load(&p->z);
    v.w = __builtin_nontemporal_load(&p->w);
    return v;
}
__device__ inline void stream_store(float4* p, float4 v) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
    __builtin_nontemporal_store(v.z, &p->z);
    __builtin_nontemporal_store(v.w, &p->w);
}

// Grasps per block: the most whole grasps whose contacts fit the block and
// number a multiple of 4, so that every slab starts on a 16-byte boundary
// (given 16-byte aligned arrays) and moves as float4.
__host__ __device__ inline int grasps_per_block(int M) {
    int g = kThreads / M;
    while ((g * M) & 3) --g;
    return g;
}

// Copy n floats (n a multiple of 4 when V4) from global src to LDS dst with
// consecutive lanes on consecutive words; all loads are issued before the
// first LDS write.
template <bool V4, int MAXN>
__device__ inline void stage_in(const float* __restrict__ src, float* dst, int n, int tid) {
    if constexpr (V4) {
        constexpr int U = (MAXN / 4 + kThreads - 1) / kThreads;
        float4 r[U];
        const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = tid + u * kThreads;
            if (k < n / 4) r[u] = stream_load(s4 + k);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = tid + u * kThreads;
            if (k < n / 4) reinterpret_cast<float4*>(dst)[k] = r[u];
        }
    } else {
        constexpr int U = (MAXN + kThreads - 1) / kThreads;
        float r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = tid + u * kThreads;
            if (k < n) r[u] = __builtin_nontemporal_load(src + k);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = tid + u * kThreads;
            if (k < n) dst[k] = r[u];
        }
    }
}

// LDS src to global dst (added to dst when acc).
template <bool V4, int MAXN>
__device__ inline void stage_out(const float* src, float* __restrict__ dst, int n, int tid, bool acc) {
    if constexpr (V4) {
        constexpr int U = (MAXN / 4 + kThreads - 1) / kThreads;
        float4* d4 = reinterpret_cast<float4*>(dst);
        const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = tid + u * kThreads;
            if (k < n / 4) {
                float4 v = s4[k];
                if (acc) {
                    const float4 o = d4[k];
                    v.x += o.x;
                    v.y += o.y;
                    v.z += o.z;
                    v.w += o.w;
                }
                stream_store(d4 + k, v);
            }
        }
    } else {
        constexpr int U = (MAXN + kThreads - 1) / kThreads;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = tid + u * kThreads;
            if (k < n) __builtin_nontemporal_store(acc ? dst[k] + src[k] : src[k], dst + k);
        }
    }
}

template <bool V4>
__global__ __launch_bounds__(kThreads) void detach_kernel(DetachArgs a) {
    __shared__ __align__(16) float sR[kThreads * 9];
    __shared__ __align__(16) float sV[4][kThreads * 3];  // T, c^f_w, p^f, p^c
    __shared__ float sq[kThreads], se[kThreads];
    const int M = a.M;
    const int gpb = grasps_per_block(M);
    const int g0 = blockIdx.x * gpb;
    const int ng = min(gpb, a.G - g0);
    const int nc = ng * M;
    const size_t c0 = size_t(g0) * M;
    const int tid = threadIdx.x;
    // a block's last slab may hold a count of floats that is not a multiple
    // of 4 only on the last block (ragged tail); it takes the scalar path
    const bool v4 = V4 && ((nc & 3) == 0);
    if (v4) {
        stage_in<true, kThreads * 9>(a.R + c0 * 9, sR, nc * 9, tid);
        stage_in<true, kThreads * 3>(a.T + c0 * 3, sV[0], nc * 3, tid);
        stage_in<true, kThreads * 3>(a.cw + c0 * 3, sV[1], nc * 3, tid);
        stage_in<true, kThreads * 3>(a.pf + c0 * 3, sV[2], nc * 3, tid);
        stage_in<true, kThreads * 3>(a.pc + c0 * 3, sV[3], nc * 3, tid);
    } else {
        stage_in<false, kThreads * 9>(a.R + c0 * 9, sR, nc * 9, tid);
        stage_in<false, kThreads * 3>(a.T + c0 * 3, sV[0], nc * 3, tid);
        stage_in<false, kThreads * 3>(a.cw + c0 * 3, sV[1], nc * 3, tid);
        stage_in<false, kThreads * 3>(a.pf + c0 * 3, sV[2], nc * 3, tid);
        stage_in<false, kThreads * 3>(a.pc + c0 * 3, sV[3], nc * 3, tid);
    }
    __syncthreads();
    float q = 0.0f, e = 0.0f, gr[3] = {0.0f, 0.0f, 0.0f}, cl[3] = {0.0f, 0.0f, 0.0f};
    if (tid < nc) {
        const int gl = tid / M;
        const int i = tid - gl * M;
        const int g = g0 + gl;
        const int cnt = a.counts ? a.counts[g] : M;
        if (i < cnt) {
            float R[9], T[3], cw[3], v[3], c[3];
#pragma unroll
            for (int k = 0; k < 9; ++k) R[k] = sR[tid * 9 + k];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                T[t] = sV[0][tid * 3 + t];
                cw[t] = sV[1][tid * 3 + t];
                v[t] = cw[t] - T[t];
            }
            inverse_apply(R, v, cl);
            const float wq = a.wq ? a.wq[g] : 0.0f;
            const float we = a.we ? a.we[g] : 0.0f;
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                c[t] = R[3 * t] * cl[0] + R[3 * t + 1] * cl[1] + R[3 * t + 2] * cl[2] + T[t];
                const float dc = c[t] - sV[3][tid * 3 + t];
                const float df = c[t] - sV[2][tid * 3 + t];
                q += dc * dc;
                e += df * df;
                gr[t] = 2.0f * (wq * dc + we * df);
            }
        }
    }
    sq[tid] = q;
    se[tid] = e;
    const bool grads = a.dR != nullptr;
    __syncthreads();  // every lane has its inputs in registers: the slabs are free
    if (grads && tid < nc) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int s = 0; s < 3; ++s) sR[tid * 9 + 3 * r + s] = gr[r] * cl[s];
#pragma unroll
        for (int t = 0; t < 3; ++t) sV[0][tid * 3 + t] = gr[t];
    }
    __syncthreads();
    if (tid < ng) {
        float sQ = 0.0f, sE = 0.0f;
        for (int i = 0; i < M; ++i) {
            sQ += sq[tid * M + i];
            sE += se[tid * M + i];
        }
        a.Qp[g0 + tid] = sQ;
        a.Ed[g0 + tid] = sE;
    }
    if (!grads) return;
    const bool acc = a.accumulate != 0;
    if (v4) {
        stage_out<true, kThreads * 9>(sR, a.dR + c0 * 9, nc * 9, tid, acc);
        stage_out<true, kThreads * 3>(sV[0], a.dT + c0 * 3, nc * 3, tid, acc);
    } else {
        stage_out<false, kThreads * 9>(sR, a.dR + c0 * 9, nc * 9, tid, acc);
        stage_out<false, kThreads * 3>(sV[0], a.dT + c0 * 3, nc * 3, tid, acc);
    }
}

}  // namespace

int detach_blocks(int G, int M) {
    const int gpb = grasps_per_block(M);
    return (G + gpb - 1) / gpb;
}

hipError_t launch_detach(const DetachArgs& a, hipStream_t st) {
    const int grid = detach_blocks(a.G, a.M);
    if (grid == 0) return hipSuccess;
    // float4 slabs need every streamed array 16-byte aligned
    const void* arrs[] = {a.R, a.T, a.cw, a.pf, a.pc, a.dR, a.dT};
    bool al16 = true;
    for (const void* p : arrs) al16 = al16 && (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
    if (al16)
        hipLaunchKernelGGL(detach_kernel<true>, dim3(grid), dim3(kThreads), 0, st, a);
    else
        hipLaunchKernelGGL(detach_kernel<false>, dim3(grid), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace bodex
