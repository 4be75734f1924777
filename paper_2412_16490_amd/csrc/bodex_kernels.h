// bodex_kernels.h -- gfx950 kernels of the batched contact-force QP.
//
// Mapping: one wavefront (64 lanes, one workgroup) per tile; a tile is a run
// of up to kMaxSlots grasps ("slots") whose wrench QPs total at most 64; each
// lane owns one wrench QP and keeps its ADMM state in VGPRs for the whole
// solve.  The grasp's shared matrices (G, the inverse KKT matrix) live in LDS
// and are read by all of the grasp's lanes.  There is no MFMA: the per-QP work
// is a 15x15 symmetric matrix-vector product plus structured row operations,
// not a dense contraction.
//
// Kernels:
//   admm_kernel      grasp matrix, per-grasp factorisation, fused ADMM loop with
//                    periodic residual checks and per-grasp rho adaptation;
//                    writes the state (x, z, y, rho), iterations and status.
//   finalize_kernel  FP64 polish (reduced KKT re-solve with dual active-set
//                    correction), objective, energy, KKT residual, outputs.
//   backward_kernel  recomputes f* from the state, Danskin gradient of the
//                    energy with respect to G, chain rule to points/normals.
#pragma once

#include <hip/hip_runtime.h>

#include "bodex_cone.h"
#include "bodex_gpolish.h"
#include "bodex_math.h"

namespace bodex {

// Keep each contact's projector in LDS between factorisations (else it is
// recomputed from the active rows where needed, which leaves more LDS for
// resident waves).
constexpr bool kProjectorCache = false;
constexpr int kMaxSlots = 12;  // keeps every kernel under 64 KB of LDS
constexpr int kWave = 64;

// Status bits (same values as the public header).
constexpr unsigned char kStConverged = 0x01;
constexpr unsigned char kStMaxIter = 0x02;
constexpr unsigned char kStNonfinite = 0x04;
constexpr unsigned char kStFp64 = 0x08;
constexpr unsigned char kStPolishRej = 0x10;
constexpr unsigned char kStPolished = 0x20;

struct KArgs {
    // inputs (device)
    const float* points;
    const float* normals;
    const float* mu;
    const float* wrench;
    const int* counts;
    const int* woff;
    // schedule (device): tile t covers perm[tile_start[t] .. tile_start[t+1])
    const int* perm;
    const int* tile_start;
    int n_tiles;
    int slots;  // max grasps per tile (sizes the dynamic LDS)
    int* queue; // persistent launch: tile counter (null = one tile per block)
    int W;
    int ms;     // array stride in contacts (m_max of the caller's layout, <= MM)
    // state and outputs (device)
    float* x;
    float* z;
    float* y;
    float* rho;
    float* forces;
    float* qobj;
    float* energy;
    float* kkt;
    int* iters;
    unsigned char* status;
    float* pflops;  // optional: polish flops per QP
    float* resid;   // optional state: [6][W] wrench residual G f - beta t of the returned forces (FP64, rounded)
    // state layout: column stride of x, z, y, resid; per grasp the column
    // of its first QP (null: its wrench offset) and its rho index (null: g)
    int sW;
    const int* sq;
    const int* sg;
    // backward
    const float* dLdE;
    const float* dLdQ;
    float* dP;
    float* dN;
    int accumulate;
    // parameters
    float kappa, beta, eps, fmax, gamma, tol, admm_tol, rho0, alpha, rho_min, rho_max, hyst, fp64_cond;
    int max_iters, check_every, warm, adaptive, polish, polish_steps;
    int cone;  // 1: exact circular cone (state rows 3 m + 1), 0: 8-facet pyramid
    // chunked polish (finalize_kernel): fin_mode 0 runs every polish to the
    // end; 1 suspends a polish after polish_budget factorisations and hands it
    // to the contact-parallel polish through the spill records (spill_idx[w]:
    // the record of QP w, -1 for none; spill_count: records taken); 2 forms
    // the outputs of the QPs whose records that polish finished
    int fin_mode, polish_budget;
    SpillPtrs spill;
    int* spill_count;
    int* spill_idx;
};

struct SlotInfo {
    int g, m, s, w0;
};

// Row r of a kernel compiled for MM contacts in the caller's state layout with
// ms <= MM contacts per grasp: rows of real contacts keep their index, the
// normal-sum row moves from 9 MM to 9 ms, rows of padding contacts have none.
template <int MM>
__device__ inline int state_row(int r, int ms) {
    if (r == 9 * MM) return 9 * ms;
    return r < 9 * ms ? r : -1;
}

// The same for the cone form (3 rows per contact, the sum row at 3 MM).
template <int MM>
__device__ inline int cone_state_row(int r, int ms) {
    if (r == 3 * MM) return 3 * ms;
    return r < 3 * ms ? r : -1;
}

// Slot of each lane: lanes of one grasp are contiguous, in slot order.
__device__ inline void lane_slot(const SlotInfo* info, int nsl, int lane, int& slot, int& j) {
    slot = -1;
    j = 0;
    int acc = 0;
    for (int k = 0; k < nsl; ++k) {
        const int s = info[k].s;
        if (lane >= acc && lane < acc + s) {
            slot = k;
            j = lane - acc;
        }
        acc += s;
    }
}

// State column of QP j of a slot's grasp, and the grasp's rho index.
__device__ inline unsigned state_col(const KArgs& a, const SlotInfo& si, int j) {
    return unsigned((a.sq ? a.sq[si.g] : si.w0) + j);
}
__device__ inline int rho_index(const KArgs& a, int g) { return a.sg ? a.sg[g] : g; }

__device__ inline int fetch_tile(const KArgs& a, int* sTile, int prev) {
    if (a.queue == nullptr) return prev < 0 ? int(blockIdx.x) : a.n_tiles;
    __syncthreads();
    if (threadIdx.x == 0) *sTile = atomicAdd(a.queue, 1);
    __syncthreads();
    return *sTile;
}

__device__ inline void load_slots(const KArgs& a, int t, SlotInfo* info, int& nsl) {
    const int gb = a.tile_start[t];
    nsl = a.tile_start[t + 1] - gb;
    if (int(threadIdx.x) < nsl) {
        SlotInfo si;
        si.g = a.perm[gb + threadIdx.x];
        si.m = a.counts[si.g];
        si.w0 = a.woff[si.g];
        si.s = a.woff[si.g + 1] - si.w0;
        info[threadIdx.x] = si;
    }
    __syncthreads();
}

// Cooperative inverse of an SPD NV x NV matrix per slot.  Every lane of the
// wave calls it (it contains barriers); lanes of slots with do_it set do the
// work.  Lw: the slot's packed-lower workspace (type T); Inv: the slot's
// packed-upper output (type O).  entry(i, c) gives the matrix.  Returns false
// on a lane whose slot hit a non-positive pivot.
template <typename T, int NV, typename O, typename Entry>
__device__ bool coop_inverse(bool do_it, int j, int s, T* Lw, O* Inv, T* yv, Entry entry) {
    // yv: this lane's solve vector in LDS, yv[i * kWave] (lane-interleaved)
    bool ok = true;
    if (do_it) {
#pragma unroll 1
        for (int i = j; i < NV; i += s)
#pragma unroll 1
            for (int c = 0; c <= i; ++c) Lw[lo_idx(i, c)] = entry(i, c);
    }
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < NV; ++k) {
        T d = T(1);
        if (do_it) {
            d = Lw[lo_idx(k, k)];
            if (!(d > T(0))) {
                ok = false;
                d = T(1);
            }
            d = sqrt(d);
            #pragma unroll 1
            for (int i = k + 1 + j; i < NV; i += s) Lw[lo_idx(i, k)] /= d;
        }
        __syncthreads();
        if (do_it) {
            #pragma unroll 1
            for (int i = k + 1 + j; i < NV; i += s) {
                const T lik = Lw[lo_idx(i, k)];
                #pragma unroll 1
                for (int c = k + 1; c <= i; ++c) Lw[lo_idx(i, c)] -= lik * Lw[lo_idx(c, k)];
            }
        }
        __syncthreads();
        if (do_it && j == 0) Lw[lo_idx(k, k)] = d;
    }
    __syncthreads();
    if (do_it) {
        // column col of the inverse: solve L L^T x = e_col (y = L^{-1} e_col
        // vanishes above col)
        #pragma unroll 1
        for (int col = j; col < NV; col += s) {
            #pragma unroll 1
            for (int i = 0; i < col; ++i) yv[i * kWave] = T(0);
            #pragma unroll 1
            for (int i = col; i < NV; ++i) {
                T acc = (i == col) ? T(1) : T(0);
                #pragma unroll 1
                for (int c = col; c < i; ++c) acc -= Lw[lo_idx(i, c)] * yv[c * kWave];
                yv[i * kWave] = acc / Lw[lo_idx(i, i)];
            }
            #pragma unroll 1
            for (int i = NV - 1; i >= 0; --i) {
                T acc = yv[i * kWave];
                #pragma unroll 1
                for (int c = i + 1; c < NV; ++c) acc -= Lw[lo_idx(c, i)] * yv[c * kWave];
                yv[i * kWave] = acc / Lw[lo_idx(i, i)];
            }
            #pragma unroll 1
            for (int i = 0; i <= col; ++i) Inv[up_idx<NV>(i, col)] = O(yv[i * kWave]);
        }
    }
    __syncthreads();
    return ok;
}

// ---------------------------------------------------------------------------
// Dynamic LDS layouts.
// ---------------------------------------------------------------------------
template <int MM>
struct AdmmLds {
    static constexpr int NV = 3 * MM, NK = NV * (NV + 1) / 2, NKP = Dims<MM>::NKP, NG = 6 * NV;
    static __host__ __device__ size_t bytes(int slots) {
        return size_t(slots) * (NKP * 4 + NG * 4 + 8 * 4 + NKP * 8) + size_t(64) * NV * 8 +
               size_t(64) * NV * 4 + 64 * 8 + kMaxSlots * 32 + 64;
    }
};

// State of one lane in the caller's layout: x, and z = Pi(w), y = rho (w - Pi(w)).
// Row bases are uniform across the wave; only the lane's offset is per lane.
template <int MM>
__device__ __forceinline__ void write_admm_x(const KArgs& a, unsigned w, const float* xv) {
    constexpr int NV = 3 * MM;
    asm volatile("" : "+v"(w));
#pragma unroll
    for (int c = 0; c < NV; ++c)
        if (c < 3 * a.ms) (a.x + size_t(c) * a.sW)[w] = xv[c];
}

template <int MM, bool CONE>
__device__ __forceinline__ void write_admm_zy(const KArgs& a, unsigned w, const float* wv, const float* muc,
                                              float rho) {
    asm volatile("" : "+v"(w));
    if constexpr (CONE) {
        constexpr int NR = 3 * MM + 1;
        float muv[MM], zv[NR];
#pragma unroll
        for (int i = 0; i < MM; ++i) muv[i] = muc[i];
        cone_proj_all<MM>(wv, muv, a.fmax, a.gamma, zv);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int sr = cone_state_row<MM>(r, a.ms);
            if (sr >= 0) {
                (a.z + size_t(sr) * a.sW)[w] = zv[r];
                (a.y + size_t(sr) * a.sW)[w] = rho * (wv[r] - zv[r]);
            }
        }
    } else {
        constexpr int NR = 9 * MM + 1;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r % 9 == 0) BODEX_SPLIT();
            const int sr = state_row<MM>(r, a.ms);
            const float zr = row_proj(r, MM, wv[r], a.fmax, a.gamma);
            if (sr >= 0) {
                (a.z + size_t(sr) * a.sW)[w] = zr;
                (a.y + size_t(sr) * a.sW)[w] = rho * (wv[r] - zr);
            }
        }
    }
}

// (Re)factor K = P + rho A^T A of the slots with `mine` set and store K^{-1}
// (packed upper, FP32) in LDS.  The factorisation is FP32, or FP64 for slots
// whose conditioning bound exceeds fp64_cond.  Called by every lane of the
// wave (barriers inside).  Returns bit 1 if this lane's slot used FP64, bit 2
// if its factorisation failed.
template <int MM, bool CONE>
__device__ __forceinline__ int refactor_slots(const KArgs& a, bool mine, int slot, int j, int s, int m,
                                              float rho, const float* sG, const float* sMuc, double* sLw,
                                              float* sKi, double* sYv, int* sMisc) {
    constexpr int NV = 3 * MM, NKP = Dims<MM>::NKP, NG = 6 * NV;
    const float* Gs = sG + size_t(slot) * NG;
    const float* mucs = sMuc + slot * 8;
    if (threadIdx.x == 0) sMisc[1] = 0;
    __syncthreads();
    bool want64 = false;
    if (mine) {
        const float cb = CONE ? cone_kkt_cond_bound<float, NV>(Gs, m, rho, a.eps)
                              : kkt_cond_bound<float, NV>(Gs, mucs, m, rho, a.eps);
        want64 = !(cb <= a.fp64_cond);
        if (want64) atomicOr(&sMisc[1], 1);
    }
    __syncthreads();
    const bool any64 = sMisc[1] != 0;
    double* Lw = sLw + size_t(slot) * NKP;
    float* Ki = sKi + size_t(slot) * NKP;
    bool ok = true;
    if (any64) {
        const double rr = double(rho), eps = double(a.eps);
        ok = coop_inverse<double, NV>(mine && want64, j, s, Lw, Ki, sYv + threadIdx.x, [&](int i, int c) {
            const int ci = i / 3, cj = c / 3;
            if (ci >= m || cj >= m) return (i == c) ? 1.0 : 0.0;
            double sacc = 0.0;
            for (int r = 0; r < 6; ++r) sacc += double(Gs[r * NV + i]) * double(Gs[r * NV + c]);
            double v = 2.0 * sacc + ((i == c) ? 2.0 * eps : 0.0);
            if (CONE) {
                if (i == c) v += rr;
                if (i % 3 == 0 && c % 3 == 0) v += rr;
            } else if (i % 3 == 0 && c % 3 == 0) {
                v += (ci == cj) ? rr * (8.0 * double(mucs[ci]) * double(mucs[ci]) + 2.0) : rr;
            } else if (i == c) {
                v += 4.0 * rr;
            }
            return v;
        });
    }
    float* Lf = reinterpret_cast<float*>(Lw);
    const float eps32 = a.eps;
    float* yf = reinterpret_cast<float*>(sYv) + threadIdx.x;
    const bool ok32 = coop_inverse<float, NV>(mine && !want64, j, s, Lf, Ki, yf, [&](int i, int c) {
        return CONE ? cone_kkt_entry<float, NV>(Gs, m, rho, eps32, i, c)
                    : kkt_entry<float, NV>(Gs, mucs, m, rho, eps32, i, c);
    });
    int r = 0;
    if (mine && want64) r |= 1;
    if (mine && !(ok && ok32)) r |= 2;
    return r;
}

// ---------------------------------------------------------------------------
// ADMM kernel.
// ---------------------------------------------------------------------------
// OCC: register budget expressed as resident waves per SIMD (1 = unlimited).
// CONE: the exact circular cone (3 MM + 1 state rows), else the 8-facet
// pyramid (9 MM + 1 rows).
template <int MM, int OCC, bool CONE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(OCC))) admm_kernel(const KArgs a) {
    constexpr int NV = 3 * MM, NR = CONE ? 3 * MM + 1 : 9 * MM + 1, NK = NV * (NV + 1) / 2;
    constexpr int NKP = Dims<MM>::NKP, NG = 6 * NV;
    extern __shared__ __align__(16) unsigned char smem[];
    const int S = a.slots;
    // carve: Lw (double) first for alignment
    double* sLw = reinterpret_cast<double*>(smem);                       // [S][NKP]
    double* sYv = sLw + size_t(S) * NKP;                                  // [NV][64]
    float* sKi = reinterpret_cast<float*>(sYv + size_t(NV) * kWave);     // [S][NKP]
    float* sBq = sKi + size_t(S) * NKP;                                   // [NV][64]
    float* sG = sBq + size_t(NV) * kWave;                                 // [S][NG]
    float* sMuc = sG + size_t(S) * NG;                                    // [S][8]
    float* sRp = sMuc + size_t(S) * 8;                                    // [64]
    float* sRd = sRp + 64;                                                // [64]
    SlotInfo* sInfo = reinterpret_cast<SlotInfo*>(sRd + 64);              // [kMaxSlots]
    int* sFlag = reinterpret_cast<int*>(sInfo + kMaxSlots);               // [kMaxSlots]
    float* sRho = reinterpret_cast<float*>(sFlag + kMaxSlots);            // [kMaxSlots]
    int* sMisc = reinterpret_cast<int*>(sRho + kMaxSlots);                // [4]

    const int lane = threadIdx.x;
    for (int t = fetch_tile(a, sMisc, -1); t < a.n_tiles; t = fetch_tile(a, sMisc, t)) {
        int nsl;
        load_slots(a, t, sInfo, nsl);
        int slot, j;
        lane_slot(sInfo, nsl, lane, slot, j);
        const bool act = slot >= 0;
        SlotInfo si = {0, 0, 1, 0};
        if (act) si = sInfo[slot];
        const int m = si.m;
        const int w = si.w0 + j;
        const unsigned sw = state_col(a, si, j);  // this QP's state column

        // --- grasp matrix, friction terms, initial rho -----------------------
        for (int e = lane; e < nsl * NG; e += kWave) sG[e] = 0.f;
        for (int e = lane; e < nsl * 8; e += kWave) sMuc[e] = 0.f;
        if (lane < nsl) sFlag[lane] = 0;
        __syncthreads();
        if (act) {
            for (int c = j; c < m; c += si.s) {
                const size_t base = (size_t(si.g) * a.ms + c) * 3;
                const float p[3] = {a.points[base], a.points[base + 1], a.points[base + 2]};
                const float n[3] = {a.normals[base], a.normals[base + 1], a.normals[base + 2]};
                const float mu = a.mu[size_t(si.g) * a.ms + c];
                const bool ok = grasp_columns<float, NV>(p, n, a.kappa, c, sG + size_t(slot) * NG);
                sMuc[slot * 8 + c] = CONE ? mu : mu * float(kC8);
                if (!ok || !(mu > 0.f) || !isfinite(mu)) atomicOr(&sFlag[slot], 4);
            }
            if (j == 0) {
                float r0 = a.rho0;
                if (a.warm) {
                    const float rw = a.rho[rho_index(a, si.g)];
                    if (rw > 0.f && isfinite(rw)) r0 = rw;
                }
                sRho[slot] = fminf(fmaxf(r0, a.rho_min), a.rho_max);
            }
        }
        __syncthreads();
        const float* Gs = sG + size_t(act ? slot : 0) * NG;
        const float* muc = sMuc + (act ? slot : 0) * 8;
        bool bad = act && (sFlag[slot] & 4);
        float rho = act ? sRho[slot] : 1.f;
        const unsigned wl = unsigned(w);

        // --- per-lane right-hand side (in LDS) and initial state ---------------
        const Strided<float> bq{sBq + lane, kWave};
        {
            float tw[6];
#pragma unroll
            for (int r = 0; r < 6; ++r) tw[r] = act ? a.wrench[size_t(wl) * 6 + r] : 0.f;
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                if (c % 3 == 0) BODEX_SPLIT();
                float acc = 0.f;
#pragma unroll
                for (int r = 0; r < 6; ++r) acc = fmaf(Gs[r * NV + c], tw[r], acc);
                bq[c] = 2.f * a.beta * acc;
            }
        }
        float wv[NR];
        float xv[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) xv[c] = 0.f;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r % 9 == 0) BODEX_SPLIT();
            float v = 0.f;
            const int sr = CONE ? cone_state_row<MM>(r, a.ms) : state_row<MM>(r, a.ms);
            if (act && a.warm && sr >= 0) {
                const float zr = (a.z + size_t(sr) * a.sW)[sw], yr = (a.y + size_t(sr) * a.sW)[sw];
                v = zr + yr / rho;
            }
            wv[r] = isfinite(v) ? v : 0.f;
        }

        // --- factorisation ------------------------------------------------------
        unsigned char stbits = 0;
        {
            const int fr = refactor_slots<MM, CONE>(a, act && !bad, act ? slot : 0, j, si.s, m, rho, sG, sMuc,
                                                    sLw, sKi, sYv, sMisc);
            if (fr & 1) stbits |= kStFp64;
            if (fr & 2) bad = true;
        }

        // --- ADMM loop ----------------------------------------------------------
        bool done = !act || bad;
        int it_done = 0;
        float rel_last = INFINITY;
        float rho_frz = rho;  // rho at which a converged lane's w was frozen
        if (act && bad) {
            stbits |= kStNonfinite;
            it_done = 0;
        }
        const float* Ki = sKi + size_t(act ? slot : 0) * NKP;

        int it = 0;
        for (it = 1; it <= a.max_iters; ++it) {
            BODEX_SPLIT();
            if (!done) {
                float rhs[NV];
                if constexpr (CONE) {
                    float pv[NR];
                    cone_rhs<MM>(wv, bq, muc, rho, a.fmax, a.gamma, m, pv, rhs);
                    symv_packed<NV>(Ki, rhs, xv);
                    cone_update<MM>(wv, xv, pv, a.alpha, m);
                } else {
                    admm_rhs<MM>(wv, bq, muc, rho, a.fmax, a.gamma, m, rhs);
                    symv_packed<NV>(Ki, rhs, xv);
                    admm_update<MM>(wv, xv, muc, a.alpha, a.fmax, a.gamma, m);
                }
            }
            if (it % a.check_every != 0 && it != a.max_iters) continue;
            float rpn = -1.f, rdn = -1.f;
            if (!done) {
                const Residual R = CONE ? cone_residual<MM>(wv, xv, bq, muc, Gs, rho, a.eps, a.fmax, a.gamma, m)
                                        : admm_residual<MM>(wv, xv, bq, muc, Gs, rho, a.eps, a.fmax, a.gamma, m);
                rel_last = R.rel;
                if (!isfinite(R.rel)) {
                    done = true;
                    stbits |= kStNonfinite;
                    it_done = it;
                } else if (R.rel <= a.admm_tol) {
                    done = true;
                    stbits |= kStConverged;
                    it_done = it;
                    rho_frz = rho;
                    write_admm_x<MM>(a, sw, xv);
                } else {
                    rpn = R.rp_n;
                    rdn = R.rd_n;
                }
            }
            if (__all(done)) break;
            if (!a.adaptive || it == a.max_iters) continue;
            // per-grasp rho from the largest normalised residuals of live lanes
            sRp[lane] = rpn;
            sRd[lane] = rdn;
            if (lane < nsl) sFlag[lane] &= ~1;
            __syncthreads();
            if (act && j == 0) {
                float mp = -1.f, md = -1.f;
                for (int l = lane; l < lane + si.s; ++l) {
                    mp = fmaxf(mp, sRp[l]);
                    md = fmaxf(md, sRd[l]);
                }
                if (mp > 0.f && md > 0.f) {
                    float rn = rho * sqrtf(mp / md);
                    rn = fminf(fmaxf(rn, a.rho_min), a.rho_max);
                    if (rn > a.hyst * rho || rn < rho / a.hyst) {
                        sRho[slot] = rn;
                        sFlag[slot] |= 1;
                    }
                }
            }
            __syncthreads();
            int anyf = 0;
            for (int k = 0; k < nsl; ++k) anyf |= sFlag[k] & 1;
            if (!anyf) continue;
            const bool mine = act && !bad && (sFlag[slot] & 1);
            if (mine) {
                const float rn = sRho[slot];
                if (!done) {
                    // keep (z, y): w' = z + y / rho'
                    if constexpr (CONE) {
                        float muv[MM], zv[NR];
#pragma unroll
                        for (int i = 0; i < MM; ++i) muv[i] = muc[i];
                        cone_proj_all<MM>(wv, muv, a.fmax, a.gamma, zv);
#pragma unroll
                        for (int r = 0; r < NR; ++r) wv[r] = zv[r] + (rho / rn) * (wv[r] - zv[r]);
                    } else {
#pragma unroll
                        for (int r = 0; r < NR; ++r) {
                            const float zr = row_proj(r, MM, wv[r], a.fmax, a.gamma);
                            wv[r] = zr + (rho / rn) * (wv[r] - zr);
                        }
                    }
                }
                rho = rn;
            }
            {
                const int fr = refactor_slots<MM, CONE>(a, mine, act ? slot : 0, j, si.s, m, rho, sG, sMuc, sLw,
                                                        sKi, sYv, sMisc);
                if (fr & 1) stbits |= kStFp64;
                if ((fr & 2) && mine && !done) {
                    done = true;
                    stbits |= kStNonfinite;
                    it_done = it;
                }
            }
        }
        if (act && !(stbits & (kStConverged | kStNonfinite))) {
            stbits |= kStMaxIter;
            it_done = a.max_iters;
            rho_frz = rho;
            write_admm_x<MM>(a, sw, xv);
        }
        if (act && (stbits & kStNonfinite)) {
#pragma unroll
            for (int c = 0; c < NV; ++c) xv[c] = NAN;
#pragma unroll
            for (int r = 0; r < NR; ++r) wv[r] = NAN;
            rel_last = NAN;
            write_admm_x<MM>(a, sw, xv);
        }
        if (act) write_admm_zy<MM, CONE>(a, sw, wv, muc, rho_frz);
        if (act) {
            a.iters[w] = it_done;
            a.status[w] = stbits;
            a.kkt[w] = rel_last;
            if (j == 0) a.rho[rho_index(a, si.g)] = rho;
        }
    }
}

// ---------------------------------------------------------------------------
// Shared FP64 setup of the finalize and backward kernels: per slot the grasp
// matrix G and mu_i cos(pi/8).
// ---------------------------------------------------------------------------
template <int MM>
struct FinLds {
    static constexpr int NV = 3 * MM, NG = 6 * NV;
    // per lane, lane-interleaved: the polish's x, z (2 NV) and, when
    // kProjectorCache, the projector cache (3 MM)
    static constexpr int NW = (2 * NV + (kProjectorCache ? 3 * MM : 0)) * kWave;
    // per slot: G64, muc64 (8); the polish space; finalize: the energy
    // reduction (one per lane); backward: Gbar per slot, and the gradient
    // reduction 6 + NV per lane, which reuses the polish space once every
    // lane has finished it.
    static __host__ __device__ size_t bytes(int slots, bool bwd) {
        return size_t(slots) * (NG + 8) * 8 + size_t(NW) * 8 + (bwd ? size_t(slots) * NG * 8 : size_t(kWave) * 8) +
               kMaxSlots * 32 + 64;
    }
};

template <int MM>
struct FinPtrs {
    double *G, *muc, *work, *Gbar, *red;
    SlotInfo* info;
    int* flag;
};

template <int MM>
__device__ inline FinPtrs<MM> fin_carve(unsigned char* smem, int S, bool bwd) {
    constexpr int NV = FinLds<MM>::NV, NG = FinLds<MM>::NG, NW = FinLds<MM>::NW;
    static_assert(kWave * (6 + NV) <= NW, "reduction buffer must fit in the polish space");
    FinPtrs<MM> P;
    double* d = reinterpret_cast<double*>(smem);
    P.G = d;
    d += size_t(S) * NG;
    P.muc = d;
    d += size_t(S) * 8;
    P.work = d;
    d += NW;
    if (bwd) {
        P.Gbar = d;
        d += size_t(S) * NG;
        P.red = P.work;
    } else {
        P.Gbar = nullptr;
        P.red = d;
        d += kWave;
    }
    P.info = reinterpret_cast<SlotInfo*>(d);
    P.flag = reinterpret_cast<int*>(P.info + kMaxSlots);
    return P;
}

// This lane's polish vectors and projector cache in the polish space.
template <int MM>
__device__ inline PolishWork<LaneVec> polish_work(const FinPtrs<MM>& P, int lane) {
    constexpr int NV = 3 * MM;
    PolishWork<LaneVec> W;
    W.x = LaneVec{P.work + lane, kWave};
    W.z = LaneVec{P.work + NV * kWave + lane, kWave};
    return W;
}

template <int MM>
__device__ inline LaneVec projector_cache(const FinPtrs<MM>& P, int lane) {
    if (!kProjectorCache) return LaneVec{nullptr, 0};
    return LaneVec{P.work + 2 * 3 * MM * kWave + lane, kWave};
}

// Returns whether the lane's grasp has finite, valid inputs.
template <int MM>
__device__ inline bool fin_setup(const KArgs& a, const FinPtrs<MM>& P, int nsl, int slot, int j,
                                 const SlotInfo& si, bool cone = false) {
    constexpr int NV = 3 * MM, NG = 6 * NV;
    const int lane = threadIdx.x;
    const bool act = slot >= 0;
    for (int e = lane; e < nsl * NG; e += kWave) P.G[e] = 0.0;
    for (int e = lane; e < nsl * 8; e += kWave) P.muc[e] = 0.0;
    if (lane < nsl) P.flag[lane] = 0;
    __syncthreads();
    if (act) {
        for (int c = j; c < si.m; c += si.s) {
            const size_t base = (size_t(si.g) * a.ms + c) * 3;
            const double p[3] = {a.points[base], a.points[base + 1], a.points[base + 2]};
            const double n[3] = {a.normals[base], a.normals[base + 1], a.normals[base + 2]};
            const double mu = a.mu[size_t(si.g) * a.ms + c];
            const bool ok = grasp_columns<double, NV>(p, n, double(a.kappa), c, P.G + size_t(slot) * NG);
            P.muc[slot * 8 + c] = cone ? mu : mu * kC8;
            if (!ok || !(mu > 0.0) || !isfinite(mu)) atomicOr(&P.flag[slot], 4);
        }
    }
    __syncthreads();
    return act && !(P.flag[slot] & 4);
}

// Lane-strided accessor for the ADMM-form duals in global memory.
template <int MM>
struct StridedY {
    const float* base;
    size_t stride;
    int ms;
    __device__ float operator[](int r) const {
        const int sr = state_row<MM>(r, ms);
        return sr >= 0 ? base[size_t(sr) * stride] : 0.f;
    }
};

template <int MM, bool GAM>
using LdsPolishData = PolishData<MM, const double*, GAM>;

template <int MM, bool GAM>
__device__ inline LdsPolishData<MM, GAM> polish_data(const KArgs& a, const FinPtrs<MM>& P, int slot,
                                                     const SlotInfo& si, const double* bt) {
    constexpr int NG = 6 * 3 * MM;
    LdsPolishData<MM, GAM> D;
    D.G = P.G + size_t(slot) * NG;
    D.muc = P.muc + slot * 8;
#pragma unroll
    for (int r = 0; r < 6; ++r) D.bt[r] = bt[r];
    D.m = si.m;
    D.fmax = a.fmax;
    D.gamma = a.gamma;
    D.eps = a.eps;
    return D;
}

// ---------------------------------------------------------------------------
// Finalize kernel: polish, objective, energy, KKT residual, outputs.  GAM:
// the polish handles the normal-sum row (gamma > 0).
// ---------------------------------------------------------------------------
// Resident waves per SIMD the finalize kernel is compiled for (its register
// budget): 2 leaves 256 VGPRs per lane.
#ifndef BODEX_FIN_WAVES
#define BODEX_FIN_WAVES 2
#endif
// Chunked first pass: once at most this many lanes of a wave are still
// polishing, each hands its QP on at its next factorisation (the wave would
// otherwise run for its slowest lanes alone; the contact-parallel polish
// finishes them with eight lanes each).  Measured at ellipsoid-m5-s16: 8
// lanes cut the solve at 8192 grasps from 1.94 to 1.86 ms and at 4096 from
// 1.55 to 1.47 ms (4 and 12 lanes less, larger budgets slower).
#ifndef BODEX_FIN_STRAGGLERS
#define BODEX_FIN_STRAGGLERS 8
#endif
constexpr int kFinStragglers = BODEX_FIN_STRAGGLERS;

template <int MM, bool GAM, int MODE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(BODEX_FIN_WAVES))) finalize_kernel(const KArgs a) {
    constexpr int NG = 6 * 3 * MM;
    extern __shared__ __align__(16) unsigned char smem[];
    const FinPtrs<MM> P = fin_carve<MM>(smem, a.slots, false);
    const int lane = threadIdx.x;
    const PolishWork<LaneVec> W = polish_work<MM>(P, lane);
    // chunked polish (gamma = 0 only; MODE is KArgs::fin_mode): 1 = hand
    // unfinished polishes on, 2 = outputs of the QPs the contact-parallel
    // polish finished
    static_assert(MODE == 0 || !GAM, "the chunked polish has no normal-sum row");
    constexpr int mode = MODE;
    __shared__ int sTile;
    for (int t = fetch_tile(a, &sTile, -1); t < a.n_tiles; t = fetch_tile(a, &sTile, t)) {
        int nsl;
        load_slots(a, t, P.info, nsl);
        int slot, j;
        lane_slot(P.info, nsl, lane, slot, j);
        const bool act = slot >= 0;
        SlotInfo si = {0, 0, 1, 0};
        if (act) si = P.info[slot];
        const int w = si.w0 + j;
        // this lane's spill record (-1: none)
        int kspill = (act && mode == 2) ? a.spill_idx[w] : -1;
        if (mode == 2 && !__syncthreads_or(kspill >= 0)) continue;  // nothing handed on in this tile
        const bool good = fin_setup<MM>(a, P, nsl, slot, j, si);
        double Q = 0.0;
        bool skip = false;  // no outputs from this lane in this pass
        if (act) {
            const double* Gs = P.G + size_t(slot) * NG;
            const double* muc = P.muc + slot * 8;
            const size_t W_ = size_t(a.sW);  // state stride
            const size_t sw = state_col(a, si, j);
            double bt[6];
#pragma unroll
            for (int r = 0; r < 6; ++r) bt[r] = double(a.beta) * double(a.wrench[size_t(w) * 6 + r]);
            unsigned char st = a.status[w];
            bool polished = false;
            const bool finite_in = good && !(st & kStNonfinite);
            const LdsPolishData<MM, GAM> D = polish_data<MM, GAM>(a, P, slot, si, bt);
            // the polish's result: point in W.x, active set, normal-sum multiplier, counts
            ActiveSet<MM> S;
            S.pc = projector_cache<MM>(P, lane);
            double lg = 0.0;
            PolishOut po;
            bool ran = false;
            if constexpr (mode == 2) {
                skip = kspill < 0;
                if (!skip) {
                    // the finished polish from the record
#pragma unroll 1
                    for (int c = 0; c < 3 * si.m; ++c) W.x[c] = a.spill.dv(c, kspill);
                    unsigned mw[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) mw[q] = unsigned(a.spill.iv(kSpMask0 + q, kspill));
                    S.mask = mask_from_words<RowMask<MM>>(mw);
                    S.gam = false;
                    po.status = a.spill.iv(kSpStatus, kspill);
                    po.steps = a.spill.iv(kSpSteps, kspill);
                    po.updates = a.spill.iv(kSpUpdates, kspill);
                    po.eqps = a.spill.iv(kSpEqps, kspill);
                    po.moves = a.spill.iv(kSpMoves, kspill);
                    po.picks = a.spill.iv(kSpPicks, kspill);
                    ran = true;
                }
            } else if (finite_in && a.polish) {
                PolishState<MM> PS;
                PS.S.pc = S.pc;
                const StridedY<MM> y0{a.y + sw, W_, a.ms};
                if constexpr (mode == 0) {
                    polish_qp<MM>(D, y0, a.polish_steps, W, PS);
                } else {
                    polish_begin<MM>(D, y0, PS);
                    PS.budget = a.polish_budget;
#pragma unroll 1
                    for (;;) {
#pragma unroll 1
                        do {
#pragma unroll 1
                            while (!polish_advance<MM, LdsPolishData<MM, GAM>, LaneVec, true>(D, a.polish_steps, W,
                                                                                              PS)) {
                                // at most kFinStragglers lanes of the wave still
                                // polishing: each hands its QP on at its next
                                // factorisation instead of keeping the wave
                                if (kFinStragglers > 0 && __popcll(__ballot(1)) <= kFinStragglers)
                                    PS.budget = min(PS.budget, PS.out.steps);
                            }
                        } while (!polish_finish<MM>(D, W, PS));
                        if (PS.out.status != kPolishSuspended) break;
                        // hand it on if a record is free, else finish it here
                        const int k = atomicAdd(a.spill_count, 1);
                        if (k < a.spill.K) {
                            polish_save<MM>(PS, W.x, si.m, a.spill, k, w, si.g);
                            kspill = k;
                            break;
                        }
                        PS.out.status = 0;
                        PS.budget = 0x7fffffff;
                    }
                }
                skip = kspill >= 0;
                ran = !skip;
                S.mask = PS.S.mask;
                S.gam = PS.S.gam;
                lg = PS.lg;
                po = PS.out;
            }
            if (mode == 1) a.spill_idx[w] = kspill;
            if (!skip) {
                if (ran) {
                    if (a.pflops) a.pflops[w] = float(polish_flops(si.m, po));
                    if (po.status == 0) {
                        polished = true;
                        st |= kStPolished;
                        st &= ~kStPolishRej;
                        // ADMM-form state of the polished point: z = A x projected
                        // on [l, u] (the bound itself on active rows), y = the
                        // multipliers of the active rows
                        double s1 = 0.0, r6[6];
                        g_times<MM>(D, W.x, true, r6);
                        const PendingRow none = {-1, -1, {0.0, 0.0, 0.0}, 0.0};
#pragma unroll 1
                        for (int i = 0; i < a.ms; ++i) {
                            const bool live = i < si.m;
                            const double f[3] = {live ? W.x[3 * i] : 0.0, live ? W.x[3 * i + 1] : 0.0,
                                                 live ? W.x[3 * i + 2] : 0.0};
                            const unsigned mk = live ? contact_mask(S.mask, i) : 0u;
                            double lam[3] = {0.0, 0.0, 0.0};
                            if (live) {
                                ContactRows R;
                                contact_rows(mk, muc[i], D.fmax, R);
                                contact_multipliers<MM>(D, R, W.x, r6, i, none, 0.0, lg, lam);
                            }
#pragma unroll
                            for (int c = 0; c < 3; ++c) a.x[size_t(3 * i + c) * W_ + sw] = float(f[c]);
#pragma unroll
                            for (int kk = 0; kk < 9; ++kk) {
                                const double zz = (kk < 8) ? facet_cos<double>(kk) * f[1] +
                                                                 facet_sin<double>(kk) * f[2] - muc[i] * f[0]
                                                           : f[0];
                                const bool on = (mk >> kk) & 1u;
                                const int jr = __builtin_popcount(mk & ((1u << kk) - 1u));
                                const float zv = on ? (kk == 8 ? a.fmax : 0.f)
                                                    : row_proj(9 * i + kk, MM, float(zz), a.fmax, a.gamma);
                                const float yv = on ? float(jr == 0 ? lam[0] : (jr == 1 ? lam[1] : lam[2])) : 0.f;
                                a.z[size_t(9 * i + kk) * W_ + sw] = zv;
                                a.y[size_t(9 * i + kk) * W_ + sw] = yv;
                            }
                            s1 += f[0];
                        }
                        const bool gam = GAM && S.gam;
                        a.z[size_t(9 * a.ms) * W_ + sw] = gam ? a.gamma : fmaxf(float(s1), a.gamma);
                        a.y[size_t(9 * a.ms) * W_ + sw] = gam ? float(-lg) : 0.f;
                    } else {
                        st |= kStPolishRej;
                        st &= ~kStPolished;
                    }
                }
                // objective and forces from the returned point (FP64: the polished
                // point, else the ADMM iterate)
                auto xval = [&](int c) -> double {
                    return polished ? (c < 3 * si.m ? W.x[c] : 0.0) : double(a.x[size_t(c) * W_ + sw]);
                };
                double r6[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) r6[k] = -bt[k];
                double ff = 0.0;
#pragma unroll 1
                for (int c = 0; c < 3 * a.ms; ++c) {
                    const double xc = xval(c);
                    if (c < 3 * si.m) {
#pragma unroll
                        for (int k = 0; k < 6; ++k) r6[k] += Gs[k * 3 * MM + c] * xc;
                    }
                    ff += xc * xc;
                    a.forces[size_t(w) * 3 * a.ms + c] = finite_in ? float(xc) : NAN;
                }
                double rr2 = 0.0;
#pragma unroll
                for (int k = 0; k < 6; ++k) rr2 += r6[k] * r6[k];
                Q = rr2 + double(a.eps) * ff;
                if (a.resid) {
#pragma unroll
                    for (int k = 0; k < 6; ++k) a.resid[size_t(k) * W_ + sw] = finite_in ? float(r6[k]) : NAN;
                }
                double rel = NAN;
                if (finite_in) {
                    const float* xs = a.x + sw;
                    const float* zs = a.z + sw;
                    const float* ys = a.y + sw;
                    rel = rel_kkt64<MM>(
                        Gs, muc, bt, si.m, double(a.eps), [&](int c) { return double(xs[size_t(c) * W_]); },
                        [&](int r) { return double(zs[size_t(r) * W_]); },
                        [&](int r) { return double(ys[size_t(r) * W_]); }, double(zs[size_t(9 * a.ms) * W_]),
                        double(ys[size_t(9 * a.ms) * W_]));
                }
                if (rel <= double(a.tol))
                    st |= kStConverged;
                else
                    st &= ~kStConverged;
                if (!finite_in) {
                    st |= kStNonfinite;
                    Q = NAN;
                }
                a.status[w] = st;
                a.kkt[w] = float(rel);
                a.qobj[w] = float(Q);
            } else if (mode == 2) {
                Q = double(a.qobj[w]);  // finished in the first pass
            }
            if (kspill >= 0) atomicOr(&P.flag[slot], 8);
        }
        P.red[lane] = Q;
        __syncthreads();
        // energies: in the first pass of grasps with nothing handed on, in
        // the second of the others
        const bool handed = act && (P.flag[slot] & 8);
        if (act && j == 0 && (mode == 0 || (mode == 1 && !handed) || (mode == 2 && handed))) {
            double E = 0.0;
            for (int l = lane; l < lane + si.s; ++l) E += P.red[l];
            a.energy[si.g] = float(E);
        }
        __syncthreads();
    }
}

// Contact-parallel polish of the handed-on QPs (see bodex_gpolish.h): a
// group of GS lanes per record, one lane per contact; all groups of the
// grid stride over the records taken by the first pass.
// Two resident waves per SIMD: with each group's factor and each lane's
// block of G kept in LDS the kernel spills 16 B per lane at that budget, and
// the handed-on QPs of the headline batch (about 1100 waves) then fit in one
// round; measured 3-4 % faster per solve at 8192 to 32,768 grasps than one
// wave per SIMD with both in registers.
#ifndef BODEX_GPOLISH_WAVES
#define BODEX_GPOLISH_WAVES 2
#endif
template <int MM, int GS>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(BODEX_GPOLISH_WAVES))) gpolish_kernel(const KArgs a) {
    constexpr int GPW = kWave / GS;
    const int lane = threadIdx.x, sub = lane % GS, grp = lane / GS;
    const int count = min(*a.spill_count, a.spill.K);
    const ShflTeam<GS> team{sub};
    // one copy of each group's 6x6 factor: the group's lanes compute the same
    // bits in lockstep, so they share it ([21][GPW], group-interleaved); each
    // lane's block of G ([18][64], lane-interleaved)
    __shared__ double sL[21 * GPW];
    __shared__ double sGb[18 * kWave];
    for (int base = int(blockIdx.x) * GPW; base < count; base += int(gridDim.x) * GPW) {
        const int k = base + grp;
        if (k < count) {
            const int w = a.spill.iv(kSpW, k), g = a.spill.iv(kSpG, k);
            const int m = a.counts[g];
            double p3[3] = {0.0, 0.0, 0.0}, n3[3] = {0.0, 0.0, 1.0}, mu = 0.5;
            if (sub < m) {
                const size_t base3 = (size_t(g) * a.ms + sub) * 3;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    p3[q] = a.points[base3 + q];
                    n3[q] = a.normals[base3 + q];
                }
                mu = a.mu[size_t(g) * a.ms + sub];
            }
            double bt[6];
#pragma unroll
            for (int r = 0; r < 6; ++r) bt[r] = double(a.beta) * double(a.wrench[size_t(w) * 6 + r]);
            GQP<MM, LdsStore> Q;
            Q.L.a.p = sL + grp;
            Q.L.a.stride = GPW;
            Q.G.p = sGb + lane;
            Q.G.stride = kWave;
            Q.sub = sub;
            gpolish_load<MM>(team, Q, a.spill, k, m, p3, n3, mu, double(a.kappa), bt, double(a.fmax),
                             double(a.eps));
#pragma unroll 1
            do {
#pragma unroll 1
                while (!gpolish_advance<MM>(team, Q, a.polish_steps)) {
                }
            } while (!gpolish_finish<MM>(team, Q));
            gpolish_store<MM>(team, Q, a.spill, k);
        }
    }
}

// ---------------------------------------------------------------------------
// Finalize kernel of the cone form: the FP64 barrier polish from the ADMM
// point, objective, energy, KKT residual, outputs and the polished state.
// ---------------------------------------------------------------------------
template <int MM>
struct ConeFinLds {
    static constexpr int NV = 3 * MM, NG = 6 * NV;
    // per slot G64 and mu (8); per lane the polish vectors f, d, ft, r
    // (lane-interleaved); the energy reduction
    static __host__ __device__ int vectors(bool) { return 4; }
    static __host__ __device__ size_t bytes(int slots, bool gam) {
        return size_t(slots) * (NG + 8) * 8 + size_t(vectors(gam)) * NV * kWave * 8 + size_t(kWave) * 8 +
               kMaxSlots * 32 + 64;
    }
};

// Polish schedule: start 1e-3 of the way toward the cone axis, barrier weight
// at most 1e5 rising 60x per centring, intermediate centring to a Newton
// decrement of 1e-2 (the last one to 1e-10), stop at nu / t <= 1e-12.
// Swept on the headline batch from ADMM points at 1e-4: looser schedules are
// up to 15 % faster (10.6-11.7 ms against 12.5 ms for growth 25-40 and
// decrements 0.05-0.3; a decrement of 1 leaves QPs unconverged) but end
// less accurate in the weakly determined force directions (largest force
// error in the cone parity tests 5.8e-5 to 1.0e-4 against 1.3e-5, the bar
// being 1e-4), so the tight schedule stays.  (The macros exist for such
// sweeps at build time.)
#ifndef BODEX_CONE_PULL
#define BODEX_CONE_PULL 1e-3
#endif
#ifndef BODEX_CONE_T0
#define BODEX_CONE_T0 1e5
#endif
#ifndef BODEX_CONE_GROWTH
#define BODEX_CONE_GROWTH 60.0
#endif
#ifndef BODEX_CONE_LOOSE
#define BODEX_CONE_LOOSE 1e-2
#endif
constexpr double kConePull = BODEX_CONE_PULL, kConeT0 = BODEX_CONE_T0, kConeGap = 1e-12,
                 kConeGrowth = BODEX_CONE_GROWTH, kConeLoose = BODEX_CONE_LOOSE;
constexpr double kConeRetryPull = 0.5;

// One wave per SIMD: the polish factors its 3 MM x 3 MM Newton matrix in
// registers.
template <int MM, bool GAM>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1))) cone_finalize_kernel(const KArgs a) {
    constexpr int NV = 3 * MM, NG = 6 * NV;
    extern __shared__ __align__(16) unsigned char smem[];
    const int S = a.slots;
    double* d = reinterpret_cast<double*>(smem);
    FinPtrs<MM> P;
    P.G = d;
    d += size_t(S) * NG;
    P.muc = d;
    d += size_t(S) * 8;
    double* work = d;
    d += size_t(ConeFinLds<MM>::vectors(GAM)) * NV * kWave;
    P.red = d;
    d += kWave;
    P.Gbar = nullptr;
    P.work = work;
    P.info = reinterpret_cast<SlotInfo*>(d);
    P.flag = reinterpret_cast<int*>(P.info + kMaxSlots);
    const int lane = threadIdx.x;
    const ConeWork<LaneVec> W(LaneVec{work + lane, kWave}, LaneVec{work + NV * kWave + lane, kWave},
                              LaneVec{work + 2 * NV * kWave + lane, kWave}, LaneVec{work + 3 * NV * kWave + lane, kWave});
    __shared__ int sTile;
    for (int t = fetch_tile(a, &sTile, -1); t < a.n_tiles; t = fetch_tile(a, &sTile, t)) {
        int nsl;
        load_slots(a, t, P.info, nsl);
        int slot, j;
        lane_slot(P.info, nsl, lane, slot, j);
        const bool act = slot >= 0;
        SlotInfo si = {0, 0, 1, 0};
        if (act) si = P.info[slot];
        const bool good = fin_setup<MM>(a, P, nsl, slot, j, si, true);
        const int w = si.w0 + j;
        double Q = 0.0;
        if (act) {
            const double* Gs = P.G + size_t(slot) * NG;
            const size_t W_ = size_t(a.sW);  // state stride
            const size_t sw = state_col(a, si, j);
            ConeData<MM, const double*, GAM> D;
            D.G = Gs;
            D.mu = P.muc + slot * 8;
            for (int r = 0; r < 6; ++r) D.bt[r] = double(a.beta) * double(a.wrench[size_t(w) * 6 + r]);
            D.m = si.m;
            D.fmax = a.fmax;
            D.gamma = a.gamma;
            D.eps = a.eps;
            unsigned char st = a.status[w];
            bool polished = false;
            const bool finite_in = good && !(st & kStNonfinite);
            if (finite_in && a.polish) {
                const float* zs = a.z + sw;
                // a failed polish is taken once more from a point well inside
                // (half way to the cone axis), whose central path the barrier
                // follows from a small weight
                ConePolishOut po;
                int n1 = 0, e1 = 0, g1 = 0;
#pragma unroll 1
                for (int attempt = 0; attempt < 2; ++attempt) {
                    cone_start<MM>(D, [&](int r) { return double(zs[size_t(r) * W_]); },
                                   attempt ? kConeRetryPull : kConePull, W);
                    po = cone_polish<MM>(D, kConeT0, kConeGap, kConeGrowth, kConeLoose, a.polish_steps, W);
                    po.newton += n1;
                    po.evals += e1;
                    po.grads += g1;
                    if (po.status == 0) break;
                    n1 = po.newton;
                    e1 = po.evals;
                    g1 = po.grads;
                }
                if (a.pflops) a.pflops[w] = float(cone_polish_flops(si.m, po));
                if (po.status == 0) {
                    polished = true;
                    st |= kStPolished;
                    st &= ~kStPolishRej;
                    // ADMM-form state of the polished (interior) point: z = x,
                    // y from stationarity with the barrier's normal-sum
                    // multiplier
                    double r6[6], s1 = 0.0;
                    cone_g_times<MM>(D, W.f, true, r6);
#pragma unroll 1
                    for (int i = 0; i < si.m; ++i) s1 += W.f[3 * i];
                    const bool gam = GAM && a.gamma > 0.f;
                    const double yg = gam ? -1.0 / (po.t * (s1 - D.gamma)) : 0.0;
#pragma unroll 1
                    for (int i = 0; i < a.ms; ++i) {
                        const bool live = i < si.m;
                        double g[3] = {0.0, 0.0, 0.0};
                        if (live) cone_contact_grad<MM>(D, i, r6, W.f, g);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const double fv = live ? W.f[3 * i + c] : 0.0;
                            a.x[size_t(3 * i + c) * W_ + sw] = float(fv);
                            a.z[size_t(3 * i + c) * W_ + sw] = float(fv);
                            a.y[size_t(3 * i + c) * W_ + sw] = live ? float(-g[c] - (c == 0 ? yg : 0.0)) : 0.f;
                        }
                    }
                    a.z[size_t(3 * a.ms) * W_ + sw] = fmaxf(float(s1), a.gamma);
                    a.y[size_t(3 * a.ms) * W_ + sw] = float(yg);
                } else {
                    st |= kStPolishRej;
                    st &= ~kStPolished;
                }
            }
            auto xval = [&](int c) -> double {
                return polished ? (c < 3 * si.m ? W.f[c] : 0.0) : double(a.x[size_t(c) * W_ + sw]);
            };
            double r6[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) r6[k] = -D.bt[k];
            double ff = 0.0;
#pragma unroll 1
            for (int c = 0; c < 3 * a.ms; ++c) {
                const double xc = xval(c);
                if (c < 3 * si.m) {
#pragma unroll
                    for (int k = 0; k < 6; ++k) r6[k] += Gs[k * NV + c] * xc;
                }
                ff += xc * xc;
                a.forces[size_t(w) * 3 * a.ms + c] = finite_in ? float(xc) : NAN;
            }
            double rr2 = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) rr2 += r6[k] * r6[k];
            Q = rr2 + double(a.eps) * ff;
            if (a.resid) {
#pragma unroll
                for (int k = 0; k < 6; ++k) a.resid[size_t(k) * W_ + sw] = finite_in ? float(r6[k]) : NAN;
            }
            double rel = NAN;
            if (finite_in) {
                const float* xs = a.x + sw;
                const float* zs = a.z + sw;
                const float* ys = a.y + sw;
                rel = cone_rel_kkt64<MM>(
                    Gs, D.bt, si.m, double(a.eps), [&](int c) { return double(xs[size_t(c) * W_]); },
                    [&](int r) { return double(zs[size_t(r) * W_]); }, [&](int r) { return double(ys[size_t(r) * W_]); },
                    double(zs[size_t(3 * a.ms) * W_]), double(ys[size_t(3 * a.ms) * W_]));
            }
            if (rel <= double(a.tol))
                st |= kStConverged;
            else
                st &= ~kStConverged;
            if (!finite_in) {
                st |= kStNonfinite;
                Q = NAN;
            }
            a.status[w] = st;
            a.kkt[w] = float(rel);
            a.qobj[w] = float(Q);
        }
        P.red[lane] = Q;
        __syncthreads();
        if (act && j == 0) {
            double E = 0.0;
            for (int l = lane; l < lane + si.s; ++l) E += P.red[l];
            a.energy[si.g] = float(E);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Backward kernel.
// ---------------------------------------------------------------------------
// f* is the point the solve left in state.x (FP32 rounding of its FP64
// polish).  With the state's residual (state.r, G f* - beta t formed in FP64
// by the solve) the gradient uses it directly; without it the pyramid form
// re-runs its polish from the state's duals to recover f* in FP64, and the
// cone form forms the residual from the FP32 forces.
template <int MM, bool GAM, bool CONE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) backward_kernel(const KArgs a) {
    constexpr int NV = 3 * MM, NG = 6 * NV;
    extern __shared__ __align__(16) unsigned char smem[];
    const FinPtrs<MM> P = fin_carve<MM>(smem, a.slots, true);
    const int lane = threadIdx.x;
    const PolishWork<LaneVec> W = polish_work<MM>(P, lane);
    __shared__ int sTile;
    for (int t = fetch_tile(a, &sTile, -1); t < a.n_tiles; t = fetch_tile(a, &sTile, t)) {
        int nsl;
        load_slots(a, t, P.info, nsl);
        int slot, j;
        lane_slot(P.info, nsl, lane, slot, j);
        const bool act = slot >= 0;
        SlotInfo si = {0, 0, 1, 0};
        if (act) si = P.info[slot];
        const bool good = fin_setup<MM>(a, P, nsl, slot, j, si);
        const int w = si.w0 + j;
        double f[NV], tw[6], om = 0.0;
#pragma unroll
        for (int c = 0; c < NV; ++c) f[c] = 0.0;
#pragma unroll
        for (int r = 0; r < 6; ++r) tw[r] = 0.0;
        if (act && good) {
#pragma unroll
            for (int r = 0; r < 6; ++r) tw[r] = a.wrench[size_t(w) * 6 + r];
#pragma unroll
            for (int c = 0; c < NV; ++c) f[c] = (c < 3 * a.ms) ? a.x[size_t(c) * a.sW + state_col(a, si, j)] : 0.0;
            double bt[6];
#pragma unroll
            for (int r = 0; r < 6; ++r) bt[r] = double(a.beta) * tw[r];
            if (!CONE && !a.resid) {
                const LdsPolishData<MM, GAM> D = polish_data<MM, GAM>(a, P, slot, si, bt);
                PolishState<MM> PS;
                PS.S.pc = projector_cache<MM>(P, lane);
                const StridedY<MM> y0{a.y + state_col(a, si, j), size_t(a.sW), a.ms};
                const PolishOut po = polish_qp<MM>(D, y0, a.polish_steps, W, PS);
                if (po.status == 0) {
#pragma unroll
                    for (int c = 0; c < NV; ++c) f[c] = (c < 3 * si.m) ? W.x[c] : 0.0;
                }
            }
            if (a.dLdQ) om += a.dLdQ[w];
            if (a.dLdE) om += a.dLdE[si.g];
        }
        __syncthreads();  // the polish space becomes the reduction buffer
        double* rw = P.red + size_t(lane) * (6 + NV);  // 2 * omega * r (6), f (NV)
        if (act && good) {
            const double* Gs = P.G + size_t(slot) * NG;
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                double v = -double(a.beta) * tw[r];
#pragma unroll
                for (int c = 0; c < NV; ++c) v += Gs[r * NV + c] * f[c];
                // the stored residual carries the digits that G f - beta t
                // loses to cancellation when formed from FP32 forces
                if (a.resid) v = a.resid[size_t(r) * a.sW + state_col(a, si, j)];
                rw[r] = 2.0 * om * v;
            }
#pragma unroll
            for (int c = 0; c < NV; ++c) rw[6 + c] = f[c];
        } else {
#pragma unroll
            for (int e = 0; e < 6 + NV; ++e) rw[e] = 0.0;
        }
        __syncthreads();
        // Gbar = sum over the grasp's wrenches of 2 omega r f^T
        if (act) {
            double* Gb = P.Gbar + size_t(slot) * NG;
            const int l0 = lane - j;
            for (int e = j; e < NG; e += si.s) {
                const int r = e / NV, c = e % NV;
                double acc = 0.0;
                for (int l = l0; l < l0 + si.s; ++l) {
                    const double* o = P.red + size_t(l) * (6 + NV);
                    acc += o[r] * o[6 + c];
                }
                Gb[e] = acc;
            }
        }
        __syncthreads();
        if (act) {
            const double* Gb = P.Gbar + size_t(slot) * NG;
            const double kap = a.kappa;
            for (int c = j; c < a.ms; c += si.s) {
                double dp[3] = {0, 0, 0}, dn[3] = {0, 0, 0};
                const size_t base = (size_t(si.g) * a.ms + c) * 3;
                if (c < si.m && good) {
                    const double p[3] = {a.points[base], a.points[base + 1], a.points[base + 2]};
                    const double n[3] = {a.normals[base], a.normals[base + 1], a.normals[base + 2]};
                    double nh[3], d[3], e[3];
                    contact_frame<double>(n[0], n[1], n[2], nh, d, e);
                    const double* vec[3] = {nh, d, e};
                    double dv[3][3];
                    for (int col = 0; col < 3; ++col) {
                        double gf[3], gt[3], cx[3];
                        for (int r = 0; r < 3; ++r) {
                            gf[r] = Gb[r * NV + 3 * c + col];
                            gt[r] = Gb[(3 + r) * NV + 3 * c + col];
                        }
                        // d/dp of gt . (p x v) is v x gt
                        cross3(vec[col], gt, cx);
                        for (int r = 0; r < 3; ++r) dp[r] += kap * cx[r];
                        // d/dv of gf . v + gt . (p x v) is gf + gt x p
                        cross3(gt, p, cx);
                        for (int r = 0; r < 3; ++r) dv[col][r] = gf[r] + kap * cx[r];
                    }
                    // derivatives of the basis formula in nhat (sign fixed off z = 0)
                    const double x = nh[0], yy = nh[1], zz = nh[2];
                    const double sg = copysign(1.0, zz);
                    const double aa = -1.0 / (sg + zz), a2 = aa * aa;
                    const double Jd[3][3] = {{2 * sg * x * aa, 0.0, sg * x * x * a2},
                                             {sg * yy * aa, sg * x * aa, sg * x * yy * a2},
                                             {-sg, 0.0, 0.0}};
                    const double Je[3][3] = {{yy * aa, x * aa, x * yy * a2},
                                             {0.0, 2 * yy * aa, yy * yy * a2},
                                             {0.0, -1.0, 0.0}};
                    double dnh[3];
                    for (int kx = 0; kx < 3; ++kx) {
                        dnh[kx] = dv[0][kx];
                        for (int r = 0; r < 3; ++r) dnh[kx] += Jd[r][kx] * dv[1][r] + Je[r][kx] * dv[2][r];
                    }
                    const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
                    const double pr = dnh[0] * nh[0] + dnh[1] * nh[1] + dnh[2] * nh[2];
                    for (int kx = 0; kx < 3; ++kx) dn[kx] = (dnh[kx] - pr * nh[kx]) / len;
                } else if (c < si.m) {
                    dp[0] = dp[1] = dp[2] = NAN;
                    dn[0] = dn[1] = dn[2] = NAN;
                }
                for (int r = 0; r < 3; ++r) {
                    if (a.accumulate) {
                        a.dP[base + r] += float(dp[r]);
                        a.dN[base + r] += float(dn[r]);
                    } else {
                        a.dP[base + r] = float(dp[r]);
                        a.dN[base + r] = float(dn[r]);
                    }
                }
            }
        }
        __syncthreads();
    }
}


}  // namespace bodex
