// bodex_math.h -- per-lane arithmetic of the batched contact-force QP.
//
// Everything here is straight-line code on small fixed-size arrays, written as
// __host__ __device__ templates over the maximum contact count MM so that the
// loops unroll and every array index is a compile-time constant (the arrays
// then live in VGPRs).  Matrices shared by the lanes of one grasp (G, the
// inverse KKT matrix, P^{-1}) are passed as pointers: LDS on the GPU.
//
// Problem (BODex Sec. IV-A, Eq. 7-9, with the 8-facet pyramid): for one grasp
// with m <= MM contacts and one desired wrench direction t,
//     min_f ||G f - beta t||^2 + eps ||f||^2
//     s.t. per contact i: facets  cos(phi_k) f_i2 + sin(phi_k) f_i3
//                                 - mu_i cos(pi/8) f_i1 <= 0,  k = 0..7,
//                                 phi_k = (2k+1) pi/8
//          0 <= f_i1 <= fmax,  sum_i f_i1 >= gamma.
// ADMM form: P = 2(G^T G + eps I), q = -2 beta G^T t, r = 9 MM + 1 rows
// l <= A f <= u: rows 9i..9i+7 the facets (l = -inf, u = 0), row 9i+8 the
// normal bound [0, fmax], row 9 MM the normal-sum row [gamma, +inf).  Rows of
// padded contacts (i >= m) are inert and stay zero.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define BODEX_HD __host__ __device__
#else
#define BODEX_HD
#endif
#define BODEX_FI BODEX_HD inline __attribute__((always_inline))

// Compiler-only ordering point: keeps the scheduler from issuing every load of
// a long unrolled sequence at once (which would hold them all in registers).
#if defined(__HIP_DEVICE_COMPILE__)
#define BODEX_SPLIT() asm volatile("" ::: "memory")
#else
#define BODEX_SPLIT() ((void)0)
#endif

namespace bodex {

// cos(pi/8), sin(pi/8)
constexpr double kC8 = 0.92387953251128673848;
constexpr double kS8 = 0.38268343236508978178;

// Lane-interleaved array in memory: element i at p[i * stride].
template <typename T>
struct Strided {
    T* p;
    int stride;
    BODEX_FI T& operator[](int i) const { return p[i * stride]; }
};

template <int MM>
struct Dims {
    static constexpr int NV = 3 * MM;             // variables
    static constexpr int NR = 9 * MM + 1;         // ADMM-form rows
    static constexpr int NK = NV * (NV + 1) / 2;  // packed symmetric matrix
    static constexpr int NKP = (NK + 3) & ~3;     // padded to 16 bytes
    static constexpr int NG = 6 * NV;             // grasp matrix entries
};

// Packed upper triangle, row-major (i <= j).
template <int N>
BODEX_FI constexpr int up_idx(int i, int j) {
    return i * N - (i * (i - 1)) / 2 + (j - i);
}
// Packed lower triangle, row-major (j <= i).
BODEX_FI constexpr int lo_idx(int i, int j) { return (i * (i + 1)) / 2 + j; }

// Tangent direction of facet k (phi_k = (2k+1) pi/8).
template <typename T>
BODEX_FI T facet_cos(int k) {
    const T c = T(kC8), s = T(kS8);
    switch (k & 7) {
        case 0: return c;
        case 1: return s;
        case 2: return -s;
        case 3: return -c;
        case 4: return -c;
        case 5: return -s;
        case 6: return s;
        default: return c;
    }
}
template <typename T>
BODEX_FI T facet_sin(int k) {
    const T c = T(kC8), s = T(kS8);
    switch (k & 7) {
        case 0: return s;
        case 1: return c;
        case 2: return c;
        case 3: return s;
        case 4: return -s;
        case 5: return -c;
        case 6: return -c;
        default: return -s;
    }
}

// ---------------------------------------------------------------------------
// Contact frame and grasp matrix (Sec. III, Eq. 2).
// ---------------------------------------------------------------------------

// Unit normal and tangents (d, e) with nhat = d x e: the branchless
// orthonormal basis of Duff et al. (JCGT 2017); the branch sign is the sign
// bit of the normal's z component.
template <typename T>
BODEX_FI void contact_frame(T nx, T ny, T nz, T nh[3], T d[3], T e[3]) {
    const T len = sqrt(nx * nx + ny * ny + nz * nz);
    const T x = nx / len, y = ny / len, z = nz / len;
    const T s = copysign(T(1), z);
    const T a = T(-1) / (s + z);
    const T b = x * y * a;
    nh[0] = x;
    nh[1] = y;
    nh[2] = z;
    d[0] = T(1) + s * x * x * a;
    d[1] = s * b;
    d[2] = -s * x;
    e[0] = b;
    e[1] = s + y * y * a;
    e[2] = -y;
}

// Columns 3i..3i+2 of G (row-major [6][NV]) for contact i: the columns are
// (c, kappa * p x c) for c in (nhat, d, e).  Returns false for a degenerate
// input (non-finite values or a zero normal).
template <typename T, int NV>
BODEX_FI bool grasp_columns(const T p[3], const T n[3], T kappa, int i, T* G) {
    T nh[3], d[3], e[3];
    contact_frame<T>(n[0], n[1], n[2], nh, d, e);
    const T* col[3] = {nh, d, e};
    bool ok = true;
    for (int c = 0; c < 3; ++c) {
        const T* v = col[c];
        T tq0 = p[1] * v[2] - p[2] * v[1];
        T tq1 = p[2] * v[0] - p[0] * v[2];
        T tq2 = p[0] * v[1] - p[1] * v[0];
        G[0 * NV + 3 * i + c] = v[0];
        G[1 * NV + 3 * i + c] = v[1];
        G[2 * NV + 3 * i + c] = v[2];
        G[3 * NV + 3 * i + c] = kappa * tq0;
        G[4 * NV + 3 * i + c] = kappa * tq1;
        G[5 * NV + 3 * i + c] = kappa * tq2;
        ok = ok && isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]) &&
             isfinite(tq0) && isfinite(tq1) && isfinite(tq2);
    }
    return ok;
}

// Entry (i, j) of K = P + rho A^T A = 2(G^T G + eps I) + rho A^T A in closed
// form: A^T A has diag(8 mu_i^2 cos^2(pi/8) + 1 + 1, 4, 4) per contact (the
// facet Gram matrix, the bound row and the normal-sum row) and 1 between the
// normal components of different contacts (normal-sum row).  Variables of
// padded contacts get an identity block so that they stay decoupled at zero.
template <typename T, int NV>
BODEX_FI T kkt_entry(const T* G, const T* muc, int m, T rho, T eps, int i, int j) {
    const int ci = i / 3, cj = j / 3;
    if (ci >= m || cj >= m) return (i == j) ? T(1) : T(0);
    T s = T(0);
    for (int a = 0; a < 6; ++a) s += G[a * NV + i] * G[a * NV + j];
    T v = T(2) * s;
    if (i == j) v += T(2) * eps;
    const int ri = i % 3, rj = j % 3;
    if (ri == 0 && rj == 0) {
        if (ci == cj)
            v += rho * (T(8) * muc[ci] * muc[ci] + T(2));
        else
            v += rho;
    } else if (i == j) {
        v += rho * T(4);
    }
    return v;
}

// Entry (i, j) of P = 2(G^T G + eps I); padded variables get 2 eps.
template <typename T, int NV>
BODEX_FI T hess_entry(const T* G, T eps, int i, int j) {
    T s = T(0);
    for (int a = 0; a < 6; ++a) s += G[a * NV + i] * G[a * NV + j];
    return T(2) * s + ((i == j) ? T(2) * eps : T(0));
}

// Upper bound on cond(K) that can be evaluated before factoring:
// lambda_max <= 2||G||_F^2 + 2 eps + rho (max_i(8 mu_i^2 c^2 + 2) + m),
// lambda_min >= 2 eps + rho min_i min(8 mu_i^2 c^2 + 1, 4).
template <typename T, int NV>
BODEX_FI T kkt_cond_bound(const T* G, const T* muc, int m, T rho, T eps) {
    T gf = T(0);
    for (int a = 0; a < 6 * NV; ++a) gf += G[a] * G[a];
    T amax = T(0), amin = T(4);
#pragma unroll
    for (int i = 0; i < NV / 3; ++i) {
        if (i < m) {
            T v = T(8) * muc[i] * muc[i] + T(1);
            amax = v + T(1) > amax ? v + T(1) : amax;
            amin = v < amin ? v : amin;
        }
    }
    T hi = T(2) * gf + T(2) * eps + rho * (amax + T(m));
    T lo = T(2) * eps + rho * amin;
    return hi / lo;
}

// ---------------------------------------------------------------------------
// ADMM iteration in the reduced state w (FP32, one lane per QP).
//
// With sigma = 0 the OSQP-form iteration depends on (z, y) only through
// w = z + y/rho: z = Pi(w) (projection on [l, u]) and y = rho (w - Pi(w)).
// One iteration is
//     v  = 2 Pi(w) - w                       (= (rho z - y)/rho)
//     x~ = K^{-1} (rho A^T v - q)            (K = P + rho A^T A)
//     w <- w + alpha (A x~ - Pi(w))
// i.e. an affine map followed by the clamp of the next iteration.
// ---------------------------------------------------------------------------

// Padding contacts (i >= m) need no branches: their state rows are zero,
// their G columns are zero and their block of K^{-1} is the identity, so every
// row update leaves them at zero.  Only the normal-sum row couples contacts,
// and it is masked to the real ones.
template <int MM, typename BQ, typename MU>
BODEX_FI void admm_rhs(const float* w, BQ bq, MU muc,
                       float rho, float fmax, float gamma, int m, float* rhs) {
    const float wg = w[9 * MM];
    const float vg = 2.f * fmaxf(wg, gamma) - wg;
#pragma unroll
    for (int i = 0; i < MM; ++i) {
        // facet rows: 2 min(w, 0) - w = -|w|
        float v[8], sum = 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v[k] = -fabsf(w[9 * i + k]);
            sum += v[k];
        }
        const float wb = w[9 * i + 8];
        const float vb = 2.f * fminf(fmaxf(wb, 0.f), fmax) - wb;
        const float d0 = v[0] - v[4], d1 = v[1] - v[5];
        const float d2 = v[2] - v[6], d3 = v[3] - v[7];
        const float a1 = fmaf(-muc[i], sum, vb + ((i < m) ? vg : 0.f));
        const float a2 = fmaf(float(kC8), d0 - d3, float(kS8) * (d1 - d2));
        const float a3 = fmaf(float(kS8), d0 + d3, float(kC8) * (d1 + d2));
        rhs[3 * i + 0] = fmaf(rho, a1, bq[3 * i + 0]);
        rhs[3 * i + 1] = fmaf(rho, a2, bq[3 * i + 1]);
        rhs[3 * i + 2] = fmaf(rho, a3, bq[3 * i + 2]);
    }
}

// x = K r with K symmetric, packed upper triangle (each off-diagonal entry is
// read once and used twice).  The split every three rows bounds the loads of
// K that are in flight (and held in registers) at any point.
template <int N, typename KPtr>
BODEX_FI void symv_packed(KPtr K, const float* r, float* x) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = K[up_idx<N>(i, i)] * r[i];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (i % 3 == 2) BODEX_SPLIT();
#pragma unroll
        for (int j = i + 1; j < N; ++j) {
            const float k = K[up_idx<N>(i, j)];
            x[i] = fmaf(k, r[j], x[i]);
            x[j] = fmaf(k, r[i], x[j]);
        }
    }
}

// w <- w + alpha (A x - Pi(w)).
template <int MM, typename MU>
BODEX_FI void admm_update(float* w, const float* x, MU muc, float alpha,
                          float fmax, float gamma, int m) {
    float s1 = 0.f;
#pragma unroll
    for (int i = 0; i < MM; ++i) {
        const float x1 = x[3 * i], x2 = x[3 * i + 1], x3 = x[3 * i + 2];
        const float t[4] = {fmaf(float(kC8), x2, float(kS8) * x3),
                            fmaf(float(kS8), x2, float(kC8) * x3),
                            fmaf(-float(kS8), x2, float(kC8) * x3),
                            fmaf(-float(kC8), x2, float(kS8) * x3)};
        const float am = muc[i] * x1;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float wk = w[9 * i + k];
            w[9 * i + k] = fmaf(alpha, (t[k] - am) - fminf(wk, 0.f), wk);
            const float wl = w[9 * i + 4 + k];
            w[9 * i + 4 + k] = fmaf(alpha, (-t[k] - am) - fminf(wl, 0.f), wl);
        }
        const float wb = w[9 * i + 8];
        w[9 * i + 8] = fmaf(alpha, x1 - fminf(fmaxf(wb, 0.f), fmax), wb);
        s1 += (i < m) ? x1 : 0.f;
    }
    const float wg = w[9 * MM];
    w[9 * MM] = fmaf(alpha, s1 - fmaxf(wg, gamma), wg);
}

// Projection of one ADMM-form row.
BODEX_FI float row_proj(int r, int MMr, float w, float fmax, float gamma) {
    if (r == 9 * MMr) return fmaxf(w, gamma);
    if (r % 9 == 8) return fminf(fmaxf(w, 0.f), fmax);
    return fminf(w, 0.f);
}

struct Residual {
    float rel;   // relative KKT residual (OSQP form, eps_abs = eps_rel)
    float rp_n;  // primal residual / primal scale
    float rd_n;  // dual residual / dual scale
};

// Residuals of the triple (x, z = Pi(w), y = rho (w - Pi(w))):
//   r_p = ||A x - z||, r_d = ||P x + q + A^T y||   (infinity norms),
//   rel = max(r_p / (1 + max(||Ax||, ||z||)),
//             r_d / (1 + max(||Px||, ||A^T y||, ||q||))).
// P x is formed from G directly: 2 (G^T (G x) + eps x).
template <int MM, typename BQ, typename MU, typename GPtr>
BODEX_FI Residual admm_residual(const float* w, const float* x, BQ bq,
                                MU muc, GPtr G, float rho, float eps,
                                float fmax, float gamma, int m) {
    constexpr int NV = 3 * MM;
    float rp = 0.f, nAx = 0.f, nz = 0.f;
    float aty[NV];
    float s1 = 0.f;
    const float wg = w[9 * MM];
    const float zg = fmaxf(wg, gamma);
    const float yg = rho * (wg - zg);
#pragma unroll
    for (int i = 0; i < MM; ++i) {
        float a1 = 0.f, a2 = 0.f, a3 = 0.f;
        const float x1 = x[3 * i], x2 = x[3 * i + 1], x3 = x[3 * i + 2];
        const float am = muc[i] * x1;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float ck = facet_cos<float>(k), sk = facet_sin<float>(k);
            const float zt = fmaf(ck, x2, fmaf(sk, x3, -am));
            const float wk = w[9 * i + k];
            const float zk = fminf(wk, 0.f);
            const float yk = rho * (wk - zk);
            rp = fmaxf(rp, fabsf(zt - zk));
            nAx = fmaxf(nAx, fabsf(zt));
            nz = fmaxf(nz, fabsf(zk));
            a1 = fmaf(-muc[i], yk, a1);
            a2 = fmaf(ck, yk, a2);
            a3 = fmaf(sk, yk, a3);
        }
        const float wb = w[9 * i + 8];
        const float zb = fminf(fmaxf(wb, 0.f), fmax);
        a1 += rho * (wb - zb) + ((i < m) ? yg : 0.f);
        rp = fmaxf(rp, fabsf(x1 - zb));
        nAx = fmaxf(nAx, fabsf(x1));
        nz = fmaxf(nz, fabsf(zb));
        s1 += (i < m) ? x1 : 0.f;
        aty[3 * i] = a1;
        aty[3 * i + 1] = a2;
        aty[3 * i + 2] = a3;
    }
    rp = fmaxf(rp, fabsf(s1 - zg));
    nAx = fmaxf(nAx, fabsf(s1));
    nz = fmaxf(nz, fabsf(zg));
    float gx[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < NV; ++c) s = fmaf(G[a * NV + c], x[c], s);
        gx[a] = s;
        BODEX_SPLIT();
    }
    float rd = 0.f, nPx = 0.f, nAty = 0.f, nq = 0.f;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        if (c % 3 == 0) BODEX_SPLIT();
        float s = eps * x[c];
#pragma unroll
        for (int a = 0; a < 6; ++a) s = fmaf(G[a * NV + c], gx[a], s);
        const float px = 2.f * s;
        rd = fmaxf(rd, fabsf(px - bq[c] + aty[c]));
        nPx = fmaxf(nPx, fabsf(px));
        nAty = fmaxf(nAty, fabsf(aty[c]));
        nq = fmaxf(nq, fabsf(bq[c]));
    }
    const float ps = fmaxf(nAx, nz), ds = fmaxf(fmaxf(nPx, nAty), nq);
    Residual R;
    R.rel = fmaxf(rp / (1.f + ps), rd / (1.f + ds));
    R.rp_n = rp / fmaxf(ps, 1e-30f);
    R.rd_n = rd / fmaxf(ds, 1e-30f);
    return R;
}

// ---------------------------------------------------------------------------
// FP64 polish: dual active-set (Goldfarb-Idnani) correction warm-started from
// the active set that ADMM identified.
//
// One-sided rows C f <= b with the ADMM-form row ids: 9i+k facet k of contact
// i (b = 0), 9i+8 the upper normal bound f_i1 <= fmax, 9 MM the normal-sum
// row -sum f_i1 <= -gamma (used only when gamma > 0).  The lower normal bound
// f_i1 >= 0 is implied by the facets and is not a separate row.
// ---------------------------------------------------------------------------

struct RowMask {
    uint64_t lo, hi;
    BODEX_FI void clear() { lo = hi = 0; }
    BODEX_FI bool has(int r) const { return r < 64 ? ((lo >> r) & 1) : ((hi >> (r - 64)) & 1); }
    BODEX_FI void set(int r) {
        if (r < 64) lo |= (uint64_t(1) << r); else hi |= (uint64_t(1) << (r - 64));
    }
    BODEX_FI void unset(int r) {
        if (r < 64) lo &= ~(uint64_t(1) << r); else hi &= ~(uint64_t(1) << (r - 64));
    }
};

// Coefficients of a per-contact row on its contact's 3 variables.
BODEX_FI void row3(int r, double muc, double fm, double c[3], double* b) {
    const int k = r % 9;
    if (k == 8) {
        c[0] = 1.0; c[1] = 0.0; c[2] = 0.0;
        *b = fm;
    } else {
        c[0] = -muc;
        c[1] = facet_cos<double>(k);
        c[2] = facet_sin<double>(k);
        *b = 0.0;
    }
}

// Accessors into a packed symmetric matrix stored in memory that the caller
// chooses (LDS on the GPU).
template <int N, typename P>
BODEX_FI double sym_at(P A, int i, int j) {
    return i <= j ? A[up_idx<N>(i, j)] : A[up_idx<N>(j, i)];
}

template <int MM>
struct PolishCtx {
    static constexpr int NV = 3 * MM;
    static constexpr int GR = 9 * MM;  // id of the normal-sum row
    int m;
    double fmax, gamma, eps, beta;
    const double* muc;  // [MM] mu_i cos(pi/8)
};

// out = P^{-1} c_r (dense NV-vector).
template <int MM, typename PP>
BODEX_FI void pinv_row(const PolishCtx<MM>& X, PP Pinv, int r, double* out) {
    constexpr int NV = 3 * MM;
    if (r == PolishCtx<MM>::GR) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s = 0.0;
            for (int i = 0; i < X.m; ++i) s -= sym_at<NV>(Pinv, v, 3 * i);
            out[v] = s;
        }
        return;
    }
    double c[3], b;
    const int i = r / 9;
    row3(r, X.muc[i], X.fmax, c, &b);
#pragma unroll
    for (int v = 0; v < NV; ++v)
        out[v] = c[0] * sym_at<NV>(Pinv, v, 3 * i) + c[1] * sym_at<NV>(Pinv, v, 3 * i + 1) +
                 c[2] * sym_at<NV>(Pinv, v, 3 * i + 2);
}

// C_r . v and the row's right-hand side.
template <int MM>
BODEX_FI double row_dot(const PolishCtx<MM>& X, int r, const double* v, double* b) {
    if (r == PolishCtx<MM>::GR) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < MM; ++i)
            if (i < X.m) s -= v[3 * i];
        *b = -X.gamma;
        return s;
    }
    double c[3];
    const int i = r / 9;
    row3(r, X.muc[i], X.fmax, c, b);
    double s = 0.0;
#pragma unroll
    for (int ii = 0; ii < MM; ++ii)
        if (ii == i) s = c[0] * v[3 * ii] + c[1] * v[3 * ii + 1] + c[2] * v[3 * ii + 2];
    return s;
}

// v += a * C_r^T.
template <int MM>
BODEX_FI void row_axpy(const PolishCtx<MM>& X, int r, double a, double* v) {
    if (r == PolishCtx<MM>::GR) {
#pragma unroll
        for (int i = 0; i < MM; ++i)
            if (i < X.m) v[3 * i] -= a;
        return;
    }
    double c[3], b;
    const int i = r / 9;
    row3(r, X.muc[i], X.fmax, c, &b);
#pragma unroll
    for (int ii = 0; ii < MM; ++ii)
        if (ii == i) {
            v[3 * ii] += a * c[0];
            v[3 * ii + 1] += a * c[1];
            v[3 * ii + 2] += a * c[2];
        }
}

// C_r P^{-1} C_s^T.
template <int MM, typename PP>
BODEX_HD inline double row_pinv_row(const PolishCtx<MM>& X, PP Pinv, int r, int s) {
    constexpr int NV = 3 * MM;
    constexpr int GR = PolishCtx<MM>::GR;
    if (r == GR || s == GR) {
        double t[NV];
        pinv_row<MM>(X, Pinv, r == GR ? s : r, t);
        double b;
        return row_dot<MM>(X, r == GR ? r : s, t, &b);
    }
    double cr[3], cs[3], b;
    const int i = r / 9, j = s / 9;
    row3(r, X.muc[i], X.fmax, cr, &b);
    row3(s, X.muc[j], X.fmax, cs, &b);
    double acc = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) acc += cr[a] * cs[c] * sym_at<NV>(Pinv, 3 * i + a, 3 * j + c);
    return acc;
}

// Dense helpers on NV-vectors.
template <int NV, typename PP>
BODEX_FI void symv64(PP A, const double* x, double* y) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NV; ++j) s += sym_at<NV>(A, i, j) * x[j];
        y[i] = s;
    }
}

// act[j] for a run-time j, without dynamic indexing of the register array.
template <int NV>
BODEX_FI int act_at(const int* act, int j) {
    int v = act[0];
#pragma unroll
    for (int i = 1; i < NV; ++i) v = (j == i) ? act[i] : v;
    return v;
}

// Cholesky of the k x k matrix M_jl = C_{act_j} P^{-1} C_{act_l}^T into
// packed-lower storage L (accessed through L[idx * stride]).  Returns false if
// a pivot is not positive.
template <int MM, typename PP, typename LP>
BODEX_FI bool factor_active(const PolishCtx<MM>& X, PP Pinv, const int* act, int k, LP L,
                            int stride) {
    constexpr int NV = 3 * MM;
#pragma unroll 1
    for (int j = 0; j < k; ++j) {
        const int rj = act_at<NV>(act, j);
#pragma unroll 1
        for (int l = 0; l <= j; ++l)
            L[lo_idx(j, l) * stride] = row_pinv_row<MM>(X, Pinv, rj, act_at<NV>(act, l));
    }
#pragma unroll 1
    for (int j = 0; j < k; ++j) {
        double d = L[lo_idx(j, j) * stride];
        for (int l = 0; l < j; ++l) {
            const double v = L[lo_idx(j, l) * stride];
            d -= v * v;
        }
        if (!(d > 0.0)) return false;
        d = sqrt(d);
        L[lo_idx(j, j) * stride] = d;
        for (int i = j + 1; i < k; ++i) {
            double s = L[lo_idx(i, j) * stride];
            for (int l = 0; l < j; ++l) s -= L[lo_idx(i, l) * stride] * L[lo_idx(j, l) * stride];
            L[lo_idx(i, j) * stride] = s / d;
        }
    }
    return true;
}

// Solve (L L^T) x = v in place for the first k entries.
template <int NV, typename LP>
BODEX_FI void chol_solve(LP L, int stride, int k, double* v) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < k) {
            double s = v[i];
#pragma unroll
            for (int l = 0; l < i; ++l) s -= L[lo_idx(i, l) * stride] * v[l];
            v[i] = s / L[lo_idx(i, i) * stride];
        }
    }
#pragma unroll
    for (int i = NV - 1; i >= 0; --i) {
        if (i < k) {
            double s = v[i];
#pragma unroll
            for (int l = i + 1; l < NV; ++l)
                if (l < k) s -= L[lo_idx(l, i) * stride] * v[l];
            v[i] = s / L[lo_idx(i, i) * stride];
        }
    }
}

// Equality-constrained minimiser on the active rows (L already factored):
//   lam = -M^{-1}(b_W + C_W g0),  x = -(g0 + P^{-1} C_W^T lam),  g0 = P^{-1} q.
template <int MM, typename PP, typename LP>
BODEX_FI void eqp_solve(const PolishCtx<MM>& X, PP Pinv, LP L, int stride, const int* act,
                        int k, const double* g0, double* x, double* lam) {
    constexpr int NV = 3 * MM;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        if (j < k) {
            double b;
            const double cg = row_dot<MM>(X, act[j], g0, &b);
            lam[j] = -(b + cg);
        } else {
            lam[j] = 0.0;
        }
    }
    chol_solve<NV>(L, stride, k, lam);
    double t[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) t[v] = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j)
        if (j < k) row_axpy<MM>(X, act[j], lam[j], t);
    double pt[NV];
    symv64<NV>(Pinv, t, pt);
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = -(g0[v] + pt[v]);
}

// One step of iterative refinement of the equality-constrained solve: the
// residuals r1 = P x + q + C_W^T lam (P x formed from G, exactly) and
// r2 = C_W x - b_W are removed with the same factors:
//   dlam = M^{-1}(r2 - C_W P^{-1} r1),  dx = -P^{-1}(r1 + C_W^T dlam).
template <int MM, typename GP, typename PP, typename LP>
BODEX_FI void eqp_refine(const PolishCtx<MM>& X, GP G, PP Pinv, LP L, int stride, const int* act,
                         int k, const double* q, double* x, double* lam) {
    constexpr int NV = 3 * MM;
    double gx[6];
    for (int a = 0; a < 6; ++a) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < NV; ++c) s += G[a * NV + c] * x[c];
        gx[a] = s;
    }
    double r1[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double s = X.eps * x[c];
        for (int a = 0; a < 6; ++a) s += G[a * NV + c] * gx[a];
        r1[c] = 2.0 * s + q[c];
    }
#pragma unroll
    for (int j = 0; j < NV; ++j)
        if (j < k) row_axpy<MM>(X, act[j], lam[j], r1);
    double pr1[NV];
    symv64<NV>(Pinv, r1, pr1);
    double dl[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        if (j < k) {
            double b;
            const double cx = row_dot<MM>(X, act[j], x, &b);
            double bb;
            const double cp = row_dot<MM>(X, act[j], pr1, &bb);
            dl[j] = (cx - b) - cp;
        } else {
            dl[j] = 0.0;
        }
    }
    chol_solve<NV>(L, stride, k, dl);
    double t[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) t[c] = r1[c];
#pragma unroll
    for (int j = 0; j < NV; ++j)
        if (j < k) row_axpy<MM>(X, act[j], dl[j], t);
    double pt[NV];
    symv64<NV>(Pinv, t, pt);
#pragma unroll
    for (int c = 0; c < NV; ++c) x[c] -= pt[c];
#pragma unroll
    for (int j = 0; j < NV; ++j)
        if (j < k) lam[j] += dl[j];
}

// Three-vector helpers for the per-contact independence test.
BODEX_FI double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
BODEX_FI void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

struct PolishOut {
    int status;  // 0 accepted, 1 rejected by the KKT check, 2 step cap, 3 breakdown
    int steps;
    int k;
};

// The polish of one QP.  Inputs: y0 (ADMM-form duals, used to pick the warm
// active set: rows with positive dual), G (FP64 [6][NV]), Pinv (FP64 packed
// upper), q (FP64), L workspace (NV(NV+1)/2 entries at stride `stride`).
// Outputs: x, lam (multipliers of act[0..k-1]), act, k.
template <int MM, typename YP, typename GP, typename PP, typename LP>
BODEX_FI PolishOut polish_qp(const PolishCtx<MM>& X, YP y0, GP G, PP Pinv, const double* q,
                                    LP L, int stride, int max_steps, double* x, double* lam,
                                    int* act, int* kout) {
    constexpr int NV = 3 * MM;
    constexpr int GR = PolishCtx<MM>::GR;
    PolishOut out;
    out.status = 0;
    out.steps = 0;
    out.k = 0;
    int k = 0;
    RowMask mask;
    mask.clear();
    double g0[NV];
    symv64<NV>(Pinv, q, g0);

    // Warm start: per contact, the rows with positive ADMM dual, largest first,
    // kept while linearly independent (at most three per contact).
#pragma unroll
    for (int i = 0; i < MM; ++i) {
        if (i >= X.m) continue;
        double s0[3] = {0, 0, 0}, s1[3] = {0, 0, 0};
        int ns = 0;
        uint32_t used = 0;
        for (int pass = 0; pass < 9 && ns < 3; ++pass) {
            int best = -1;
            double by = 0.0;
            for (int kk = 0; kk < 9; ++kk) {
                const double yv = double(y0[9 * i + kk]);
                if (!((used >> kk) & 1) && yv > by) {
                    by = yv;
                    best = kk;
                }
            }
            if (best < 0) break;
            used |= 1u << best;
            double c[3], b;
            row3(9 * i + best, X.muc[i], X.fmax, c, &b);
            const double nc = sqrt(dot3(c, c));
            bool indep = true;
            if (ns == 1) {
                double cr[3];
                cross3(s0, c, cr);
                indep = sqrt(dot3(cr, cr)) > 1e-6 * nc * sqrt(dot3(s0, s0));
            } else if (ns == 2) {
                double cr[3];
                cross3(s0, s1, cr);
                indep = fabs(dot3(cr, c)) > 1e-6 * nc * sqrt(dot3(cr, cr));
            }
            if (!indep) continue;
            if (ns == 0) {
                s0[0] = c[0]; s0[1] = c[1]; s0[2] = c[2];
            } else if (ns == 1) {
                s1[0] = c[0]; s1[1] = c[1]; s1[2] = c[2];
            }
            ns++;
#pragma unroll
            for (int j = 0; j < NV; ++j)
                if (j == k) act[j] = 9 * i + best;
            mask.set(9 * i + best);
            k++;
        }
    }

    // Minimiser on the warm set; drop rows with negative multipliers until the
    // pair is dual feasible (a valid starting point of the dual method).
    for (;;) {
        if (k > 0 && !factor_active<MM>(X, Pinv, act, k, L, stride)) {
            out.status = 3;
            *kout = k;
            return out;
        }
        eqp_solve<MM>(X, Pinv, L, stride, act, k, g0, x, lam);
        int worst = -1;
        double wv = -1e-14;
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (j < k && lam[j] < wv) {
                wv = lam[j];
                worst = j;
            }
        if (worst < 0) break;
        int dropped = -1;
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (j == worst) dropped = act[j];
        mask.unset(dropped);
#pragma unroll
        for (int j = 0; j < NV - 1; ++j)
            if (j >= worst) {
                act[j] = act[j + 1];
                lam[j] = lam[j + 1];
            }
        k--;
        out.steps++;
    }
    double u[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) u[j] = lam[j];

    const double tol_add = 1e-12 * (1.0 + X.fmax);
    for (;;) {
        // most violated inactive row
        int p = -1;
        double worst = tol_add;
        for (int i = 0; i < X.m; ++i) {
            for (int kk = 0; kk < 9; ++kk) {
                const int r = 9 * i + kk;
                if (mask.has(r)) continue;
                double b;
                const double s = row_dot<MM>(X, r, x, &b) - b;
                if (s > worst) {
                    worst = s;
                    p = r;
                }
            }
        }
        if (X.gamma > 0.0 && !mask.has(GR)) {
            double b;
            const double s = row_dot<MM>(X, GR, x, &b) - b;
            if (s > worst) {
                worst = s;
                p = GR;
            }
        }
        if (p < 0) break;
        double up = 0.0;
        for (;;) {
            if (++out.steps > max_steps) {
                out.status = 2;
                *kout = k;
                return out;
            }
            if (k > 0 && !factor_active<MM>(X, Pinv, act, k, L, stride)) {
                out.status = 3;
                *kout = k;
                return out;
            }
            double hp[NV];
            pinv_row<MM>(X, Pinv, p, hp);
            double r[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                double b;
                r[j] = (j < k) ? row_dot<MM>(X, act[j], hp, &b) : 0.0;
            }
            chol_solve<NV>(L, stride, k, r);
            // z = P^{-1} (c_p - C_W^T r)
            double t[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) t[v] = 0.0;
            row_axpy<MM>(X, p, 1.0, t);
#pragma unroll
            for (int j = 0; j < NV; ++j)
                if (j < k) row_axpy<MM>(X, act[j], -r[j], t);
            double z[NV];
            symv64<NV>(Pinv, t, z);
            double b;
            const double cz = row_dot<MM>(X, p, z, &b);
            const double cpp = row_dot<MM>(X, p, hp, &b);
            const bool dep = !(cz > 1e-10 * cpp);
            double t1 = INFINITY;
            int l = -1;
#pragma unroll
            for (int j = 0; j < NV; ++j)
                if (j < k && r[j] > 0.0 && u[j] / r[j] < t1) {
                    t1 = u[j] / r[j];
                    l = j;
                }
            if (dep && l < 0) {
                out.status = 3;
                *kout = k;
                return out;
            }
            const double sp = row_dot<MM>(X, p, x, &b) - b;
            const double t2 = dep ? INFINITY : sp / cz;
            const double st = t2 < t1 ? t2 : t1;
            if (!dep) {
#pragma unroll
                for (int v = 0; v < NV; ++v) x[v] -= st * z[v];
            }
#pragma unroll
            for (int j = 0; j < NV; ++j)
                if (j < k) u[j] -= st * r[j];
            up += st;
            if (t2 <= t1) {
                if (k >= NV) {
                    out.status = 3;
                    *kout = k;
                    return out;
                }
#pragma unroll
                for (int j = 0; j < NV; ++j)
                    if (j == k) {
                        act[j] = p;
                        u[j] = up;
                    }
                mask.set(p);
                k++;
                break;
            }
            int dropped = -1;
#pragma unroll
            for (int j = 0; j < NV; ++j)
                if (j == l) dropped = act[j];
            mask.unset(dropped);
#pragma unroll
            for (int j = 0; j < NV - 1; ++j)
                if (j >= l) {
                    act[j] = act[j + 1];
                    u[j] = u[j + 1];
                }
            k--;
        }
    }
    // Exact re-solve on the final active set (removes drift of the updates).
    if (k > 0 && !factor_active<MM>(X, Pinv, act, k, L, stride)) {
        out.status = 3;
        *kout = k;
        return out;
    }
    eqp_solve<MM>(X, Pinv, L, stride, act, k, g0, x, lam);
    eqp_refine<MM>(X, G, Pinv, L, stride, act, k, q, x, lam);
    eqp_refine<MM>(X, G, Pinv, L, stride, act, k, q, x, lam);
    *kout = k;
    out.k = k;

    // KKT check with P x formed from G (independent of the accuracy of P^{-1}).
    double gx[6];
    for (int a = 0; a < 6; ++a) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < NV; ++c) s += G[a * NV + c] * x[c];
        gx[a] = s;
    }
    double st[NV];
    double sq = 0.0, spx = 0.0;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double s = X.eps * x[c];
        for (int a = 0; a < 6; ++a) s += G[a * NV + c] * gx[a];
        st[c] = 2.0 * s + q[c];
        sq = fmax(sq, fabs(q[c]));
        spx = fmax(spx, fabs(2.0 * s));
    }
    double lmax = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j)
        if (j < k) {
            row_axpy<MM>(X, act[j], lam[j], st);
            lmax = fmax(lmax, fabs(lam[j]));
        }
    double stat = 0.0;
#pragma unroll
    for (int c = 0; c < NV; ++c) stat = fmax(stat, fabs(st[c]));
    double lneg = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j)
        if (j < k) lneg = fmax(lneg, -lam[j]);
    double viol = 0.0;
    for (int i = 0; i < X.m; ++i)
        for (int kk = 0; kk < 9; ++kk) {
            double b;
            viol = fmax(viol, row_dot<MM>(X, 9 * i + kk, x, &b) - b);
        }
    if (X.gamma > 0.0) {
        double b;
        viol = fmax(viol, row_dot<MM>(X, GR, x, &b) - b);
    }
    const bool ok = stat <= 1e-9 * (1.0 + sq + spx) && lneg <= 1e-9 * (1.0 + lmax) &&
                    viol <= 1e-9 * (1.0 + X.fmax) && isfinite(stat);
    out.status = ok ? 0 : 1;
    return out;
}

// Relative KKT residual (same definition as the ADMM check) of an FP32 state
// (x, z, y), evaluated in FP64.
template <int MM, typename GP>
BODEX_FI double rel_kkt64(GP G, const double* muc, const double* q, int m, double eps,
                                 const float* x, const float* z, const float* y) {
    constexpr int NV = 3 * MM;
    double rp = 0, nAx = 0, nz = 0, aty[NV];
    double s1 = 0.0;
#pragma unroll
    for (int i = 0; i < MM; ++i) {
        double a1 = 0, a2 = 0, a3 = 0;
        if (i < m) {
            const double x1 = x[3 * i], x2 = x[3 * i + 1], x3 = x[3 * i + 2];
            for (int k = 0; k < 8; ++k) {
                const double ck = facet_cos<double>(k), sk = facet_sin<double>(k);
                const double ax = ck * x2 + sk * x3 - muc[i] * x1;
                const double zk = z[9 * i + k], yk = y[9 * i + k];
                rp = fmax(rp, fabs(ax - zk));
                nAx = fmax(nAx, fabs(ax));
                nz = fmax(nz, fabs(zk));
                a1 -= muc[i] * yk;
                a2 += ck * yk;
                a3 += sk * yk;
            }
            const double zb = z[9 * i + 8];
            a1 += double(y[9 * i + 8]) + double(y[9 * MM]);
            rp = fmax(rp, fabs(x1 - zb));
            nAx = fmax(nAx, fabs(x1));
            nz = fmax(nz, fabs(zb));
            s1 += x1;
        }
        aty[3 * i] = a1;
        aty[3 * i + 1] = a2;
        aty[3 * i + 2] = a3;
    }
    const double zg = z[9 * MM];
    rp = fmax(rp, fabs(s1 - zg));
    nAx = fmax(nAx, fabs(s1));
    nz = fmax(nz, fabs(zg));
    double gx[6];
    for (int a = 0; a < 6; ++a) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < NV; ++c) s += G[a * NV + c] * double(x[c]);
        gx[a] = s;
    }
    double rd = 0, nPx = 0, nAty = 0, nq = 0;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double s = eps * double(x[c]);
        for (int a = 0; a < 6; ++a) s += G[a * NV + c] * gx[a];
        const double px = 2.0 * s;
        rd = fmax(rd, fabs(px + q[c] + aty[c]));
        nPx = fmax(nPx, fabs(px));
        nAty = fmax(nAty, fabs(aty[c]));
        nq = fmax(nq, fabs(q[c]));
    }
    return fmax(rp / (1.0 + fmax(nAx, nz)), rd / (1.0 + fmax(fmax(nPx, nAty), nq)));
}

}  // namespace bodex
