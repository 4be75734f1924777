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

#include <type_traits>

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
// Constraint rows of the polish, one-sided C f <= b, with the ADMM-form row
// ids: 9i+k facet k of contact i (b = 0), 9i+8 the upper normal bound
// f_i1 <= fmax, 9 MM the normal-sum row -sum f_i1 <= -gamma (used only when
// gamma > 0).  The lower normal bound f_i1 >= 0 is implied by the facets and
// is not a separate row.
// ---------------------------------------------------------------------------

// cos and sin of facet k's angle (2k+1) pi/8 for a run-time k: the
// magnitudes are cos(pi/8) or sin(pi/8) (cos is the larger for k in
// {0, 3, 4, 7}); cos is negative for k in 2..5, sin for k in 4..7.
BODEX_FI void facet_cs(int k, double* ck, double* sk) {
    const bool cbig = ((k ^ (k >> 1)) & 1) == 0;
    const double a = cbig ? kC8 : kS8, b = cbig ? kS8 : kC8;
    *ck = ((k + 2) & 4) ? -a : a;
    *sk = (k & 4) ? -b : b;
}

// Coefficients of row kk (0..8) of a contact on its 3 variables: facet kk
// (b = 0) or the upper normal bound (kk = 8, b = fmax).
BODEX_FI void row3(int kk, double muc, double fm, double c[3], double* b) {
    double ck, sk;
    facet_cs(kk & 7, &ck, &sk);
    const bool bound = kk == 8;
    c[0] = bound ? 1.0 : -muc;
    c[1] = bound ? 0.0 : ck;
    c[2] = bound ? 0.0 : sk;
    *b = bound ? fm : 0.0;
}

// Three-vector helpers.
BODEX_FI double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
BODEX_FI void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// ---------------------------------------------------------------------------
// FP64 polish (the finishing step of the solver).  A dual active-set method
// (Goldfarb-Idnani) on the QP, warm-started from the ADMM duals, whose linear
// algebra uses the structure of the problem instead of a dense reduced
// matrix:
//  * the active rows are kept per contact (at most three independent rows of
//    the nine each), plus optionally the normal-sum row, which couples all
//    contacts;
//  * per contact, the projector Pi_i onto the null space of its active rows
//    has a closed form (identity, minus one direction, one direction, zero),
//    so with Pi = diag(Pi_i) and P = 2 (G^T G + eps I) the reduced inverse is
//      H v = Z (Z^T P Z)^{-1} Z^T v
//          = (Pi v - Pi G^T (eps I6 + G Pi G^T)^{-1} G Pi v) / (2 eps),
//    one 6x6 Cholesky factor per active set (Woodbury identity), whose
//    matrix changes by a rank-one term when one row joins or leaves;
//  * an active normal-sum row a removes one more direction from Pi: the unit
//    vector along u = Pi a (u lies in the contacts' null spaces).
// Multipliers follow from stationarity: per contact from the closed-form
// inverse of its <= 3 rows, the normal-sum multiplier from a least-squares
// fit over the contacts' null spaces.
// ---------------------------------------------------------------------------

// Active rows of one contact, ascending row ids taken from the mask bits
// (callers keep at most three); unused entries repeat row 8.
struct ContactRows {
    int n;
    int id[3];
    double c[3][3];
    double b[3];
};

BODEX_FI void contact_rows(unsigned mask, double muc, double fm, ContactRows& R) {
    R.n = __builtin_popcount(mask);
    unsigned mk = mask;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int id = mk ? __builtin_ctz(mk) : 8;
        mk &= mk - 1u;
        R.id[j] = id;
        row3(id, muc, fm, R.c[j], &R.b[j]);
    }
}

// Null-space projector of one contact, Pi v = a v + k (e . v) e: with n
// active rows, n = 0: a = 1, k = 0; n = 1: e along the row, a = 1,
// k = -1/|e|^2; n = 2: e along c0 x c1, a = 0, k = 1/|e|^2; n = 3: a = k = 0.
// e need not be a unit vector (k carries the scale, so building a projector
// takes one division and no square root).
struct ContactProj {
    double e[3];
    double k, a;
};

// Coefficients for a unit e.
BODEX_FI void proj_coeffs(int n, ContactProj& P) {
    P.k = (n == 1) ? -1.0 : (n == 2 ? 1.0 : 0.0);
    P.a = (n <= 1) ? 1.0 : 0.0;
}

BODEX_FI void contact_proj(const ContactRows& R, ContactProj& P) {
    if (R.n == 2) {
        cross3(R.c[0], R.c[1], P.e);
    } else {
#pragma unroll
        for (int t = 0; t < 3; ++t) P.e[t] = R.c[0][t];
    }
    const double q = (R.n == 1 || R.n == 2) ? 1.0 / dot3(P.e, P.e) : 0.0;
    P.k = (R.n == 1) ? -q : q;
    P.a = (R.n <= 1) ? 1.0 : 0.0;
}

// The unit direction of a projector (for the cache, which keeps only e).
BODEX_FI void proj_unit(const ContactProj& P, double* e) {
    const double s = P.k != 0.0 ? sqrt(fabs(P.k)) : 1.0;
#pragma unroll
    for (int t = 0; t < 3; ++t) e[t] = s * P.e[t];
}

BODEX_FI void proj_apply(const ContactProj& P, double* v) {
    const double d = dot3(P.e, v) * P.k;
#pragma unroll
    for (int t = 0; t < 3; ++t) v[t] = P.a * v[t] + d * P.e[t];
}

// u_i = Pi_i a_i with a_i = (-1, 0, 0), the contact's share of the
// normal-sum row.
BODEX_FI void sum_row_complement(const ContactProj& P, double* u) {
    const double d = -P.e[0] * P.k;
#pragma unroll
    for (int t = 0; t < 3; ++t) u[t] = d * P.e[t];
    u[0] -= P.a;
}

// Coefficients r with sum_j r_j c_j = w for w in the span of the rows.
BODEX_FI void rows_coeffs(const ContactRows& R, const double* w, double* r) {
    r[0] = r[1] = r[2] = 0.0;
    if (R.n == 1) {
        r[0] = dot3(R.c[0], w) / dot3(R.c[0], R.c[0]);
    } else if (R.n == 2) {
        const double a = dot3(R.c[0], R.c[0]), b = dot3(R.c[0], R.c[1]), d = dot3(R.c[1], R.c[1]);
        const double p = dot3(R.c[0], w), q = dot3(R.c[1], w);
        const double id = 1.0 / (a * d - b * b);
        r[0] = (d * p - b * q) * id;
        r[1] = (a * q - b * p) * id;
    } else if (R.n >= 3) {
        double k[3], t[3];
        cross3(R.c[1], R.c[2], k);
        const double iD = 1.0 / dot3(R.c[0], k);
        r[0] = dot3(w, k) * iD;
        cross3(w, R.c[2], t);
        r[1] = dot3(R.c[0], t) * iD;
        cross3(R.c[1], w, t);
        r[2] = dot3(R.c[0], t) * iD;
    }
}

// Row coefficients of two vectors in the span of the rows (w -> r, h -> l),
// sharing the inverse of the rows' Gram (or triple-product) denominator.
BODEX_FI void rows_coeffs2(const ContactRows& R, const double* w, const double* h, double* r, double* l) {
    r[0] = r[1] = r[2] = 0.0;
    l[0] = l[1] = l[2] = 0.0;
    if (R.n == 1) {
        const double ia = 1.0 / dot3(R.c[0], R.c[0]);
        r[0] = dot3(R.c[0], w) * ia;
        l[0] = dot3(R.c[0], h) * ia;
    } else if (R.n == 2) {
        const double a = dot3(R.c[0], R.c[0]), b = dot3(R.c[0], R.c[1]), d = dot3(R.c[1], R.c[1]);
        const double id = 1.0 / (a * d - b * b);
        const double p = dot3(R.c[0], w), q = dot3(R.c[1], w);
        const double ph = dot3(R.c[0], h), qh = dot3(R.c[1], h);
        r[0] = (d * p - b * q) * id;
        r[1] = (a * q - b * p) * id;
        l[0] = (d * ph - b * qh) * id;
        l[1] = (a * qh - b * ph) * id;
    } else if (R.n >= 3) {
        double k[3], t[3];
        cross3(R.c[1], R.c[2], k);
        const double iD = 1.0 / dot3(R.c[0], k);
        r[0] = dot3(w, k) * iD;
        l[0] = dot3(h, k) * iD;
        cross3(w, R.c[2], t);
        r[1] = dot3(R.c[0], t) * iD;
        cross3(h, R.c[2], t);
        l[1] = dot3(R.c[0], t) * iD;
        cross3(R.c[1], w, t);
        r[2] = dot3(R.c[0], t) * iD;
        cross3(R.c[1], h, t);
        l[2] = dot3(R.c[0], t) * iD;
    }
}

// Least-norm point of {c_j . f = b_j}.
BODEX_FI void rows_point(const ContactRows& R, double* f) {
    f[0] = f[1] = f[2] = 0.0;
    if (R.n == 1) {
        const double s = R.b[0] / dot3(R.c[0], R.c[0]);
        for (int t = 0; t < 3; ++t) f[t] = s * R.c[0][t];
    } else if (R.n == 2) {
        const double a = dot3(R.c[0], R.c[0]), b = dot3(R.c[0], R.c[1]), d = dot3(R.c[1], R.c[1]);
        const double id = 1.0 / (a * d - b * b);
        const double y0 = (d * R.b[0] - b * R.b[1]) * id, y1 = (a * R.b[1] - b * R.b[0]) * id;
        for (int t = 0; t < 3; ++t) f[t] = y0 * R.c[0][t] + y1 * R.c[1][t];
    } else if (R.n >= 3) {
        double k0[3], k1[3], k2[3];
        cross3(R.c[1], R.c[2], k0);
        cross3(R.c[2], R.c[0], k1);
        cross3(R.c[0], R.c[1], k2);
        const double iD = 1.0 / dot3(R.c[0], k0);
        for (int t = 0; t < 3; ++t) f[t] = (R.b[0] * k0[t] + R.b[1] * k1[t] + R.b[2] * k2[t]) * iD;
    }
}

// 6x6 symmetric positive definite matrix, packed lower, and its Cholesky.
struct Sym6 {
    double a[21];
};

// The same matrix in memory shared by the lanes that hold identical copies
// (entry e at p[e * stride]); the chol6 routines take either form.
struct Sym6Shared {
    struct Entries {
        double* p;
        int stride;
        BODEX_FI double& operator[](int e) const { return p[e * stride]; }
    } a;
};

template <class S6>
BODEX_FI bool chol6(S6& M) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double d = M.a[lo_idx(j, j)];
#pragma unroll
        for (int l = 0; l < j; ++l) d -= M.a[lo_idx(j, l)] * M.a[lo_idx(j, l)];
        if (!(d > 0.0)) return false;
        d = sqrt(d);
        M.a[lo_idx(j, j)] = d;
        const double id = 1.0 / d;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double s = M.a[lo_idx(i, j)];
#pragma unroll
            for (int l = 0; l < j; ++l) s -= M.a[lo_idx(i, l)] * M.a[lo_idx(j, l)];
            M.a[lo_idx(i, j)] = s * id;
        }
        // keep the reciprocal of the pivot for the solves
        M.a[lo_idx(j, j)] = id;
    }
    return true;
}

// Solve (L L^T) v = rhs in place; the diagonal of L holds reciprocals.
template <class S6>
BODEX_FI void chol6_solve(const S6& L, double* v) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = v[i];
#pragma unroll
        for (int l = 0; l < i; ++l) s -= L.a[lo_idx(i, l)] * v[l];
        v[i] = s * L.a[lo_idx(i, i)];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = v[i];
#pragma unroll
        for (int l = i + 1; l < 6; ++l) s -= L.a[lo_idx(l, i)] * v[l];
        v[i] = s * L.a[lo_idx(i, i)];
    }
}

// M = L L^T in place (L packed lower with reciprocal diagonal): rows from
// the last, each from its diagonal down, so that every entry of L is read
// before it is overwritten.
template <class S6>
BODEX_FI void chol6_product(S6& L) {
    double d[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) d[k] = 1.0 / L.a[lo_idx(k, k)];
#pragma unroll
    for (int i = 5; i >= 0; --i)
#pragma unroll
        for (int j = i; j >= 0; --j) {
            double s = (j == i) ? d[i] * d[i] : L.a[lo_idx(i, j)] * d[j];
#pragma unroll
            for (int k = 0; k < j; ++k) s += L.a[lo_idx(i, k)] * L.a[lo_idx(j, k)];
            L.a[lo_idx(i, j)] = s;
        }
}

// The problem data the polish reads: G in FP64 [6][3 MM] (row-major), mu_i
// cos(pi/8), beta t of the lane's wrench, and the scalars.  GAM: code for the
// normal-sum row is compiled in.
template <int MM, typename GP, bool GAM>
struct PolishData {
    static constexpr int kMM = MM;
    static constexpr bool kGam = GAM;
    GP G;
    const double* muc;
    double bt[6];
    int m;
    double fmax, gamma, eps;
};

// One lane's vector in memory shared by the lanes: element c at
// p[c * stride] (lane-interleaved).
struct LaneVec {
    double* p;
    int stride;
    BODEX_FI double& operator[](int c) const { return p[c * stride]; }
};

// One lane's vector in its registers (a local array of the caller).  The
// polish indexes it only with wave-uniform indices (loops over contacts
// run the same trip count on every lane), which the compiler can serve
// from registers without unrolling the loops.
struct RegVec {
    double* p;
    BODEX_FI double& operator[](int c) const { return p[c]; }
};

// The polish's per-lane vectors: the point x and the step z (3 m each).
template <class V>
struct PolishWork {
    V x, z;
};

// Active set: bit 9i+kk of mask is row kk of contact i; gam: the normal-sum
// row; L: the factor of eps I6 + G Pi G^T; the contacts' projectors, kept
// from the last factorisation.
// Bits of the contact rows' active set: 9 per contact (64 bits up to 7
// contacts, 128 for 8).
template <int MM>
using RowMask = typename std::conditional<(9 * MM <= 64), uint64_t, unsigned __int128>::type;

template <int MM>
struct ActiveSet {
    RowMask<MM> mask;
    bool gam;
    Sym6 L;
    LaneVec pc;  // per contact: the unit e of its projector (a, k follow from the mask)
};

template <class Mask>
BODEX_FI unsigned contact_mask(Mask mask, int i) { return unsigned(mask >> (9 * i)) & 0x1FFu; }

template <typename D, int MM>
BODEX_FI void contact_geom(const D& Dt, const ActiveSet<MM>& S, int i, ContactRows& R, ContactProj& P) {
    contact_rows(contact_mask(S.mask, i), Dt.muc[i], Dt.fmax, R);
    contact_proj(R, P);
}

// Contact i's projector: from the cache the last factorisation filled, or,
// when no cache is attached (pc.p null), recomputed from the active rows.
template <typename D, int MM>
BODEX_FI ContactProj cached_proj(const D& Dt, const ActiveSet<MM>& S, int i) {
    ContactProj P;
    if (S.pc.p == nullptr) {
        ContactRows R;
        contact_rows(contact_mask(S.mask, i), Dt.muc[i], Dt.fmax, R);
        contact_proj(R, P);
        return P;
    }
    P.e[0] = S.pc[3 * i];
    P.e[1] = S.pc[3 * i + 1];
    P.e[2] = S.pc[3 * i + 2];
    proj_coeffs(__builtin_popcount(contact_mask(S.mask, i)), P);
    return P;
}

// r6 = G v (minus beta t when with_t).
template <int MM, typename D, class V>
BODEX_FI void g_times(const D& Dt, const V& v, bool with_t, double* r6) {
    constexpr int NV = 3 * MM;
#pragma unroll
    for (int k = 0; k < 6; ++k) r6[k] = with_t ? -Dt.bt[k] : 0.0;
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= Dt.m) continue;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const double vc = v[3 * i + t];
#pragma unroll
            for (int k = 0; k < 6; ++k) r6[k] += Dt.G[k * NV + 3 * i + t] * vc;
        }
    }
}

// Contact i's part of 2 (G^T r6 + eps v).
template <int MM, typename D, class V>
BODEX_FI void contact_grad(const D& Dt, int i, const double* r6, const V& v, double* g) {
    constexpr int NV = 3 * MM;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        double s = Dt.eps * v[3 * i + t];
#pragma unroll
        for (int k = 0; k < 6; ++k) s += Dt.G[k * NV + 3 * i + t] * r6[k];
        g[t] = 2.0 * s;
    }
}

// In place: v <- H v.
template <int MM, typename D, class V>
BODEX_FI void apply_h(const D& Dt, const ActiveSet<MM>& S, const V& v) {
    constexpr int NV = 3 * MM;
    const bool gam = D::kGam && S.gam;
    const int m = Dt.m;
    // v <- Pi v (per contact; the normal-sum direction below)
    double uu = 0.0, uv = 0.0;
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= m) continue;
        const ContactProj P = cached_proj(Dt, S, i);
        double f[3] = {v[3 * i], v[3 * i + 1], v[3 * i + 2]};
        proj_apply(P, f);
        if (gam) {
            double u[3];
            sum_row_complement(P, u);
            uu += dot3(u, u);
            uv += dot3(u, f);
        }
#pragma unroll
        for (int t = 0; t < 3; ++t) v[3 * i + t] = f[t];
    }
    const double su = gam ? uv / uu : 0.0;
    double gv[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) gv[k] = 0.0;
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= m) continue;
        double f[3] = {v[3 * i], v[3 * i + 1], v[3 * i + 2]};
        if (gam) {
            double u[3];
            sum_row_complement(cached_proj(Dt, S, i), u);
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                f[t] -= su * u[t];
                v[3 * i + t] = f[t];
            }
        }
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int k = 0; k < 6; ++k) gv[k] += Dt.G[k * NV + 3 * i + t] * f[t];
    }
    chol6_solve(S.L, gv);
    // v <- (v - Pi G^T gv) / (2 eps)
    const double s2 = 0.5 / Dt.eps;
    double ut = 0.0;
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= m) continue;
        double t3[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) s += Dt.G[k * NV + 3 * i + t] * gv[k];
            t3[t] = s;
        }
        const ContactProj P = cached_proj(Dt, S, i);
        proj_apply(P, t3);
        if (gam) {
            double u[3];
            sum_row_complement(P, u);
            ut += dot3(u, t3);
        }
#pragma unroll
        for (int t = 0; t < 3; ++t) v[3 * i + t] = s2 * (v[3 * i + t] - t3[t]);
    }
    if (gam) {
        const double sc = s2 * ut / uu;
#pragma unroll 1
        for (int i = 0; i < MM; ++i) {
            if (i >= m) continue;
            double u[3];
            sum_row_complement(cached_proj(Dt, S, i), u);
#pragma unroll
            for (int t = 0; t < 3; ++t) v[3 * i + t] += sc * u[t];
        }
    }
}

// |u|^2 for the current masks (0 when the normal-sum row is dependent on
// the contacts' rows).
template <typename D, int MM>
BODEX_FI double sum_row_norm2(const D& Dt, const ActiveSet<MM>& S) {
    double un = 0.0;
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= Dt.m) continue;
        ContactRows R;
        ContactProj P;
        contact_geom(Dt, S, i, R, P);
        double u[3];
        sum_row_complement(P, u);
        un += dot3(u, u);
    }
    return un;
}

// Refresh the projectors and form (in S.L, to be factored) eps I6 + G Pi G^T
// = eps I6 + sum_i (G_i Pi_i)(G_i Pi_i)^T, minus (G u)(G u)^T / |u|^2 with
// the normal-sum row.
template <int MM, typename D>
BODEX_FI bool set_matrix(const D& Dt, ActiveSet<MM>& S) {
    constexpr int NV = 3 * MM;
    const bool gam = D::kGam && S.gam;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) S.L.a[lo_idx(r, c)] = (r == c) ? Dt.eps : 0.0;
    double gu[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, uu = 0.0;
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= Dt.m) continue;
        ContactRows R;
        ContactProj P;
        contact_geom(Dt, S, i, R, P);
        if (S.pc.p != nullptr) {
            double e[3];
            proj_unit(P, e);
#pragma unroll
            for (int t = 0; t < 3; ++t) S.pc[3 * i + t] = e[t];
        }
        double b[6][3];
#pragma unroll
        for (int k = 0; k < 6; ++k)
#pragma unroll
            for (int t = 0; t < 3; ++t) b[k][t] = Dt.G[k * NV + 3 * i + t];
        if (gam) {
            double u[3];
            sum_row_complement(P, u);
            uu += dot3(u, u);
#pragma unroll
            for (int k = 0; k < 6; ++k) gu[k] += dot3(b[k], u);
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) proj_apply(P, b[k]);
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) S.L.a[lo_idx(r, c)] += dot3(b[r], b[c]);
    }
    if (gam) {
        if (!(uu > 0.0)) return false;
        const double iu = 1.0 / uu;
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) S.L.a[lo_idx(r, c)] -= gu[r] * gu[c] * iu;
    }
    return true;
}

// One row (kk) of contact i has just joined (sgn = -1) or left (sgn = +1)
// the active set; S.mask holds the new set and S.L the factor of the old
// one.  With Q the projector of the contact's other active rows and
// e = Q c / |Q c| (c the row's coefficients), the contact's projector goes
// from Q to Q - e e^T when the row joins and back when it leaves, so
// eps I6 + G Pi G^T changes by sgn (G_i e)(G_i e)^T: the new matrix is
// formed from the old factor (to be factored like a fresh one) instead of
// from every contact.  Also refreshes the contact's cached projector.
template <int MM, typename D>
BODEX_FI bool matrix_row_change(const D& Dt, ActiveSet<MM>& S, int i, int kk, double sgn) {
    constexpr int NV = 3 * MM;
    const unsigned now = contact_mask(S.mask, i);
    ContactRows R;
    ContactProj Q;
    contact_rows(now & ~(1u << kk), Dt.muc[i], Dt.fmax, R);
    contact_proj(R, Q);
    double c[3], b;
    row3(kk, Dt.muc[i], Dt.fmax, c, &b);
    proj_apply(Q, c);
    const double n2 = dot3(c, c);
    if (!(n2 > 0.0)) return false;
    const double s = sgn / n2;
    double v[6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        v[k] = Dt.G[k * NV + 3 * i] * c[0] + Dt.G[k * NV + 3 * i + 1] * c[1] + Dt.G[k * NV + 3 * i + 2] * c[2];
    chol6_product(S.L);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int q = 0; q <= r; ++q) S.L.a[lo_idx(r, q)] += s * v[r] * v[q];
    if (S.pc.p != nullptr) {
        ContactProj P;
        double e[3];
        contact_rows(now, Dt.muc[i], Dt.fmax, R);
        contact_proj(R, P);
        proj_unit(P, e);
#pragma unroll
        for (int t = 0; t < 3; ++t) S.pc[3 * i + t] = e[t];
    }
    return true;
}

// The pending row p of the one-row steps: contact pi, row pk (pk = 9: the
// normal-sum row, pk < 0: none) and its coefficients on one contact.
struct PendingRow {
    int pi, pk;
    double c[3];
    double b;
};

BODEX_FI bool pending_on(const PendingRow& p, int i) { return p.pk == 9 || (p.pk >= 0 && i == p.pi); }

// Multipliers from stationarity at x with a partial multiplier up on the
// pending row: -grad(x) - up c_p = sum_i C_i^T lam_i + lg a.  They are not
// stored: sum_row_multiplier gives lg (a least-squares fit over the
// contacts' null spaces, using the projectors of the last factorisation),
// contact_multipliers contact i's lam_i (ascending row order) when needed.
// r6 = G x - beta t.
template <int MM, typename D, class V>
BODEX_FI double sum_row_multiplier(const D& Dt, const ActiveSet<MM>& S, const V& x, const double* r6,
                                   const PendingRow& p, double up) {
    if (!(D::kGam && S.gam)) return 0.0;
    double num = 0.0, den = 0.0;
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= Dt.m) continue;
        double h[3], u[3];
        contact_grad<MM>(Dt, i, r6, x, h);
        const bool on = pending_on(p, i);
#pragma unroll
        for (int t = 0; t < 3; ++t) h[t] = -h[t] - (on ? up * p.c[t] : 0.0);
        sum_row_complement(cached_proj(Dt, S, i), u);
        num += dot3(u, h);
        den += dot3(u, u);
    }
    return num / den;
}

// h = -grad_i(x) - up c_p (on the pending row's contact) + lg e_0: the
// right-hand side whose row coefficients are contact i's multipliers.
template <int MM, typename D, class V>
BODEX_FI void multiplier_rhs(const D& Dt, const V& x, const double* r6, int i, const PendingRow& p, double up,
                             double lg, double* h) {
    contact_grad<MM>(Dt, i, r6, x, h);
    const bool on = pending_on(p, i);
#pragma unroll
    for (int t = 0; t < 3; ++t) h[t] = -h[t] - (on ? up * p.c[t] : 0.0);
    h[0] += lg;
}

template <int MM, typename D, class V>
BODEX_FI void contact_multipliers(const D& Dt, const ContactRows& R, const V& x, const double* r6, int i,
                                  const PendingRow& p, double up, double lg, double* lam) {
    double h[3];
    multiplier_rhs<MM>(Dt, x, r6, i, p, up, lg, h);
    rows_coeffs(R, h, lam);
}

// Start of the equality-constrained solve: x <- a point on the active rows
// (per contact the least-norm point of its rows, then, with the normal-sum
// row, a move inside the contacts' null spaces onto that row; z is used as
// work space).
template <int MM, typename D, class V>
BODEX_FI void eqp_start(const D& Dt, const ActiveSet<MM>& S, const PolishWork<V>& W) {
    double un = 0.0, ax = 0.0;
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= Dt.m) continue;
        ContactRows R;
        contact_rows(contact_mask(S.mask, i), Dt.muc[i], Dt.fmax, R);
        double f[3], u[3];
        rows_point(R, f);
        sum_row_complement(cached_proj(Dt, S, i), u);
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            W.x[3 * i + t] = f[t];
            W.z[3 * i + t] = u[t];
        }
        un += dot3(u, u);
        ax -= f[0];
    }
    if (D::kGam && S.gam) {
        const double s = (-Dt.gamma - ax) / un;
#pragma unroll 1
        for (int i = 0; i < MM; ++i) {
            if (i >= Dt.m) continue;
#pragma unroll
            for (int t = 0; t < 3; ++t) W.x[3 * i + t] += s * W.z[3 * i + t];
        }
    }
}

// The most violated inactive row at x (pk < 0: none above the tolerance).
template <int MM, typename D, class V>
BODEX_FI PendingRow most_violated(const D& Dt, const ActiveSet<MM>& S, const PolishWork<V>& W, bool use_gam,
                                  double tol) {
    PendingRow p = {-1, -1, {0.0, 0.0, 0.0}, 0.0};
    double worst = tol, sum1 = 0.0;
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= Dt.m) continue;
        const double f[3] = {W.x[3 * i], W.x[3 * i + 1], W.x[3 * i + 2]};
        const unsigned mk = contact_mask(S.mask, i);
        const double mu = Dt.muc[i];
        sum1 += f[0];
#pragma unroll
        for (int kk = 0; kk < 9; ++kk) {
            double c[3], b;
            row3(kk, mu, Dt.fmax, c, &b);
            const double s = dot3(c, f) - b;
            if (!((mk >> kk) & 1u) && s > worst) {
                worst = s;
                p.pi = i;
                p.pk = kk;
            }
        }
    }
    if (use_gam && !S.gam && Dt.gamma - sum1 > worst) {
        p.pi = -1;
        p.pk = 9;
    }
    if (p.pk == 9) {
        p.c[0] = -1.0;
        p.c[1] = p.c[2] = 0.0;
        p.b = -Dt.gamma;
    } else if (p.pk >= 0) {
        row3(p.pk, Dt.muc[p.pi], Dt.fmax, p.c, &p.b);
    }
    return p;
}

struct PolishOut {
    int status;  // 0 accepted, 1 rejected by the KKT check, 2 step cap, 3 breakdown
    int steps;   // factorisations, fresh or by a rank-one change
    int updates; // ... of which rank-one changes
    int eqps;   // equality-constrained solves (two passes and the multipliers each)
    int moves;   // one-row steps (ratio test and move; the refactor and the
                 // multipliers that follow are counted in steps and moves)
    int picks;   // searches for the most violated row
};

// Algorithmic FP64 flops of one polish (FMA = 2, add/mul/div/sqrt = 1,
// selects and compares 0), from the arithmetic of each routine at m contacts
// and the counts it reports; normal-sum row terms (gamma > 0) are left out:
//   warm start            249 m per pass, 3 passes  (projector 15 + 9 rows x
//                         (projection 15, two dots 10, scale 1))
//   factorisation         231 m + 100  (6 projected G rows, 21 dots, 6x6 Cholesky 97)
//   one-row change        308          (projector of the other rows 15, projected
//                         row 20, G_i e 31, L L^T 97, plus s v v^T 48, 6x6 Cholesky 97)
//   reduced solve H v     108 m + 72   (two projections, G v, G^T w, 6x6 solves 72)
//   equality solve        527 m + 144  (start point 36 m, two passes of gradient 78 m
//                         + H v + update 3 m, multiplier check 113 m)
//   one-row step          381 m + 78   (direction 31 m + H v, G z 36 m, ratio test
//                         87 m + 1 and the multipliers at x 113 m, update 6 m)
//   violated-row search   54 m
//   acceptance            227 m
BODEX_FI double polish_flops(int m, const PolishOut& o) {
    const double dm = m;
    return 3.0 * 249.0 * dm + 227.0 * dm + (o.steps - o.updates) * (231.0 * dm + 100.0) + o.updates * 308.0 +
           o.eqps * (527.0 * dm + 144.0) + o.moves * (381.0 * dm + 78.0) + o.picks * 54.0 * dm;
}

// The polish of one QP, as a resumable state machine: polish_begin sets the
// warm active set, each polish_advance takes one step of the method and
// returns true once the QP has reached its acceptance check or failed
// (PS.out.status set), and polish_finish then runs the check.
// On finish W.x holds the point, PS.S the active set and PS.lg the
// normal-sum multiplier (contact_multipliers gives the others).  y0:
// ADMM-form duals (rows 9i+kk and the normal-sum row 9 MM); rows with
// positive dual (negative for the normal-sum row) seed the active set.
//
// The method, in order: (1) on the warm set, the minimiser with the active
// rows as equalities (x <- x0 - H grad(x0), twice); while a multiplier is
// negative, drop the most negative row and repeat; (2) while a row is
// violated, take the most violated row p and move along z = H c_p, dropping
// rows whose multipliers reach zero, until p is satisfied (then it joins the
// set) -- the dual active-set steps; (3) after any step, the minimiser on
// the final set once more, exactly, then the KKT acceptance check.  Each
// linear-algebra routine has a single call site in polish_advance (small
// code on the GPU), and a lane can start the next QP as soon as its current
// one finishes.  Every set change is one row, so after the first
// factorisation each new matrix is formed from the previous factor and that
// row's rank-one term (matrix_row_change: ~310 flops against ~1250 for a
// matrix from every contact at m = 5); the two-pass equality solves absorb
// the rounding this carries from set to set, and a QP whose acceptance
// check fails after such changes is taken once more from its last set with
// fresh factorisations only.  With the normal-sum row (whose term involves
// every contact) every matrix is formed from scratch.
enum PolishPhase { kWarm, kSteps, kFinal };
enum PolishMode { kEqp0, kEqp1, kStep, kCheck, kPick, kAccept };
enum PolishChange {
    kNoChange = 0x1FF,
    kChgJoin = 1 << 9,
    kChgUsed = 1 << 10,
    kChgAllowed = 1 << 11,
    kChgRetry = 1 << 12, // take the retry below even after an accepted check (tests)
    kChgBreak = 1 << 13, // report one breakdown of the ratio test after a one-row change (tests)
    kChgCold = 1 << 14,  // the restart from the empty active set has been taken
    kChgBreakAny = 1 << 15  // report one breakdown of the next ratio test (tests)
};

// The pending set change in PS.chg: row 9 i + kk, joined or left.
BODEX_FI int with_change(int chg, int row, bool join) {
    return (chg & ~(kNoChange | kChgJoin)) | row | (join ? int(kChgJoin) : 0);
}

template <int MM>
struct PolishState {
    ActiveSet<MM> S;
    PendingRow p, mp;  // pending row; row of the multipliers still to compute
    double up, mup, lg;
    int phase, mode;
    bool refactor, need_mult;
    // bits 0-8: row 9 i + kk of the set change the next factorisation may
    // take as a one-row change of the last factor (kNoChange: none), bit 9:
    // it joined; flags: such changes were used, they are allowed, a retry
    // is forced
    int chg;
    int step0;   // factorisations before the current attempt (the retry has its own cap)
    int budget;  // factorisations after which the polish suspends (status 4) before the next one
    PolishOut out;
};

// Status of a polish that stopped at its budget with a factorisation due:
// its state can be saved (polish_save) and continued elsewhere.
constexpr int kPolishSuspended = 4;
// Acceptance-check outcome (never returned): stationary with nonnegative
// multipliers, but a row outside the active set is violated.  The exact
// re-solve after the last step corrects what the steps' updates accumulated
// and can move the point across such a row (rarely, after long step
// sequences on ill-conditioned sets); the polish then takes more steps.
constexpr int kPolishViolated = 5;

template <int MM, typename YP, typename D>
BODEX_FI void polish_begin(const D& Dt, YP y0, PolishState<MM>& PS) {
    PolishOut& out = PS.out;
    out.status = 0;
    out.steps = 0;
    out.updates = 0;
    out.eqps = 0;
    out.moves = 0;
    out.picks = 0;
    ActiveSet<MM>& S = PS.S;
    const double fm = Dt.fmax;
    const int m = Dt.m;
    const bool use_gam = D::kGam && Dt.gamma > 0.0 && m > 0;

    // warm start: per contact, rows with positive ADMM dual, largest first,
    // kept while independent
    S.mask = 0;
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= m) continue;
        double yv[9];
#pragma unroll
        for (int kk = 0; kk < 9; ++kk) yv[kk] = double(y0[9 * i + kk]);
        unsigned mk = 0u, used = 0u;
#pragma unroll 1
        for (int pass = 0; pass < 3; ++pass) {
            // the largest remaining positive dual that is independent of the
            // rows taken so far
            ContactRows R;
            ContactProj P;
            contact_rows(mk, Dt.muc[i], fm, R);
            contact_proj(R, P);
            int best = -1;
            double by = 0.0;
#pragma unroll
            for (int kk = 0; kk < 9; ++kk) {
                double c[3], b;
                row3(kk, Dt.muc[i], fm, c, &b);
                const double nc = dot3(c, c);
                proj_apply(P, c);
                const bool indep = dot3(c, c) > 1e-12 * nc;
                if (!((used >> kk) & 1u) && indep && yv[kk] > by) {
                    by = yv[kk];
                    best = kk;
                }
            }
            if (best < 0) break;
            used |= 1u << best;
            mk |= 1u << best;
        }
        S.mask |= RowMask<MM>(mk) << (9 * i);
    }
    S.gam = false;
    if (use_gam && double(y0[9 * MM]) < 0.0) S.gam = sum_row_norm2(Dt, S) > 1e-12 * m;

    const PendingRow none = {-1, -1, {0.0, 0.0, 0.0}, 0.0};
    PS.p = none;
    PS.mp = none;
    PS.up = 0.0;
    PS.mup = 0.0;
    PS.lg = 0.0;
    PS.phase = kWarm;
    PS.mode = kEqp0;
    PS.refactor = true;
    PS.need_mult = false;
    // no rank-one changes with the normal-sum row (its term involves every contact)
    PS.chg = kNoChange | (D::kGam ? 0 : int(kChgAllowed));
    PS.step0 = 0;
    PS.budget = 0x7fffffff;
}

// Acceptance: stationarity, dual and primal feasibility.  Sets the status
// and returns true (the QP is finished).
template <int MM, typename D, class V>
BODEX_FI bool polish_accept(const D& Dt, const PolishWork<V>& W, PolishState<MM>& PS) {
    const ActiveSet<MM>& S = PS.S;
    PolishOut& out = PS.out;
    const double* lg = &PS.lg;
    const double fm = Dt.fmax;
    const int m = Dt.m;
    const bool use_gam = D::kGam && Dt.gamma > 0.0 && m > 0;
    const bool gam = D::kGam && S.gam;
    double r6[6];
    g_times<MM>(Dt, W.x, true, r6);
    double gs = 0.0, stat = 0.0, lneg = 0.0, lmax = 0.0, viol = 0.0, vin = 0.0, sum1 = 0.0;
    if (gam) {
        lneg = fmax(lneg, -*lg);
        lmax = fmax(lmax, fabs(*lg));
    }
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= m) continue;
        double g[3];
        contact_grad<MM>(Dt, i, r6, W.x, g);
        gs = fmax(gs, fmax(fabs(g[0]), fmax(fabs(g[1]), fabs(g[2]))));
        double st[3] = {g[0] - (gam ? *lg : 0.0), g[1], g[2]};
        ContactRows R;
        contact_rows(contact_mask(S.mask, i), Dt.muc[i], fm, R);
        double lam[3];
        contact_multipliers<MM>(Dt, R, W.x, r6, i, PendingRow{-1, -1, {0.0, 0.0, 0.0}, 0.0}, 0.0, *lg, lam);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j >= R.n) continue;
            const double l = lam[j];
#pragma unroll
            for (int t = 0; t < 3; ++t) st[t] += l * R.c[j][t];
            lneg = fmax(lneg, -l);
            lmax = fmax(lmax, fabs(l));
        }
        stat = fmax(stat, fmax(fabs(st[0]), fmax(fabs(st[1]), fabs(st[2]))));
        const double f[3] = {W.x[3 * i], W.x[3 * i + 1], W.x[3 * i + 2]};
        const unsigned mk = contact_mask(S.mask, i);
#pragma unroll
        for (int kk = 0; kk < 9; ++kk) {
            double c[3], b;
            row3(kk, Dt.muc[i], fm, c, &b);
            const double v = dot3(c, f) - b;
            viol = fmax(viol, v);
            if (!((mk >> kk) & 1u)) vin = fmax(vin, v);
        }
        sum1 += f[0];
    }
    if (use_gam) {
        viol = fmax(viol, Dt.gamma - sum1);
        if (!gam) vin = fmax(vin, Dt.gamma - sum1);
    }
    const bool kkt = stat <= 1e-9 * (1.0 + gs + lmax) && lneg <= 1e-9 * (1.0 + lmax) && isfinite(stat) &&
                     isfinite(gs);
    const double vb = 1e-9 * (1.0 + fm + Dt.gamma);
    // violated only outside the active set: more steps (see kPolishViolated)
    out.status = kkt && viol <= vb ? 0 : (kkt && vin > vb && viol == vin ? kPolishViolated : 1);
    return true;
}


// BUDGET: compile the check of PS.budget in (the chunked first pass).
template <int MM, typename D, class V, bool BUDGET = false>
BODEX_FI bool polish_advance(const D& Dt, int max_steps, const PolishWork<V>& W, PolishState<MM>& PS) {
    ActiveSet<MM>& S = PS.S;
    PolishOut& out = PS.out;
    double* lg = &PS.lg;
    PendingRow& p = PS.p;
    PendingRow& mp = PS.mp;
    double& up = PS.up;
    double& mup = PS.mup;
    int& phase = PS.phase;
    int& mode = PS.mode;
    bool& refactor = PS.refactor;
    bool& need_mult = PS.need_mult;
    const double fm = Dt.fmax;
    const int m = Dt.m;
    const bool use_gam = D::kGam && Dt.gamma > 0.0 && m > 0;
    const double tol_add = 1e-12 * (1.0 + fm + Dt.gamma);
    const PendingRow none = {-1, -1, {0.0, 0.0, 0.0}, 0.0};
    if (mode == kAccept) return true;
    if (refactor) {
        if (BUDGET && out.steps >= PS.budget) {
            out.status = kPolishSuspended;
            return true;
        }
        if (++out.steps - PS.step0 > max_steps) {
            out.status = 2;
            return true;
        }
        // the matrix of the new set from the old factor and the one-row
        // change when there is one, else (or if that does not factor) from
        // every contact; one Cholesky call site
        const int row = PS.chg & kNoChange;
        bool quick = (PS.chg & kChgAllowed) && row != kNoChange;
        bool ok = false;
#pragma unroll 1
        for (;;) {
            if (quick) {
                const int ci = row / 9;
                ok = matrix_row_change<MM>(Dt, S, ci, row - 9 * ci, (PS.chg & kChgJoin) ? -1.0 : 1.0);
            } else {
                ok = set_matrix<MM>(Dt, S);
            }
            ok = ok && chol6(S.L);
            if (ok || !quick) break;
            quick = false;
        }
        if (!ok) {
            out.status = 3;
            return true;
        }
        if (quick) {
            ++out.updates;
            PS.chg |= kChgUsed;
        }
        PS.chg = with_change(PS.chg, kNoChange, false);
        refactor = false;
    }
    if (need_mult) {
        // the normal-sum multiplier of the new point / set (the per-contact
        // multipliers are computed where they are used)
        *lg = 0.0;
        if (D::kGam && S.gam) {
            double r6[6];
            g_times<MM>(Dt, W.x, true, r6);
            *lg = sum_row_multiplier<MM>(Dt, S, W.x, r6, mp, mup);
        }
        need_mult = false;
    }
    if (mode == kCheck) {
        // after an equality solve: done (final re-solve), or in the warm
        // phase drop the most negative multiplier
        if (phase == kFinal) {
            mode = kAccept;
            return true;
        }
        if (phase == kWarm) {
            int wbit = -1;
            double wv = -1e-14;
            if (D::kGam && S.gam && *lg < wv) {
                wv = *lg;
                wbit = 9 * MM;
            }
            double r6[6];
            g_times<MM>(Dt, W.x, true, r6);
#pragma unroll 1
            for (int i = 0; i < MM; ++i) {
                if (i >= m) continue;
                ContactRows R;
                contact_rows(contact_mask(S.mask, i), Dt.muc[i], fm, R);
                double lam[3];
                contact_multipliers<MM>(Dt, R, W.x, r6, i, mp, mup, *lg, lam);
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (j < R.n && lam[j] < wv) {
                        wv = lam[j];
                        wbit = 9 * i + R.id[j];
                    }
                }
            }
            if (wbit >= 0) {
                if (D::kGam && wbit == 9 * MM) {
                    S.gam = false;
                } else {
                    S.mask &= ~(RowMask<MM>(1) << wbit);
                    PS.chg = with_change(PS.chg, wbit, false);
                }
                refactor = true;
                mode = kEqp0;
                return false;
            }
            phase = kSteps;
        }
        mode = kPick;
    }
    if (mode == kPick) {
        // next row to satisfy
        p = most_violated<MM>(Dt, S, W, use_gam, tol_add);
        ++out.picks;
        if (p.pk < 0) {
            if (phase != kFinal) {  // x is the minimiser on this set
                mode = kAccept;
                return true;
            }
            mode = kEqp0;  // after steps: re-solve exactly
        } else {
            phase = kSteps;
            up = 0.0;
            mode = kStep;
        }
    }
    const bool gam = D::kGam && S.gam;
    // the vector H is applied to: grad(x) (equality solve) or c_p (step)
    bool dep = false;
    double sp = -p.b;
    if (mode == kEqp0) {
        eqp_start<MM>(Dt, S, W);
        ++out.eqps;
    }
    if (mode != kStep) {
        double r6[6];
        g_times<MM>(Dt, W.x, true, r6);
#pragma unroll 1
        for (int i = 0; i < MM; ++i) {
            if (i >= m) continue;
            double g[3];
            contact_grad<MM>(Dt, i, r6, W.x, g);
#pragma unroll
            for (int t = 0; t < 3; ++t) W.z[3 * i + t] = g[t];
        }
    } else {
        // c_p into z; is it in the span of the active rows?
        double res2 = 0.0, cn2 = 0.0, uv = 0.0, uu = 0.0;
#pragma unroll 1
        for (int i = 0; i < MM; ++i) {
            if (i >= m) continue;
            const bool on = pending_on(p, i);
            double v[3] = {on ? p.c[0] : 0.0, on ? p.c[1] : 0.0, on ? p.c[2] : 0.0};
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                W.z[3 * i + t] = v[t];
                sp += v[t] * W.x[3 * i + t];
            }
            const ContactProj P = cached_proj(Dt, S, i);
            cn2 += dot3(v, v);
            proj_apply(P, v);
            res2 += dot3(v, v);
            if (gam) {
                double u[3];
                sum_row_complement(P, u);
                uv += dot3(u, v);
                uu += dot3(u, u);
            }
        }
        if (gam) res2 -= uv * uv / uu;
        dep = !(res2 > 1e-12 * cn2);
    }
    if (dep) {
#pragma unroll 1
        for (int i = 0; i < MM; ++i) {
            if (i >= m) continue;
#pragma unroll
            for (int t = 0; t < 3; ++t) W.z[3 * i + t] = 0.0;
        }
    } else {
        apply_h<MM>(Dt, S, W.z);
    }

    if (mode != kStep) {
        // equality solve pass: x <- x - H grad(x)
#pragma unroll 1
        for (int i = 0; i < MM; ++i) {
            if (i >= m) continue;
#pragma unroll
            for (int t = 0; t < 3; ++t) W.x[3 * i + t] -= W.z[3 * i + t];
        }
        if (mode == kEqp0) {
            mode = kEqp1;
        } else {
            mp = none;
            mup = 0.0;
            need_mult = true;
            mode = kCheck;
        }
        return false;
    }
    // one-row step: w = c_p - P z over the active rows (r per contact,
    // rg for the normal-sum row); the largest step keeping the
    // multipliers nonnegative (t1) against the step that satisfies p (t2)
    ++out.moves;
    double cz = 0.0;
    double gz[6];
    g_times<MM>(Dt, W.z, false, gz);
    double rg = 0.0;
    if (gam) {
        double num = 0.0, den = 0.0;
#pragma unroll 1
        for (int i = 0; i < MM; ++i) {
            if (i >= m) continue;
            double w[3], u[3];
            contact_grad<MM>(Dt, i, gz, W.z, w);
            const bool on = pending_on(p, i);
#pragma unroll
            for (int t = 0; t < 3; ++t) w[t] = (on ? p.c[t] : 0.0) - w[t];
            sum_row_complement(cached_proj(Dt, S, i), u);
            num += dot3(u, w);
            den += dot3(u, u);
        }
        rg = num / den;
    }
    // the smallest ratio lam_j / r_j over r_j > 0, kept as a fraction tn / td
    // (compared by cross-multiplication, one division at the end)
    double tn = INFINITY, td = 1.0;
    int lbit = -1;
    if (gam && rg > 0.0) {
        tn = *lg;
        td = rg;
        lbit = 9 * MM;
    }
    double r6x[6];
    g_times<MM>(Dt, W.x, true, r6x);
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= m) continue;
        const bool on = pending_on(p, i);
        if (on) cz += p.c[0] * W.z[3 * i] + p.c[1] * W.z[3 * i + 1] + p.c[2] * W.z[3 * i + 2];
        ContactRows R;
        contact_rows(contact_mask(S.mask, i), Dt.muc[i], fm, R);
        double w[3], r[3], lam[3];
        contact_grad<MM>(Dt, i, gz, W.z, w);
#pragma unroll
        for (int t = 0; t < 3; ++t) w[t] = (on ? p.c[t] : 0.0) - w[t];
        w[0] += rg;
        double h[3];
        multiplier_rhs<MM>(Dt, W.x, r6x, i, mp, mup, *lg, h);
        rows_coeffs2(R, w, h, r, lam);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j < R.n && r[j] > 0.0 && lam[j] * td < tn * r[j]) {
                tn = lam[j];
                td = r[j];
                lbit = 9 * i + R.id[j];
            }
        }
    }
    const double t1 = tn / td;
    const double t2 = (dep || !(cz > 0.0)) ? INFINITY : sp / cz;
    const double st = t2 < t1 ? t2 : t1;
    if (!(st < INFINITY) || !(st >= 0.0) || ((PS.chg & kChgBreak) && (PS.chg & kChgUsed)) ||
        (PS.chg & kChgBreakAny)) {
        PS.chg &= ~int(kChgBreak | kChgBreakAny);
        out.status = 3;  // infeasible or broken down
        return true;
    }
#pragma unroll 1
    for (int i = 0; i < MM; ++i) {
        if (i >= m) continue;
#pragma unroll
        for (int t = 0; t < 3; ++t) W.x[3 * i + t] -= st * W.z[3 * i + t];
    }
    up += st;
    refactor = true;
    need_mult = true;
    if (t2 <= t1) {
        // p joins the active set; an exact re-solve follows the last step
        if (p.pk == 9) {
            S.gam = true;
        } else {
            S.mask |= RowMask<MM>(1) << (9 * p.pi + p.pk);
            PS.chg = with_change(PS.chg, 9 * p.pi + p.pk, true);
        }
        phase = kFinal;
        mp = none;
        mup = 0.0;
        mode = kPick;
    } else {
        // drop the row whose multiplier reached zero, continue with p
        if (D::kGam && lbit == 9 * MM) {
            S.gam = false;
        } else {
            S.mask &= ~(RowMask<MM>(1) << lbit);
            PS.chg = with_change(PS.chg, lbit, false);
        }
        mp = p;
        mup = up;
        mode = kStep;
    }
    return false;
}

// After polish_advance has returned true: the acceptance check of a QP
// that reached it (others keep their failure status).  Returns false when
// the QP is to be taken once more: failed after one-row changes of the
// factor (rejected by the check, out of steps, or broken down in the ratio
// test), it restarts from its last set with fresh factorisations only
// (equality solve, multiplier drops, steps) and a step cap of its own.  If
// it fails without such changes, or again after that restart, it is taken
// once from the empty active set: the unconstrained minimiser, from which
// the dual active-set steps are the textbook method (its infeasibility test
// is then sound), again with fresh factorisations and a cap of its own.
// This happens for about one QP in 1e9 (a warm set whose first step finds
// the violated row dependent on the active rows with no multiplier to drop).
template <int MM, typename D, class V>
BODEX_FI bool polish_finish(const D& Dt, const PolishWork<V>& W, PolishState<MM>& PS) {
    if (PS.out.status == kPolishSuspended) return true;
    const bool reached = PS.mode == kAccept;
    if (reached) polish_accept<MM>(Dt, W, PS);
    if (PS.out.status == kPolishViolated) {
        PS.out.status = 0;
        PS.phase = kSteps;
        PS.mode = kPick;
        return false;
    }
    const bool forced = reached && (PS.chg & kChgRetry);
    if ((PS.out.status != 0 || forced) && (PS.chg & kChgUsed)) {
        PS.out.status = 0;
        PS.chg = kNoChange | (PS.chg & kChgCold);
        PS.step0 = PS.out.steps;
        PS.refactor = true;
        PS.phase = kWarm;
        PS.mode = kEqp0;
        return false;
    }
    if (PS.out.status != 0 && !(PS.chg & kChgCold)) {
        const PendingRow none = {-1, -1, {0.0, 0.0, 0.0}, 0.0};
        PS.out.status = 0;
        PS.chg = kNoChange | kChgCold;
        PS.step0 = PS.out.steps;
        PS.S.mask = 0;
        PS.S.gam = false;
        PS.p = none;
        PS.mp = none;
        PS.up = 0.0;
        PS.mup = 0.0;
        PS.lg = 0.0;
        PS.need_mult = false;
        PS.refactor = true;
        PS.phase = kWarm;
        PS.mode = kEqp0;
        return false;
    }
    return true;
}

// The whole polish of one QP (see polish_begin / polish_advance /
// polish_finish).  The acceptance check sits after the stepping loop, so
// the lanes of a wave, which reach it at different times, run it together
// once instead of once per lane.
template <int MM, typename YP, typename D, class V>
BODEX_FI PolishOut polish_qp(const D& Dt, YP y0, int max_steps, const PolishWork<V>& W, PolishState<MM>& PS) {
    polish_begin<MM>(Dt, y0, PS);
#pragma unroll 1
    do {
#pragma unroll 1
        while (!polish_advance<MM>(Dt, max_steps, W, PS)) {
        }
    } while (!polish_finish<MM>(Dt, W, PS));
    return PS.out;
}

// Relative KKT residual (same definition as the ADMM check) of a state
// (x, z, y), evaluated in FP64.  x(c), z(r), y(r): accessors of the force
// entries and of the contact rows r = 9i+kk; zg, yg: the normal-sum row;
// bt = beta t.  Contacts are visited in a loop (no per-lane arrays).
template <int MM, typename GP, typename XA, typename ZA, typename YA>
BODEX_FI double rel_kkt64(GP G, const double* muc, const double* bt, int m, double eps, XA x, ZA z, YA y,
                          double zg, double yg) {
    constexpr int NV = 3 * MM;
    double gx[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) gx[k] = 0.0;
#pragma unroll 1
    for (int c = 0; c < 3 * m; ++c) {
        const double xc = x(c);
#pragma unroll
        for (int k = 0; k < 6; ++k) gx[k] += G[k * NV + c] * xc;
    }
    double rp = 0, nAx = 0, nz = 0, rd = 0, nPx = 0, nAty = 0, nq = 0, s1 = 0.0;
#pragma unroll 1
    for (int i = 0; i < m; ++i) {
        const double x1 = x(3 * i), x2 = x(3 * i + 1), x3 = x(3 * i + 2);
        double aty[3] = {yg, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double ck = facet_cos<double>(k), sk = facet_sin<double>(k);
            const double ax = ck * x2 + sk * x3 - muc[i] * x1;
            const double zk = z(9 * i + k), yk = y(9 * i + k);
            rp = fmax(rp, fabs(ax - zk));
            nAx = fmax(nAx, fabs(ax));
            nz = fmax(nz, fabs(zk));
            aty[0] -= muc[i] * yk;
            aty[1] += ck * yk;
            aty[2] += sk * yk;
        }
        const double zb = z(9 * i + 8);
        aty[0] += y(9 * i + 8);
        rp = fmax(rp, fabs(x1 - zb));
        nAx = fmax(nAx, fabs(x1));
        nz = fmax(nz, fabs(zb));
        s1 += x1;
        const double xi[3] = {x1, x2, x3};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            double s = eps * xi[t], qc = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                s += G[k * NV + 3 * i + t] * gx[k];
                qc += G[k * NV + 3 * i + t] * bt[k];
            }
            const double px = 2.0 * s;
            qc *= -2.0;
            rd = fmax(rd, fabs(px + qc + aty[t]));
            nPx = fmax(nPx, fabs(px));
            nAty = fmax(nAty, fabs(aty[t]));
            nq = fmax(nq, fabs(qc));
        }
    }
    rp = fmax(rp, fabs(s1 - zg));
    nAx = fmax(nAx, fabs(s1));
    nz = fmax(nz, fabs(zg));
    return fmax(rp / (1.0 + fmax(nAx, nz)), rd / (1.0 + fmax(fmax(nPx, nAty), nq)));
}

}  // namespace bodex
