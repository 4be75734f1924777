// bodex_cone.h -- the contact-force QP with the exact circular friction cone
// of Eq. 1 (arXiv 2412.16490, Sec. III) in place of the 8-facet pyramid of
// Sec. IV-A: per contact |(f_2, f_3)| <= mu f_1 and f_1 <= fmax, plus the
// normal-sum row of Eq. 9.
//
// ADMM form: A = [I_{3m}; s^T] (s sums the normal components), so the state
// has 3 MM + 1 rows: rows 3i..3i+2 contact i's force, row 3 MM the
// normal-sum row.  The projection onto the constraint set is per contact
// onto the truncated cone (closed form, below) and a clamp for the sum row.
// The FP64 polish is a primal log-barrier method warm-started from the ADMM
// point: per barrier weight t, damped Newton steps on t Q(f) + phi(f) with
// phi = -sum_i log(mu_i^2 f_i1^2 - |f_it|^2) - sum_i log(fmax - f_i1)
// [- log(sum_i f_i1 - gamma)], each solving the dense 3m x 3m system
// t 2 (G^T G + eps I) + Hess(phi) (scaled symmetrically by its diagonal, then
// Cholesky), until the duality-gap bound nu / t is below the target.
#pragma once

#include "bodex_math.h"

namespace bodex {

// ---------------------------------------------------------------------------
// Projection onto the truncated cone C = {|t| <= mu a, a <= fmax} of a point
// (a, t) (a the normal component, t the two tangential ones).  C is
// rotationally symmetric, so the projection stays in the half-plane of
// (a, r = |t|) and is the closest point of the triangle (0, 0), (fmax, 0),
// (fmax, mu fmax): the apex when a + mu r <= 0 (the polar cone), the cone
// line at tau = (a + mu r) / (1 + mu^2) when r > mu a (capped at the rim),
// else the normal bound a <= fmax with r capped at the rim.
// ---------------------------------------------------------------------------
enum ConeRegion { kFree = 0, kSurface = 1, kApex = 2, kBound = 3, kRim = 4 };

template <typename T>
BODEX_FI int cone_project(T a, T t2, T t3, T mu, T fmax, T* z) {
    const T r = sqrt(t2 * t2 + t3 * t3);
    const bool apex = a + mu * r <= T(0);
    const bool above = r > mu * a;
    const T tau = (a + mu * r) / (T(1) + mu * mu);
    T na = above ? fmin(tau, fmax) : fmin(a, fmax);
    T nr = above ? mu * na : fmin(r, mu * fmax);
    na = apex ? T(0) : na;
    nr = apex ? T(0) : nr;
    const T s = r > T(0) ? nr / r : T(0);
    z[0] = na;
    z[1] = t2 * s;
    z[2] = t3 * s;
    const bool top = above ? !(tau < fmax) : (a > fmax);
    const bool rim = top && (above || r > mu * fmax);
    return apex ? kApex : (rim ? kRim : (top ? kBound : (above ? kSurface : kFree)));
}

// ---------------------------------------------------------------------------
// ADMM in the reduced state w (see the pyramid form in bodex_math.h): with
// p = Pi(w), one iteration is
//     x~ = K^{-1} (rho A^T (2p - w) + bq),   w <- w + alpha (A x~ - p),
// where K = P + rho A^T A and A^T A = I + (normal-sum outer product).
// ---------------------------------------------------------------------------
template <int MM>
BODEX_FI void cone_proj_all(const float* w, const float* mu, float fmax, float gamma, float* p) {
#pragma unroll
    for (int i = 0; i < MM; ++i) cone_project<float>(w[3 * i], w[3 * i + 1], w[3 * i + 2], mu[i], fmax, p + 3 * i);
    p[3 * MM] = fmaxf(w[3 * MM], gamma);
}

template <int MM, typename BQ, typename MU>
BODEX_FI void cone_rhs(const float* w, BQ bq, MU mu, float rho, float fmax, float gamma, int m, float* p,
                       float* rhs) {
    float muv[MM];
#pragma unroll
    for (int i = 0; i < MM; ++i) muv[i] = mu[i];
    cone_proj_all<MM>(w, muv, fmax, gamma, p);
    const float vg = 2.f * p[3 * MM] - w[3 * MM];
#pragma unroll
    for (int c = 0; c < 3 * MM; ++c) {
        float v = 2.f * p[c] - w[c];
        if (c % 3 == 0 && c / 3 < m) v += vg;
        rhs[c] = fmaf(rho, v, bq[c]);
    }
}

template <int MM>
BODEX_FI void cone_update(float* w, const float* x, const float* p, float alpha, int m) {
    float s1 = 0.f;
#pragma unroll
    for (int c = 0; c < 3 * MM; ++c) {
        w[c] = fmaf(alpha, x[c] - p[c], w[c]);
        if (c % 3 == 0 && c / 3 < m) s1 += x[c];
    }
    w[3 * MM] = fmaf(alpha, s1 - p[3 * MM], w[3 * MM]);
}

// Residuals of (x, z = Pi(w), y = rho (w - Pi(w))), same definitions as the
// pyramid form.
template <int MM, typename BQ, typename MU, typename GPtr>
BODEX_FI Residual cone_residual(const float* w, const float* x, BQ bq, MU mu, GPtr G, float rho, float eps,
                                float fmax, float gamma, int m) {
    constexpr int NV = 3 * MM;
    float muv[MM], z[NV + 1];
#pragma unroll
    for (int i = 0; i < MM; ++i) muv[i] = mu[i];
    cone_proj_all<MM>(w, muv, fmax, gamma, z);
    const float yg = rho * (w[NV] - z[NV]);
    float rp = 0.f, nAx = 0.f, nz = 0.f, s1 = 0.f;
    float aty[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        rp = fmaxf(rp, fabsf(x[c] - z[c]));
        nAx = fmaxf(nAx, fabsf(x[c]));
        nz = fmaxf(nz, fabsf(z[c]));
        const bool nrm = (c % 3 == 0) && (c / 3 < m);
        aty[c] = rho * (w[c] - z[c]) + (nrm ? yg : 0.f);
        s1 += nrm ? x[c] : 0.f;
    }
    rp = fmaxf(rp, fabsf(s1 - z[NV]));
    nAx = fmaxf(nAx, fabsf(s1));
    nz = fmaxf(nz, fabsf(z[NV]));
    float gx[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < NV; ++c) s = fmaf(G[a * NV + c], x[c], s);
        gx[a] = s;
    }
    float rd = 0.f, nPx = 0.f, nAty = 0.f, nq = 0.f;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
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

// Entry (i, j) of K = 2 (G^T G + eps I) + rho (I + s s^T) for the cone form;
// padded contacts get an identity block.
template <typename T, int NV>
BODEX_FI T cone_kkt_entry(const T* G, int m, T rho, T eps, int i, int j) {
    const int ci = i / 3, cj = j / 3;
    if (ci >= m || cj >= m) return (i == j) ? T(1) : T(0);
    T s = T(0);
    for (int a = 0; a < 6; ++a) s += G[a * NV + i] * G[a * NV + j];
    T v = T(2) * s;
    if (i == j) v += T(2) * eps + rho;
    if (i % 3 == 0 && j % 3 == 0) v += rho;
    return v;
}

// lambda_max <= 2 ||G||_F^2 + 2 eps + rho (1 + m), lambda_min >= 2 eps + rho.
template <typename T, int NV>
BODEX_FI T cone_kkt_cond_bound(const T* G, int m, T rho, T eps) {
    T gf = T(0);
    for (int a = 0; a < 6 * NV; ++a) gf += G[a] * G[a];
    return (T(2) * gf + T(2) * eps + rho * T(1 + m)) / (T(2) * eps + rho);
}

// Relative KKT residual (FP64) of a cone-form state: x(c), z(r), y(r) for
// r < 3 m, zg, yg the normal-sum row; bt = beta t.
template <int MM, typename GP, typename XA, typename ZA, typename YA>
BODEX_FI double cone_rel_kkt64(GP G, const double* bt, int m, double eps, XA x, ZA z, YA y, double zg, double yg) {
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
    for (int c = 0; c < 3 * m; ++c) {
        const double xc = x(c), zc = z(c);
        rp = fmax(rp, fabs(xc - zc));
        nAx = fmax(nAx, fabs(xc));
        nz = fmax(nz, fabs(zc));
        const double aty = y(c) + ((c % 3 == 0) ? yg : 0.0);
        if (c % 3 == 0) s1 += xc;
        double s = eps * xc, qc = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            s += G[k * NV + c] * gx[k];
            qc += G[k * NV + c] * bt[k];
        }
        const double px = 2.0 * s;
        qc *= -2.0;
        rd = fmax(rd, fabs(px + qc + aty));
        nPx = fmax(nPx, fabs(px));
        nAty = fmax(nAty, fabs(aty));
        nq = fmax(nq, fabs(qc));
    }
    rp = fmax(rp, fabs(s1 - zg));
    nAx = fmax(nAx, fabs(s1));
    nz = fmax(nz, fabs(zg));
    return fmax(rp / (1.0 + fmax(nAx, nz)), rd / (1.0 + fmax(fmax(nPx, nAty), nq)));
}

// ---------------------------------------------------------------------------
// FP64 polish for the cone form: the barrier method (Boyd & Vandenberghe,
// Convex Optimization, Sec. 11.3) warm-started from the ADMM point.  For a
// barrier weight t it minimises t Q(f) + phi(f) with
//   phi = - sum_i log(mu_i^2 f_i1^2 - |f_it|^2) - sum_i log(fmax - f_i1)
//         - log(sum_i f_i1 - gamma)                 (the last with gamma > 0)
// by Newton's method with a backtracking line search that keeps f strictly
// feasible, for t growing geometrically until nu / t (nu = 3 m + [gamma > 0],
// the barrier's parameter) is below the target gap.  The Newton matrix
// t P + grad^2 phi = 2 t G^T G + blockdiag(B_i) (+ the normal-sum row's
// rank-one term), B_i = 2 t eps I + the contact's barrier Hessian, is
// factored densely (3 m x 3 m Cholesky in registers) after symmetric
// diagonal scaling: near the constraint boundaries its diagonal spans up to
// 1e20, which a structured (Woodbury) inverse through the 6x6 range of G
// does not survive, while the scaled Cholesky stays backward stable.
// ---------------------------------------------------------------------------

template <int MM, typename GP, bool GAM>
struct ConeData {
    static constexpr int kMM = MM;
    static constexpr bool kGam = GAM;
    GP G;
    const double* mu;
    double bt[6];
    int m;
    double fmax, gamma, eps;
};

// r6 = G v - (with_t ? beta t : 0) and contact i's part of 2 (G^T r6 + eps v).
template <int MM, typename D, class V>
BODEX_FI void cone_g_times(const D& Dt, const V& v, bool with_t, double* r6) {
    constexpr int NV = 3 * MM;
    for (int k = 0; k < 6; ++k) r6[k] = with_t ? -Dt.bt[k] : 0.0;
#pragma unroll 1
    for (int i = 0; i < Dt.m; ++i)
        for (int t = 0; t < 3; ++t) {
            const double vc = v[3 * i + t];
            for (int k = 0; k < 6; ++k) r6[k] += Dt.G[k * NV + 3 * i + t] * vc;
        }
}

template <int MM, typename D, class V>
BODEX_FI void cone_contact_grad(const D& Dt, int i, const double* r6, const V& v, double* g) {
    constexpr int NV = 3 * MM;
    for (int t = 0; t < 3; ++t) {
        double s = Dt.eps * v[3 * i + t];
        for (int k = 0; k < 6; ++k) s += Dt.G[k * NV + 3 * i + t] * r6[k];
        g[t] = 2.0 * s;
    }
}

// Slacks of contact i with x0 = mu f_1, r = |f_t|: dm = x0 - r, dp = x0 + r
// (the cone's s = mu^2 f_1^2 - |f_t|^2 = dm dp, formed as a product to keep
// its relative accuracy near the surface) and the bound's b = fmax - f_1;
// false unless all are positive.
BODEX_FI bool cone_slacks(const double* f, double mu, double fmax, double* dm, double* dp, double* b) {
    const double r = sqrt(f[1] * f[1] + f[2] * f[2]);
    *dm = mu * f[0] - r;
    *dp = mu * f[0] + r;
    *b = fmax - f[0];
    return *dm > 0.0 && *b > 0.0;
}

// Contact i's barrier Hessian plus e I (e = 2 t eps), packed lower 3x3;
// false when f is not strictly inside.  With x = (mu f_1, f_t),
// J = diag(1, -1, -1), the cone term -log(x^T J x) has the Hessian
// 4 (Jx)(Jx)^T / s^2 - 2 J / s, which in the frame (axis, radial t,
// tangent t_perp) is the sum of positive terms
//   2 / dp^2 v+ v+^T + 2 / dm^2 v- v-^T + 2 / s t_perp t_perp^T,
// v+- = (e_axis +- e_radial) / sqrt 2, mapped to f by diag(mu, 1, 1): the
// entries are formed from these terms, so no large terms cancel near the
// surface.  The bound adds 1 / b^2 on the normal component.
BODEX_FI bool cone_block(const double* f, double mu, double fmax, double e, double* B) {
    double dm, dp, b;
    if (!cone_slacks(f, mu, fmax, &dm, &dp, &b)) return false;
    const double r = sqrt(f[1] * f[1] + f[2] * f[2]);
    const double t0 = r > 0.0 ? f[1] / r : 1.0, t1 = r > 0.0 ? f[2] / r : 0.0;
    const double h = 0.70710678118654752440;
    const double ap[3] = {h * mu, h * t0, h * t1}, am[3] = {h * mu, -h * t0, -h * t1}, tp[3] = {0.0, -t1, t0};
    const double cp = 2.0 / (dp * dp), cm = 2.0 / (dm * dm), cc = 2.0 / (dm * dp);
#pragma unroll
    for (int r2 = 0; r2 < 3; ++r2)
#pragma unroll
        for (int c = 0; c <= r2; ++c)
            B[lo_idx(r2, c)] = cp * ap[r2] * ap[c] + cm * am[r2] * am[c] + cc * tp[r2] * tp[c] + ((r2 == c) ? e : 0.0);
    B[0] += 1.0 / (b * b);
    return true;
}

// The polish's per-lane vectors: the point f, the Newton step d, the
// negated gradient ft, the trial point r.
template <class V>
struct ConeWork {
    V f, d, ft, r;
    // every vector must be given (no default-constructed members)
    BODEX_FI ConeWork(V f_, V d_, V ft_, V r_) : f(f_), d(d_), ft(ft_), r(r_) {}
};

// Barrier merit t Q(f) + phi(f) (INFINITY outside) and, when grad is set,
// its gradient into W.d (negated: the Newton right-hand side).
template <int MM, typename D, class V>
BODEX_FI double cone_merit(const D& Dt, const V& f, double t, const V* rhs, double* qout) {
    double r6[6], ff = 0.0;
    cone_g_times<MM>(Dt, f, true, r6);
    // phi = -log of the product of all slacks (one logarithm; the product
    // of at most 3 MM + 1 slacks in (0, fmax] stays in range)
    double prod = 1.0, s1 = 0.0;
#pragma unroll 1
    for (int i = 0; i < Dt.m; ++i) {
        const double fi[3] = {f[3 * i], f[3 * i + 1], f[3 * i + 2]};
        double dm, dp, b;
        if (!cone_slacks(fi, Dt.mu[i], Dt.fmax, &dm, &dp, &b)) return INFINITY;
        prod *= dm * dp * b;
        s1 += fi[0];
        ff += dot3(fi, fi);
    }
    const bool gam = D::kGam && Dt.gamma > 0.0;
    const double sg = s1 - Dt.gamma;
    if (gam) {
        if (!(sg > 0.0)) return INFINITY;
        prod *= sg;
    }
    const double phi = -log(prod);
    double rr = 0.0;
    for (int k = 0; k < 6; ++k) rr += r6[k] * r6[k];
    const double q = rr + Dt.eps * ff;
    if (qout) *qout = q;
    if (rhs) {
#pragma unroll 1
        for (int i = 0; i < Dt.m; ++i) {
            const double fi[3] = {f[3 * i], f[3 * i + 1], f[3 * i + 2]};
            double g[3], dm, dp, b;
            cone_contact_grad<MM>(Dt, i, r6, f, g);
            cone_slacks(fi, Dt.mu[i], Dt.fmax, &dm, &dp, &b);
            const double s = dm * dp;
            const double ds[3] = {2.0 * Dt.mu[i] * Dt.mu[i] * fi[0], -2.0 * fi[1], -2.0 * fi[2]};
            for (int j = 0; j < 3; ++j) {
                double v = t * g[j] - ds[j] / s;
                if (j == 0) v += 1.0 / b - (gam ? 1.0 / sg : 0.0);
                (*rhs)[3 * i + j] = -v;
            }
        }
    }
    return t * q + phi;
}

// In place: v <- A^{-1} v for the Newton matrix at f, weight t:
// A = 2 t (G^T G + eps I) + blockdiag(barrier Hessians) (+ iu^2 s s^T with
// the normal-sum row, s the normal-component pattern, iu = 1 / (sum f_1 -
// gamma)).  Dense: formed in registers with compile-time indices, scaled to
// unit diagonal, Cholesky-factored; padded contacts get identity rows.  The
// scale factors go to the lane's vector sc (free during the solve) and the
// substitutions run in v, so that only the matrix occupies registers.
// Returns false on a non-positive pivot.
template <int MM, typename D, class V>
BODEX_FI bool cone_newton_solve(const D& Dt, const V& f, double t, double iu, const V& v, const V& sc) {
    constexpr int NV = 3 * MM, NK = NV * (NV + 1) / 2;
    const int m = Dt.m;
    // 2 t G^T G, one row of G at a time (few values live besides the matrix)
    double a[NK];
#pragma unroll
    for (int e = 0; e < NK; ++e) a[e] = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double gk[NV];
#pragma unroll
        for (int r = 0; r < NV; ++r) gk[r] = Dt.G[k * NV + r];
#pragma unroll
        for (int r = 0; r < NV; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) a[lo_idx(r, c)] += gk[r] * gk[c];
    }
#pragma unroll
    for (int e = 0; e < NK; ++e) a[e] *= 2.0 * t;
    // the normal-sum row's rank-one term, then per contact its block (padded
    // contacts: identity rows)
#pragma unroll
    for (int r = 0; r < NV; r += 3)
#pragma unroll
        for (int c = 0; c <= r; c += 3) a[lo_idx(r, c)] += iu * iu;
#pragma unroll
    for (int i = 0; i < MM; ++i) {
        double fi[3] = {0.5 * Dt.fmax, 0.0, 0.0};
        if (i < m) {
            fi[0] = f[3 * i];
            fi[1] = f[3 * i + 1];
            fi[2] = f[3 * i + 2];
        }
        double blk[6];
        if (!cone_block(fi, Dt.mu[i < m ? i : 0], Dt.fmax, 2.0 * t * Dt.eps, blk)) return false;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) a[lo_idx(3 * i + r, 3 * i + c)] += blk[lo_idx(r, c)];
    }
#pragma unroll
    for (int r = 0; r < NV; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c)
            if (r / 3 >= m || c / 3 >= m) a[lo_idx(r, c)] = (r == c) ? 1.0 : 0.0;
    // the scale factors and the solution in the lane's vectors sc and v
#pragma unroll
    for (int r = 0; r < NV; ++r) {
        const double sr = 1.0 / sqrt(a[lo_idx(r, r)]);
        sc[r] = sr;
        v[r] = (r < 3 * m) ? double(v[r]) * sr : 0.0;
    }
#pragma unroll
    for (int r = 0; r < NV; ++r) {
        const double sr = sc[r];
#pragma unroll
        for (int c = 0; c <= r; ++c) a[lo_idx(r, c)] *= sr * sc[c];
    }
    // Cholesky (reciprocal pivots on the diagonal)
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double dj = a[lo_idx(j, j)];
#pragma unroll
        for (int l = 0; l < j; ++l) dj -= a[lo_idx(j, l)] * a[lo_idx(j, l)];
        if (!(dj > 0.0)) return false;
        const double id = 1.0 / sqrt(dj);
#pragma unroll
        for (int i = j + 1; i < NV; ++i) {
            double sv = a[lo_idx(i, j)];
#pragma unroll
            for (int l = 0; l < j; ++l) sv -= a[lo_idx(i, l)] * a[lo_idx(j, l)];
            a[lo_idx(i, j)] = sv * id;
        }
        a[lo_idx(j, j)] = id;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double sv = v[i];
#pragma unroll
        for (int l = 0; l < i; ++l) sv -= a[lo_idx(i, l)] * v[l];
        v[i] = sv * a[lo_idx(i, i)];
    }
#pragma unroll
    for (int i = NV - 1; i >= 0; --i) {
        double sv = v[i];
#pragma unroll
        for (int l = i + 1; l < NV; ++l) sv -= a[lo_idx(l, i)] * v[l];
        v[i] = sv * a[lo_idx(i, i)];
    }
#pragma unroll
    for (int r = 0; r < NV; ++r)
        if (r < 3 * m) v[r] = v[r] * sc[r];
    return true;
}

struct ConePolishOut {
    int status;  // 0 accepted (nu / t reached the gap), 2 iteration cap, 3 breakdown
    int newton;  // Newton steps (one factorisation each)
    int evals;   // line-search trial points
    int grads;   // merit evaluations with the gradient
    double t;    // final barrier weight
    double q;    // objective at the final point
};

// Algorithmic FP64 flops of one cone polish (FMA = 2, other operations 1),
// counted from the arithmetic of each routine at m contacts, n = 3 m:
//   Newton step        forming the matrix 6 n (n + 1) (G^T G entries) +
//                      n (n + 1) (scaling) + 40 m (barrier blocks), Cholesky
//                      2 n^3 / 3 + 2 n, two triangular solves 2 n^2 + 3 n
//   line-search trial  100 m + 15   (trial point, G f, slacks, one logarithm)
//   merit and gradient 140 m + 20
BODEX_FI double cone_polish_flops(int m, const ConePolishOut& o) {
    const double dm = m, n = 3.0 * m;
    const double step = 6.0 * n * (n + 1.0) + n * (n + 1.0) + 40.0 * dm + 2.0 * n * n * n / 3.0 + 2.0 * n + 2.0 * n * n +
                        3.0 * n;
    return o.newton * step + o.evals * (100.0 * dm + 15.0) + o.grads * (140.0 * dm + 20.0);
}

// Strictly feasible start near the ADMM point z (rows 3i..3i+2): each
// contact moved a fraction `pull` toward (c0, 0, 0), c0 inside (0, fmax);
// with gamma > 0 further toward (fmax, 0, 0) until sum f_1 exceeds gamma.
template <int MM, typename D, class V, typename ZA>
BODEX_FI void cone_start(const D& Dt, ZA z, double pull, const ConeWork<V>& W) {
    const double fm = Dt.fmax;
    double s1 = 0.0;
#pragma unroll 1
    for (int i = 0; i < Dt.m; ++i) {
        double p[3];
        cone_project<double>(double(z(3 * i)), double(z(3 * i + 1)), double(z(3 * i + 2)), Dt.mu[i], fm, p);
        const double c0 = 0.5 * fm;
        W.f[3 * i] = (1.0 - pull) * p[0] + pull * c0;
        W.f[3 * i + 1] = (1.0 - pull) * p[1];
        W.f[3 * i + 2] = (1.0 - pull) * p[2];
        s1 += W.f[3 * i];
    }
    if (D::kGam && Dt.gamma > 0.0) {
        const double target = Dt.gamma + 0.5 * (Dt.m * fm - Dt.gamma) * pull;
        if (s1 < target) {
            // toward (fm (1 - pull / 2), 0, 0), strictly inside every cone
            const double top = fm * (1.0 - 0.5 * pull);
            const double tau = (target - s1) / (Dt.m * top - s1);
#pragma unroll 1
            for (int i = 0; i < Dt.m; ++i) {
                W.f[3 * i] += tau * (top - W.f[3 * i]);
                W.f[3 * i + 1] *= 1.0 - tau;
                W.f[3 * i + 2] *= 1.0 - tau;
            }
        }
    }
}

// The barrier iteration from W.f (strictly feasible) until nu / t <= gap,
// starting at the weight where W.f is closest to central (at most t0).  On
// return W.f is the point.
template <int MM, typename D, class V>
BODEX_FI ConePolishOut cone_polish(const D& Dt, double t0, double gap, double growth, double loose, int max_newton,
                                   const ConeWork<V>& W) {
    const bool gam = D::kGam && Dt.gamma > 0.0;
    const double nu = 2.0 * Dt.m + Dt.m + (gam ? 1.0 : 0.0);
    ConePolishOut out = {2, 0, 0, 2, t0, 0.0};
    double qv = 0.0;
    // starting weight: the t at which the start is closest to central,
    // t = -(grad Q . grad phi) / |grad Q|^2 (the merit's gradient at weight t
    // is t grad Q + grad phi), clamped to [1, t0]
    double t = 1.0;
    {
        // -grad at weights 0 and 1 give -grad phi and -(grad Q + grad phi)
        // (one call site for both)
#pragma unroll 1
        for (int k = 0; k < 2; ++k) {
            const double mv = cone_merit<MM>(Dt, W.f, double(k), k ? &W.r : &W.d, &qv);
            if (k == 0 && !isfinite(mv)) {
                out.status = 3;
                return out;
            }
        }
        double gh = 0.0, gg = 0.0;
#pragma unroll 1
        for (int c = 0; c < 3 * Dt.m; ++c) {
            const double gq = W.d[c] - W.r[c];  // grad Q
            gh += gq * (-W.d[c]);               // grad Q . grad phi
            gg += gq * gq;
        }
        if (gg > 0.0 && -gh > gg) t = fmin(-gh / gg, t0);
    }
    double val = 0.0;
    // every pass starts from the merit and -grad at (f, t) (one call site):
    // at the start, after an accepted line search and after raising t
#pragma unroll 1
    for (;;) {
        val = cone_merit<MM>(Dt, W.f, t, &W.d, &qv);
        if (!(out.newton < max_newton)) break;
        ++out.newton;
        // d = A^{-1} (-grad) (the normal-sum row's barrier term iu^2 s s^T is
        // part of A)
        double iu = 0.0;
        if (gam) {
            double s1 = 0.0;
#pragma unroll 1
            for (int i = 0; i < Dt.m; ++i) s1 += W.f[3 * i];
            iu = 1.0 / (s1 - Dt.gamma);
        }
#pragma unroll 1
        for (int c = 0; c < 3 * Dt.m; ++c) W.ft[c] = W.d[c];  // keep -grad
        if (!cone_newton_solve<MM>(Dt, W.f, t, iu, W.d, W.r)) {
            out.status = (nu / t <= 1e3 * gap) ? 0 : 3;
            break;
        }
        double grad_d = 0.0;
#pragma unroll 1
        for (int c = 0; c < 3 * Dt.m; ++c) grad_d -= W.ft[c] * W.d[c];  // grad . d (< 0)
        const double dec2 = -grad_d;
        // the rounding floor: the direction is no longer a descent direction
        // (near the boundary the Newton system is too ill-conditioned for
        // FP64 at large t); accept when the gap is already within 1e3 of the
        // target (nu / t <= 1e-9 for the default target)
        if (!(dec2 > 0.0)) {
            out.status = (nu / t <= 1e3 * gap) ? 0 : 3;
            break;
        }
        // centring: loose on the way (the next weight's Newton steps absorb
        // the rest), tight at the final weight -- but never below the noise
        // of the merit's evaluation (~1e-13 of its value at large t)
        const bool last = nu / t <= gap;
        const double ctol = last ? 1e-10 : loose;
        const bool centred = !(dec2 * 0.5 > fmax(ctol, 1e-12 * fabs(val)));
        if (!centred) {
            // backtracking line search (strict feasibility, Armijo)
            double a = 1.0, nv = INFINITY;
#pragma unroll 1
            for (int ls = 0; ls < 60; ++ls) {
#pragma unroll 1
                for (int c = 0; c < 3 * Dt.m; ++c) W.r[c] = W.f[c] + a * W.d[c];
                nv = cone_merit<MM>(Dt, W.r, t, (const V*)nullptr, nullptr);
                ++out.evals;
                if (nv <= val + 0.25 * a * grad_d) break;
                a *= 0.5;
            }
            if (!(nv <= val + 0.25 * a * grad_d)) {
                // no decrease resolvable: the rounding floor; the point is
                // accepted only when the gap is already within 1e3 of the
                // target (never by raising t without moving)
                out.status = (nu / t <= 1e3 * gap) ? 0 : 3;
                break;
            } else {
#pragma unroll 1
                for (int c = 0; c < 3 * Dt.m; ++c) W.f[c] = W.r[c];
                ++out.grads;
                continue;
            }
        }
        // centred at t: done, or raise t
        if (nu / t <= gap) {
            out.status = 0;
            break;
        }
        t *= growth;
        ++out.grads;
    }
    out.t = t;
    out.q = qv;
    return out;
}

}  // namespace bodex
