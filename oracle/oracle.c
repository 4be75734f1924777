/*
 * oracle.c -- FP64 CPU reference for the BODex lower-level contact-force QP.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain C11, no GPU, no code shared
 * with the HIP library.  Every matrix factorisation is recomputed from scratch
 * where it is used so that each step can be checked by eye against its
 * definition.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define MAXV ORC_MAX_VARS
#define MAXR ORC_MAX_ROWS

/* ------------------------------------------------------------------------- */
/* Small dense linear algebra (row-major).                                    */
/* ------------------------------------------------------------------------- */

/* Cholesky A = L L^T of an SPD n x n matrix; returns 0 on success. */
static int chol(int n, const double *A, double *L) {
    memset(L, 0, sizeof(double) * (size_t)n * (size_t)n);
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) return -1;
        double ljj = sqrt(s);
        L[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = t / ljj;
        }
    }
    return 0;
}

/* Solve L y = b in place (L lower triangular). */
static void lsolve(int n, const double *L, double *v) {
    for (int i = 0; i < n; ++i) {
        double s = v[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * v[k];
        v[i] = s / L[i * n + i];
    }
}

/* Solve L^T x = y in place. */
static void ltsolve(int n, const double *L, double *v) {
    for (int i = n - 1; i >= 0; --i) {
        double s = v[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * v[k];
        v[i] = s / L[i * n + i];
    }
}

/* Householder QR of B (n x q, column-major in the array cols[j][0..n-1]).
 * On return cols holds R in its upper triangle (R[i][j] = cols[j][i], i <= j)
 * and the unit Householder vectors in hv[j][j..n-1].  Returns 0, or -1 when a
 * column is numerically zero. */
static int house_qr(int n, int q, double cols[][MAXV], double hv[][MAXV]) {
    for (int k = 0; k < q; ++k) {
        double nrm = 0.0;
        for (int i = k; i < n; ++i) nrm += cols[k][i] * cols[k][i];
        nrm = sqrt(nrm);
        if (nrm == 0.0) return -1;
        double alpha = cols[k][k] > 0.0 ? -nrm : nrm;
        double vn = 0.0;
        for (int i = 0; i < n; ++i) hv[k][i] = 0.0;
        for (int i = k; i < n; ++i) hv[k][i] = cols[k][i];
        hv[k][k] -= alpha;
        for (int i = k; i < n; ++i) vn += hv[k][i] * hv[k][i];
        vn = sqrt(vn);
        if (vn > 0.0)
            for (int i = k; i < n; ++i) hv[k][i] /= vn;
        /* apply H_k = I - 2 v v^T to columns k..q-1 */
        for (int j = k; j < q; ++j) {
            double dot = 0.0;
            for (int i = k; i < n; ++i) dot += hv[k][i] * cols[j][i];
            for (int i = k; i < n; ++i) cols[j][i] -= 2.0 * dot * hv[k][i];
        }
    }
    return 0;
}

/* v <- Q^T v, Q = H_0 H_1 ... H_{q-1}. */
static void apply_qt(int n, int q, double hv[][MAXV], double *v) {
    for (int k = 0; k < q; ++k) {
        double dot = 0.0;
        for (int i = k; i < n; ++i) dot += hv[k][i] * v[i];
        for (int i = k; i < n; ++i) v[i] -= 2.0 * dot * hv[k][i];
    }
}

/* v <- Q v. */
static void apply_q(int n, int q, double hv[][MAXV], double *v) {
    for (int k = q - 1; k >= 0; --k) {
        double dot = 0.0;
        for (int i = k; i < n; ++i) dot += hv[k][i] * v[i];
        for (int i = k; i < n; ++i) v[i] -= 2.0 * dot * hv[k][i];
    }
}

/* Symmetric eigenvalues by cyclic Jacobi rotations; A (k x k) is destroyed,
 * eigenvalues returned in ev. */
static void jacobi_eig(int k, double *A, double *ev) {
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < k; ++i) {
            diag += A[i * k + i] * A[i * k + i];
            for (int j = i + 1; j < k; ++j) off += A[i * k + j] * A[i * k + j];
        }
        if (off <= 1e-30 * diag || off == 0.0) break;
        for (int p = 0; p < k; ++p)
            for (int r = p + 1; r < k; ++r) {
                double apr = A[p * k + r];
                if (apr == 0.0) continue;
                double theta = (A[r * k + r] - A[p * k + p]) / (2.0 * apr);
                double t = (theta >= 0 ? 1.0 : -1.0) /
                           (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int i = 0; i < k; ++i) {
                    double aip = A[i * k + p], air = A[i * k + r];
                    A[i * k + p] = c * aip - s * air;
                    A[i * k + r] = s * aip + c * air;
                }
                for (int i = 0; i < k; ++i) {
                    double api = A[p * k + i], ari = A[r * k + i];
                    A[p * k + i] = c * api - s * ari;
                    A[r * k + i] = s * api + c * ari;
                }
            }
    }
    for (int i = 0; i < k; ++i) ev[i] = A[i * k + i];
}

/* ------------------------------------------------------------------------- */
/* Contact frame, grasp matrix, constraints (Sec. III, Eq. 1-2; Sec. IV-A).   */
/* ------------------------------------------------------------------------- */

static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

void orc_frame(const double n[3], double nhat[3], double d[3], double e[3]) {
    double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    double x = n[0] / len, y = n[1] / len, z = n[2] / len;
    nhat[0] = x;
    nhat[1] = y;
    nhat[2] = z;
    /* Duff et al. 2017: branchless ONB, sign taken from the sign bit of z. */
    double s = copysign(1.0, z);
    double a = -1.0 / (s + z);
    double b = x * y * a;
    d[0] = 1.0 + s * x * x * a;
    d[1] = s * b;
    d[2] = -s * x;
    e[0] = b;
    e[1] = s + y * y * a;
    e[2] = -y;
}

void orc_grasp_matrix(int m, const double *p, const double *n, double kappa,
                      double *G) {
    int nv = 3 * m;
    for (int i = 0; i < m; ++i) {
        double nh[3], d[3], e[3];
        orc_frame(n + 3 * i, nh, d, e);
        const double *col[3] = {nh, d, e};
        for (int c = 0; c < 3; ++c) {
            double tq[3];
            cross3(p + 3 * i, col[c], tq);
            for (int a = 0; a < 3; ++a) {
                G[a * nv + 3 * i + c] = col[c][a];
                G[(3 + a) * nv + 3 * i + c] = kappa * tq[a];
            }
        }
    }
}

/* Facet k of the inscribed 8-edge pyramid: edges at angles k*pi/4 lie on the
 * cone f2^2 + f3^2 = mu^2 f1^2; the facet between edges k and k+1 has outward
 * normal direction (2k+1)*pi/8 in the tangent plane and reads
 *     cos(phi_k) f2 + sin(phi_k) f3 - mu cos(pi/8) f1 <= 0. */
static void facet_row(double mu, int k, double row3[3]) {
    double phi = (2.0 * k + 1.0) * M_PI / 8.0;
    row3[0] = -mu * cos(M_PI / 8.0);
    row3[1] = cos(phi);
    row3[2] = sin(phi);
}

int orc_constraints(int m, const double *mu, double fmax, double gamma,
                    double *C, double *b) {
    int nv = 3 * m, r = 0;
    for (int i = 0; i < m; ++i) {
        for (int k = 0; k < 8; ++k, ++r) {
            double row3[3];
            facet_row(mu[i], k, row3);
            for (int j = 0; j < nv; ++j) C[r * nv + j] = 0.0;
            for (int c = 0; c < 3; ++c) C[r * nv + 3 * i + c] = row3[c];
            b[r] = 0.0;
        }
        for (int j = 0; j < nv; ++j) C[r * nv + j] = 0.0;
        C[r * nv + 3 * i] = 1.0;
        b[r] = fmax;
        ++r;
    }
    if (gamma > 0.0) {
        for (int j = 0; j < nv; ++j) C[r * nv + j] = 0.0;
        for (int i = 0; i < m; ++i) C[r * nv + 3 * i] = -1.0;
        b[r] = -gamma;
        ++r;
    }
    return r;
}

/* P = 2 (G^T G + eps I), q = -2 beta G^T t. */
static void qp_terms(int m, const double *G, const double *t,
                     const orc_params *prm, double *P, double *q) {
    int nv = 3 * m;
    for (int i = 0; i < nv; ++i) {
        for (int j = 0; j < nv; ++j) {
            double s = 0.0;
            for (int a = 0; a < 6; ++a) s += G[a * nv + i] * G[a * nv + j];
            P[i * nv + j] = 2.0 * s + (i == j ? 2.0 * prm->eps : 0.0);
        }
        double s = 0.0;
        for (int a = 0; a < 6; ++a) s += G[a * nv + i] * t[a];
        q[i] = -2.0 * prm->beta * s;
    }
}

static double objective(int m, const double *G, const double *t,
                        const orc_params *prm, const double *f) {
    int nv = 3 * m;
    double Q = 0.0;
    for (int a = 0; a < 6; ++a) {
        double w = -prm->beta * t[a];
        for (int j = 0; j < nv; ++j) w += G[a * nv + j] * f[j];
        Q += w * w;
    }
    double ff = 0.0;
    for (int j = 0; j < nv; ++j) ff += f[j] * f[j];
    return Q + prm->eps * ff;
}

/* ------------------------------------------------------------------------- */
/* Goldfarb-Idnani dual active-set method.                                    */
/*   minimise 1/2 x^T P x + q^T x  s.t.  C x <= b,                            */
/*   KKT: P x + q + C_A^T lam_A = 0, lam >= 0, C_A x = b_A.                   */
/* ------------------------------------------------------------------------- */

typedef struct {
    int nv, q;               /* variables, active-set size                    */
    const double *L;         /* Cholesky factor of P                          */
    double cols[MAXV][MAXV]; /* columns of B = L^{-1} N, then R after QR      */
    double hv[MAXV][MAXV];   /* Householder vectors                           */
} gi_fact;

/* Factor B = L^{-1} N for the active rows act[0..q-1]. */
static int gi_factor(gi_fact *F, const double *C, const int *act) {
    int nv = F->nv;
    for (int j = 0; j < F->q; ++j) {
        for (int i = 0; i < nv; ++i) F->cols[j][i] = C[act[j] * nv + i];
        lsolve(nv, F->L, F->cols[j]);
    }
    return house_qr(nv, F->q, F->cols, F->hv);
}

/* For constraint normal c: r = (N^T P^-1 N)^{-1} N^T P^-1 c, the primal
 * direction z = P^{-1}(c - N r), and ||Q_2^T L^{-1} c||, ||L^{-1} c||. */
static void gi_direction(gi_fact *F, const double *c, double *r, double *z,
                         double *h2, double *gn) {
    int nv = F->nv, q = F->q;
    double h[MAXV];
    for (int i = 0; i < nv; ++i) h[i] = c[i];
    lsolve(nv, F->L, h);
    double g2 = 0.0;
    for (int i = 0; i < nv; ++i) g2 += h[i] * h[i];
    *gn = sqrt(g2);
    apply_qt(nv, q, F->hv, h);
    /* r = R^{-1} h[0:q] */
    for (int i = q - 1; i >= 0; --i) {
        double s = h[i];
        for (int j = i + 1; j < q; ++j) s -= F->cols[j][i] * r[j];
        r[i] = s / F->cols[i][i];
    }
    double s2 = 0.0;
    for (int i = q; i < nv; ++i) s2 += h[i] * h[i];
    *h2 = sqrt(s2);
    for (int i = 0; i < q; ++i) h[i] = 0.0;
    apply_q(nv, q, F->hv, h);
    ltsolve(nv, F->L, h);
    for (int i = 0; i < nv; ++i) z[i] = h[i];
}

/* Equality-constrained re-solve on the final active set (removes the drift
 * accumulated by the add/drop updates):
 *   lam = -R^{-1}(R^{-T} b_A + Q_1^T L^{-1} q),  x = -L^{-T} Q [-R^{-T} b_A ; Q_2^T L^{-1} q]. */
static void gi_resolve(gi_fact *F, const double *q, const double *b,
                       const int *act, double *x, double *lam) {
    int nv = F->nv, qa = F->q;
    double c[MAXV], w[MAXV];
    for (int i = 0; i < nv; ++i) c[i] = q[i];
    lsolve(nv, F->L, c);
    apply_qt(nv, qa, F->hv, c);
    /* w = R^{-T} b_A (forward substitution with R^T) */
    for (int i = 0; i < qa; ++i) {
        double s = b[act[i]];
        for (int j = 0; j < i; ++j) s -= F->cols[i][j] * w[j];
        w[i] = s / F->cols[i][i];
    }
    for (int i = qa - 1; i >= 0; --i) {
        double s = w[i] + c[i];
        for (int j = i + 1; j < qa; ++j) s -= F->cols[j][i] * lam[j];
        lam[i] = -s / F->cols[i][i];
    }
    double v[MAXV];
    for (int i = 0; i < qa; ++i) v[i] = -w[i];
    for (int i = qa; i < nv; ++i) v[i] = c[i];
    apply_q(nv, qa, F->hv, v);
    ltsolve(nv, F->L, v);
    for (int i = 0; i < nv; ++i) x[i] = -v[i];
}

static void kkt_measures(int nv, int nc, const double *P, const double *q,
                         const double *C, const double *b, const double *x,
                         const double *lam, orc_info *info) {
    double st = 0.0, pr = 0.0, du = 0.0, co = 0.0;
    for (int i = 0; i < nv; ++i) {
        double g = q[i];
        for (int j = 0; j < nv; ++j) g += P[i * nv + j] * x[j];
        for (int k = 0; k < nc; ++k) g += C[k * nv + i] * lam[k];
        if (fabs(g) > st) st = fabs(g);
    }
    for (int k = 0; k < nc; ++k) {
        double s = -b[k];
        for (int j = 0; j < nv; ++j) s += C[k * nv + j] * x[j];
        if (s > pr) pr = s;
        if (-lam[k] > du) du = -lam[k];
        if (fabs(lam[k] * s) > co) co = fabs(lam[k] * s);
    }
    info->stat = st;
    info->primal = pr;
    info->dual = du;
    info->comp = co;
}

static int gi_solve(int nv, const double *P, const double *q, int nc,
                    const double *C, const double *b, double *x,
                    double *lam_full, orc_info *info) {
    double L[MAXV * MAXV];
    gi_fact F;
    int act[MAXV], is_act[MAXR];
    double u[MAXV + 1], r[MAXV], z[MAXV];
    const double tol_add = 1e-12, tol_dep = 1e-10;
    int steps = 0, status = 0;

    info->steps = 0;
    info->n_active = 0;
    if (chol(nv, P, L)) {
        info->status = 3;
        return 3;
    }
    F.nv = nv;
    F.L = L;
    F.q = 0;
    memset(is_act, 0, sizeof(is_act));

    /* unconstrained minimiser x = -P^{-1} q */
    for (int i = 0; i < nv; ++i) x[i] = -q[i];
    lsolve(nv, L, x);
    ltsolve(nv, L, x);

    int cap = 20 * nc + 100;
    for (;;) {
        /* most violated inactive constraint */
        int p = -1;
        double worst = tol_add;
        for (int k = 0; k < nc; ++k) {
            if (is_act[k]) continue;
            double s = -b[k];
            for (int j = 0; j < nv; ++j) s += C[k * nv + j] * x[j];
            if (s > worst) {
                worst = s;
                p = k;
            }
        }
        if (p < 0) break;
        double up = 0.0;
        const double *cp = C + (size_t)p * nv;
        for (;;) {
            if (++steps > cap) {
                status = 1;
                goto done;
            }
            if (gi_factor(&F, C, act)) {
                status = 1;
                goto done;
            }
            double h2, gn;
            gi_direction(&F, cp, r, z, &h2, &gn);
            double t1 = INFINITY;
            int l = -1;
            for (int j = 0; j < F.q; ++j)
                if (r[j] > 0.0 && u[j] / r[j] < t1) {
                    t1 = u[j] / r[j];
                    l = j;
                }
            int dependent = !(h2 > tol_dep * gn);
            double sp = -b[p];
            for (int j = 0; j < nv; ++j) sp += cp[j] * x[j];
            double t2 = dependent ? INFINITY : sp / (h2 * h2);
            if (dependent && l < 0) {
                status = 2; /* no multiplier can absorb it: infeasible */
                goto done;
            }
            double t = t2 < t1 ? t2 : t1;
            if (!dependent)
                for (int i = 0; i < nv; ++i) x[i] -= t * z[i];
            for (int j = 0; j < F.q; ++j) u[j] -= t * r[j];
            up += t;
            if (t2 <= t1) { /* full step: p joins the active set */
                act[F.q] = p;
                u[F.q] = up;
                is_act[p] = 1;
                F.q++;
                break;
            }
            /* partial step: drop active constraint l, retry p */
            is_act[act[l]] = 0;
            for (int j = l; j < F.q - 1; ++j) {
                act[j] = act[j + 1];
                u[j] = u[j + 1];
            }
            F.q--;
        }
    }
done:
    for (int k = 0; k < nc; ++k) lam_full[k] = 0.0;
    for (int j = 0; j < F.q; ++j) lam_full[act[j]] = u[j] > 0.0 ? u[j] : 0.0;

    if (status == 0 && F.q > 0 && gi_factor(&F, C, act) == 0) {
        /* keep the exact re-solve when it is at least as good */
        double x2[MAXV], lam2[MAXV], lf2[MAXR];
        orc_info a, bi;
        gi_resolve(&F, q, b, act, x2, lam2);
        for (int k = 0; k < nc; ++k) lf2[k] = 0.0;
        for (int j = 0; j < F.q; ++j) lf2[act[j]] = lam2[j];
        kkt_measures(nv, nc, P, q, C, b, x, lam_full, &a);
        kkt_measures(nv, nc, P, q, C, b, x2, lf2, &bi);
        double ea = fmax(fmax(a.stat, a.primal), fmax(a.dual, a.comp));
        double eb = fmax(fmax(bi.stat, bi.primal), fmax(bi.dual, bi.comp));
        if (eb <= ea) {
            memcpy(x, x2, sizeof(double) * nv);
            memcpy(lam_full, lf2, sizeof(double) * nc);
        }
    }
    kkt_measures(nv, nc, P, q, C, b, x, lam_full, info);
    info->status = status;
    info->steps = steps;
    info->n_active = F.q;
    return status;
}

int orc_qp_solve(int m, const double *G, const double *mu, const double *t,
                 const orc_params *prm, double *f, double *lam, double *Q,
                 orc_info *info) {
    orc_info dummy;
    if (!info) info = &dummy;
    if (m < 1 || m > ORC_MAX_CONTACTS) {
        info->status = 3;
        return 3;
    }
    int nv = 3 * m;
    double P[MAXV * MAXV], q[MAXV], C[MAXR * MAXV], b[MAXR], lf[MAXR];
    qp_terms(m, G, t, prm, P, q);
    int nc = orc_constraints(m, mu, prm->fmax, prm->gamma, C, b);
    int st = gi_solve(nv, P, q, nc, C, b, f, lf, info);
    if (lam)
        for (int k = 0; k < nc; ++k) lam[k] = lf[k];
    if (Q) *Q = objective(m, G, t, prm, f);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Energy gradient (Danskin) and chain rule to points and normals.            */
/* ------------------------------------------------------------------------- */

void orc_grasp_grad(int m, int s, const double *p, const double *n,
                    const double *f, const double *t, const double *w,
                    const orc_params *prm, double *dp, double *dn) {
    int nv = 3 * m;
    double G[6 * MAXV], Gb[6 * MAXV];
    orc_grasp_matrix(m, p, n, prm->kappa, G);
    memset(Gb, 0, sizeof(Gb));
    for (int j = 0; j < s; ++j) {
        const double *fj = f + (size_t)j * nv;
        for (int a = 0; a < 6; ++a) {
            double r = -prm->beta * t[6 * j + a];
            for (int c = 0; c < nv; ++c) r += G[a * nv + c] * fj[c];
            for (int c = 0; c < nv; ++c) Gb[a * nv + c] += 2.0 * w[j] * r * fj[c];
        }
    }
    double kap = prm->kappa;
    for (int i = 0; i < m; ++i) {
        const double *pi = p + 3 * i, *ni = n + 3 * i;
        double nh[3], d[3], e[3];
        orc_frame(ni, nh, d, e);
        const double *vec[3] = {nh, d, e};
        double dvec[3][3];
        double dpi[3] = {0, 0, 0};
        for (int c = 0; c < 3; ++c) {
            double gf[3], gt[3], cx[3];
            for (int a = 0; a < 3; ++a) {
                gf[a] = Gb[a * nv + 3 * i + c];
                gt[a] = Gb[(3 + a) * nv + 3 * i + c];
            }
            /* d/dp of gt . (p x v) = v x gt */
            cross3(vec[c], gt, cx);
            for (int a = 0; a < 3; ++a) dpi[a] += kap * cx[a];
            /* d/dv of gf . v + gt . (p x v) = gf + gt x p */
            cross3(gt, pi, cx);
            for (int a = 0; a < 3; ++a) dvec[c][a] = gf[a] + kap * cx[a];
        }
        /* Jacobians of the basis formula with respect to nhat = (x, y, z),
         * the sign s held fixed (it only changes across z = 0). */
        double x = nh[0], y = nh[1], zz = nh[2];
        double sg = copysign(1.0, zz);
        double a = -1.0 / (sg + zz);
        double a2 = a * a;
        double Jd[3][3] = {{2 * sg * x * a, 0.0, sg * x * x * a2},
                           {sg * y * a, sg * x * a, sg * x * y * a2},
                           {-sg, 0.0, 0.0}};
        double Je[3][3] = {{y * a, x * a, x * y * a2},
                           {0.0, 2 * y * a, y * y * a2},
                           {0.0, -1.0, 0.0}};
        double dnh[3];
        for (int k = 0; k < 3; ++k) {
            dnh[k] = dvec[0][k];
            for (int r = 0; r < 3; ++r)
                dnh[k] += Jd[r][k] * dvec[1][r] + Je[r][k] * dvec[2][r];
        }
        double len = sqrt(ni[0] * ni[0] + ni[1] * ni[1] + ni[2] * ni[2]);
        double proj = dnh[0] * nh[0] + dnh[1] * nh[1] + dnh[2] * nh[2];
        for (int k = 0; k < 3; ++k) {
            dn[3 * i + k] = (dnh[k] - proj * nh[k]) / len;
            dp[3 * i + k] = dpi[k];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* ADMM-form relative KKT residual.                                           */
/* ------------------------------------------------------------------------- */

void orc_admm_rel_kkt(int m, const double *G, const double *mu,
                      const double *t, const orc_params *prm, const double *x,
                      const double *z, const double *y, double *out) {
    int nv = 3 * m, r = 9 * m + 1;
    double A[MAXR * MAXV], lo[MAXR], hi[MAXR];
    memset(A, 0, sizeof(double) * (size_t)r * nv);
    for (int i = 0; i < m; ++i) {
        for (int k = 0; k < 8; ++k) {
            double row3[3];
            facet_row(mu[i], k, row3);
            for (int c = 0; c < 3; ++c) A[(9 * i + k) * nv + 3 * i + c] = row3[c];
            lo[9 * i + k] = -INFINITY;
            hi[9 * i + k] = 0.0;
        }
        A[(9 * i + 8) * nv + 3 * i] = 1.0;
        lo[9 * i + 8] = 0.0;
        hi[9 * i + 8] = prm->fmax;
        A[(9 * m) * nv + 3 * i] = 1.0;
    }
    lo[9 * m] = prm->gamma;
    hi[9 * m] = INFINITY;

    double P[MAXV * MAXV], q[MAXV];
    qp_terms(m, G, t, prm, P, q);
    double nAx = 0, nz = 0, rp = 0, nPx = 0, nATy = 0, nq = 0, rd = 0, cv = 0;
    for (int k = 0; k < r; ++k) {
        double ax = 0.0;
        for (int j = 0; j < nv; ++j) ax += A[k * nv + j] * x[j];
        nAx = fmax(nAx, fabs(ax));
        nz = fmax(nz, fabs(z[k]));
        rp = fmax(rp, fabs(ax - z[k]));
        double v = fmax(fmax(lo[k] - z[k], z[k] - hi[k]), 0.0);
        if (y[k] > 0.0) v = fmax(v, fmin(y[k], hi[k] - z[k]));
        if (y[k] < 0.0) v = fmax(v, fmin(-y[k], z[k] - lo[k]));
        cv = fmax(cv, v);
    }
    for (int i = 0; i < nv; ++i) {
        double px = 0.0, aty = 0.0;
        for (int j = 0; j < nv; ++j) px += P[i * nv + j] * x[j];
        for (int k = 0; k < r; ++k) aty += A[k * nv + i] * y[k];
        nPx = fmax(nPx, fabs(px));
        nATy = fmax(nATy, fabs(aty));
        nq = fmax(nq, fabs(q[i]));
        rd = fmax(rd, fabs(px + q[i] + aty));
    }
    double pscale = 1.0 + fmax(nAx, nz);
    double dscale = 1.0 + fmax(fmax(nPx, nATy), nq);
    out[1] = rp / pscale;
    out[2] = rd / dscale;
    out[0] = fmax(out[1], out[2]);
    out[3] = cv / pscale;
}

/* ------------------------------------------------------------------------- */
/* Force-sensitivity estimate.                                                */
/* ------------------------------------------------------------------------- */

double orc_inv_reduced_curvature(int m, const double *G, const double *mu,
                                 const orc_params *prm, const double *lam) {
    int nv = 3 * m;
    double C[MAXR * MAXV], b[MAXR];
    int nc = orc_constraints(m, mu, prm->fmax, prm->gamma, C, b);
    double lmax = 1.0;
    for (int k = 0; k < nc; ++k) lmax = fmax(lmax, lam[k]);
    /* orthonormal basis of the span of strongly active normals (Gram-Schmidt
     * with re-orthogonalisation, dependent rows skipped) */
    double basis[MAXV][MAXV];
    int q = 0;
    for (int k = 0; k < nc && q < nv; ++k) {
        if (!(lam[k] > 1e-9 * lmax)) continue;
        double v[MAXV];
        for (int j = 0; j < nv; ++j) v[j] = C[k * nv + j];
        double n0 = 0.0;
        for (int j = 0; j < nv; ++j) n0 += v[j] * v[j];
        n0 = sqrt(n0);
        for (int pass = 0; pass < 2; ++pass)
            for (int a = 0; a < q; ++a) {
                double dot = 0.0;
                for (int j = 0; j < nv; ++j) dot += basis[a][j] * v[j];
                for (int j = 0; j < nv; ++j) v[j] -= dot * basis[a][j];
            }
        double nn = 0.0;
        for (int j = 0; j < nv; ++j) nn += v[j] * v[j];
        nn = sqrt(nn);
        if (nn <= 1e-8 * n0) continue;
        for (int j = 0; j < nv; ++j) basis[q][j] = v[j] / nn;
        q++;
    }
    if (q >= nv) return 0.0;
    /* complete to an orthonormal basis of R^nv; the extra vectors span Z */
    double Z[MAXV][MAXV];
    int nz = 0;
    for (int e = 0; e < nv && q + nz < nv; ++e) {
        double v[MAXV];
        for (int j = 0; j < nv; ++j) v[j] = (j == e) ? 1.0 : 0.0;
        for (int pass = 0; pass < 2; ++pass) {
            for (int a = 0; a < q; ++a) {
                double dot = 0.0;
                for (int j = 0; j < nv; ++j) dot += basis[a][j] * v[j];
                for (int j = 0; j < nv; ++j) v[j] -= dot * basis[a][j];
            }
            for (int a = 0; a < nz; ++a) {
                double dot = 0.0;
                for (int j = 0; j < nv; ++j) dot += Z[a][j] * v[j];
                for (int j = 0; j < nv; ++j) v[j] -= dot * Z[a][j];
            }
        }
        double nn = 0.0;
        for (int j = 0; j < nv; ++j) nn += v[j] * v[j];
        nn = sqrt(nn);
        if (nn < 1e-6) continue;
        for (int j = 0; j < nv; ++j) Z[nz][j] = v[j] / nn;
        nz++;
    }
    double P[MAXV * MAXV], qd[MAXV], t0[6] = {0, 0, 0, 0, 0, 0};
    qp_terms(m, G, t0, prm, P, qd);
    double H[MAXV * MAXV], ev[MAXV];
    for (int a = 0; a < nz; ++a)
        for (int c = 0; c < nz; ++c) {
            double s = 0.0;
            for (int i = 0; i < nv; ++i)
                for (int j = 0; j < nv; ++j) s += Z[a][i] * P[i * nv + j] * Z[c][j];
            H[a * nz + c] = s;
        }
    jacobi_eig(nz, H, ev);
    double emin = INFINITY;
    for (int a = 0; a < nz; ++a) emin = fmin(emin, ev[a]);
    return emin > 0.0 ? 1.0 / emin : INFINITY;
}

/* ------------------------------------------------------------------------- */
/* Batched drivers with a plain thread pool over grasps.                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n_grasps, m_max;
    const int *counts, *woff;
    const double *p, *n, *mu, *t;
    const orc_params *prm;
    double *forces, *qobj, *energy, *kkt;
    int *status;
    const double *fin, *wq, *we;
    double *dp, *dn;
    atomic_int next;
} batch_job;

static void solve_one_grasp(batch_job *J, int g) {
    int m = J->counts[g], mm = J->m_max, nv = 3 * m;
    double G[6 * MAXV];
    orc_grasp_matrix(m, J->p + (size_t)g * mm * 3, J->n + (size_t)g * mm * 3,
                     J->prm->kappa, G);
    const double *mu = J->mu + (size_t)g * mm;
    double E = 0.0;
    for (int w = J->woff[g]; w < J->woff[g + 1]; ++w) {
        double f[MAXV], Q;
        orc_info info;
        orc_qp_solve(m, G, mu, J->t + (size_t)w * 6, J->prm, f, NULL, &Q, &info);
        double *fo = J->forces + (size_t)w * 3 * mm;
        for (int j = 0; j < 3 * mm; ++j) fo[j] = j < nv ? f[j] : 0.0;
        J->qobj[w] = Q;
        J->status[w] = info.status;
        if (J->kkt) {
            J->kkt[4 * (size_t)w + 0] = info.stat;
            J->kkt[4 * (size_t)w + 1] = info.primal;
            J->kkt[4 * (size_t)w + 2] = info.dual;
            J->kkt[4 * (size_t)w + 3] = info.comp;
        }
        E += Q;
    }
    J->energy[g] = E;
}

static void grad_one_grasp(batch_job *J, int g) {
    int m = J->counts[g], mm = J->m_max, nv = 3 * m;
    int w0 = J->woff[g], s = J->woff[g + 1] - w0;
    double *f = malloc(sizeof(double) * (size_t)(s > 0 ? s : 1) * nv);
    double *w = malloc(sizeof(double) * (size_t)(s > 0 ? s : 1));
    for (int j = 0; j < s; ++j) {
        for (int c = 0; c < nv; ++c) f[j * nv + c] = J->fin[(size_t)(w0 + j) * 3 * mm + c];
        w[j] = (J->wq ? J->wq[w0 + j] : 0.0) + (J->we ? J->we[g] : 0.0);
    }
    double dp[3 * ORC_MAX_CONTACTS], dn[3 * ORC_MAX_CONTACTS];
    orc_grasp_grad(m, s, J->p + (size_t)g * mm * 3, J->n + (size_t)g * mm * 3, f,
                   J->t + (size_t)w0 * 6, w, J->prm, dp, dn);
    for (int j = 0; j < 3 * mm; ++j) {
        J->dp[(size_t)g * mm * 3 + j] = j < nv ? dp[j] : 0.0;
        J->dn[(size_t)g * mm * 3 + j] = j < nv ? dn[j] : 0.0;
    }
    free(f);
    free(w);
}

typedef struct {
    batch_job *J;
    int grad;
} worker_arg;

static void *worker(void *arg) {
    worker_arg *A = (worker_arg *)arg;
    for (;;) {
        int g = atomic_fetch_add(&A->J->next, 1);
        if (g >= A->J->n_grasps) break;
        if (A->grad)
            grad_one_grasp(A->J, g);
        else
            solve_one_grasp(A->J, g);
    }
    return NULL;
}

static void run_pool(batch_job *J, int grad, int nthreads) {
    if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    atomic_store(&J->next, 0);
    worker_arg A = {J, grad};
    if (nthreads == 1) {
        worker(&A);
        return;
    }
    pthread_t th[256];
    for (int i = 0; i < nthreads; ++i) pthread_create(&th[i], NULL, worker, &A);
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
}

static int check_batch(int n_grasps, int m_max, const int *counts, const int *woff) {
    if (n_grasps < 0 || m_max < 1 || m_max > ORC_MAX_CONTACTS) return -1;
    for (int g = 0; g < n_grasps; ++g) {
        if (counts[g] < 1 || counts[g] > m_max) return -1;
        if (woff[g + 1] < woff[g]) return -1;
    }
    return 0;
}

int orc_solve_batch(int n_grasps, int m_max, const int *counts,
                    const int *woff, const double *p, const double *n,
                    const double *mu, const double *t, const orc_params *prm,
                    int nthreads, double *forces, double *qobj,
                    double *energy, int *status, double *kkt) {
    if (check_batch(n_grasps, m_max, counts, woff)) return -1;
    batch_job J;
    memset(&J, 0, sizeof(J));
    J.n_grasps = n_grasps;
    J.m_max = m_max;
    J.counts = counts;
    J.woff = woff;
    J.p = p;
    J.n = n;
    J.mu = mu;
    J.t = t;
    J.prm = prm;
    J.forces = forces;
    J.qobj = qobj;
    J.energy = energy;
    J.status = status;
    J.kkt = kkt;
    run_pool(&J, 0, nthreads);
    return 0;
}

int orc_grad_batch(int n_grasps, int m_max, const int *counts,
                   const int *woff, const double *p, const double *n,
                   const double *t, const double *forces, const double *wq,
                   const double *we, const orc_params *prm, int nthreads,
                   double *dp, double *dn) {
    if (check_batch(n_grasps, m_max, counts, woff)) return -1;
    batch_job J;
    memset(&J, 0, sizeof(J));
    J.n_grasps = n_grasps;
    J.m_max = m_max;
    J.counts = counts;
    J.woff = woff;
    J.p = p;
    J.n = n;
    J.t = t;
    J.prm = prm;
    J.fin = forces;
    J.wq = wq;
    J.we = we;
    J.dp = dp;
    J.dn = dn;
    run_pool(&J, 1, nthreads);
    return 0;
}
