/*
 * oracle.h -- plain FP64 CPU reference for the lower-level contact-force QP of
 * BODex (arXiv 2412.16490), its energy and the energy's gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: it exists so that tests, the smoke check and the CPU leg of
 * the benchmark can compare the GPU library against an independent,
 * slow-but-obvious implementation.  It shares no code with the GPU path.
 *
 * What is computed (Sec. III Eq. 1-2, Sec. IV-A Eq. 7-9):
 *   for one grasp with m contacts (p_i, n_i, mu_i) and one desired wrench
 *   direction t (unit, R^6), the forces f = [f_1 .. f_m], f_i = (normal, d, e)
 *   components, minimise
 *        || G f - beta t ||^2 + eps ||f||^2
 *   subject to, per contact, the 8-facet pyramid that linearises Eq. 1's cone,
 *   0 <= f_i1 <= fmax, and sum_i f_i1 >= gamma (Eq. 9).
 *   G_i = [[n, d, e], [kappa p x n, kappa p x d, kappa p x e]] (Eq. 2 with the
 *   torque rows scaled by kappa = 1/L).  The tangents (d, e) come from the
 *   branchless orthonormal basis of Duff et al. (JCGT 6(1), 2017) so that
 *   n = d x e, as Sec. III requires.
 *
 * Readings of the paper that the oracle fixes (each listed in the design
 * notes): inscribed pyramid with edges at k*pi/4 and facets at (2k+1)*pi/8;
 * torque scale kappa; energy includes the eps term; gamma row dropped when
 * gamma <= 0 (it is implied by f_i1 >= 0).
 *
 * Solver: Goldfarb-Idnani dual active-set method (Math. Programming 27, 1983)
 * with every factorisation recomputed from scratch at every step (Cholesky of
 * P, Householder QR of L^{-1} N).  Finite termination for a strictly convex
 * QP; the result is the unique minimiser up to rounding.
 *
 * Parity pins: brute-force active-set enumeration (m <= 2), KKT conditions,
 * closed forms and finite differences -- see tests/.
 */
#ifndef BODEX_ORACLE_H
#define BODEX_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_CONTACTS 8
#define ORC_MAX_VARS (3 * ORC_MAX_CONTACTS)
#define ORC_MAX_ROWS (9 * ORC_MAX_CONTACTS + 1)

typedef struct {
    double kappa; /* torque scale (1/m) applied to the torque rows of G     */
    double beta;  /* desired-wrench magnitude, Eq. 7                         */
    double eps;   /* Tikhonov regulariser on f                               */
    double fmax;  /* upper bound on each normal force component, Eq. 1       */
    double gamma; /* lower bound on the sum of normal components, Eq. 9      */
} orc_params;

typedef struct {
    int status;      /* 0 ok, 1 iteration cap, 2 infeasible, 3 bad input   */
    int steps;       /* number of add/drop steps taken                       */
    int n_active;    /* size of the final active set                         */
    double stat;     /* || P f + q + C^T lam ||_inf                          */
    double primal;   /* max (C f - b)^+                                      */
    double dual;     /* max (-lam)^+                                         */
    double comp;     /* max |lam_k (C_k f - b_k)|                             */
} orc_info;

/* Contact frame: nhat = n/|n|, (d, e) orthonormal tangents with nhat = d x e. */
void orc_frame(const double n[3], double nhat[3], double d[3], double e[3]);

/* Grasp matrix G (row-major, 6 x 3m) from points p[m][3] and normals n[m][3]. */
void orc_grasp_matrix(int m, const double *p, const double *n, double kappa,
                      double *G);

/* One-sided constraints C f <= b (row-major C: nc x 3m).  Rows: per contact the
 * 8 pyramid facets then f_i1 <= fmax; last, -sum f_i1 <= -gamma if gamma > 0.
 * Returns nc. */
int orc_constraints(int m, const double *mu, double fmax, double gamma,
                    double *C, double *b);

/* Solve one QP.  G: 6 x 3m row-major, t: 6.  Outputs f[3m], lam[nc] (may be
 * NULL), Q = ||G f - beta t||^2 + eps ||f||^2.  Returns info.status. */
int orc_qp_solve(int m, const double *G, const double *mu, const double *t,
                 const orc_params *prm, double *f, double *lam, double *Q,
                 orc_info *info);

/* Energy gradient of one grasp from its optimal forces (Danskin):
 *   dE/dG = sum_j w_j * 2 (G f_j - beta t_j) f_j^T,
 * chained to points and normals.  f: [s][3m], t: [s][6], w: [s].
 * Outputs dp[m][3], dn[m][3]. */
void orc_grasp_grad(int m, int s, const double *p, const double *n,
                    const double *f, const double *t, const double *w,
                    const orc_params *prm, double *dp, double *dn);

/* Batched solve over a CSR of grasps.  p, n: [G][m_max][3]; mu: [G][m_max];
 * t: [W][6]; woff: [G+1]; counts: [G].  Outputs forces [W][3 m_max] (zero
 * padded), qobj [W], energy [G], status [W], kkt [W][4] (stat, primal, dual,
 * comp; may be NULL).  nthreads <= 0 uses all hardware threads.
 * Returns 0, or -1 on bad arguments. */
int orc_solve_batch(int n_grasps, int m_max, const int *counts,
                    const int *woff, const double *p, const double *n,
                    const double *mu, const double *t, const orc_params *prm,
                    int nthreads, double *forces, double *qobj,
                    double *energy, int *status, double *kkt);

/* Batched gradient from given forces [W][3 m_max]: dL/dp, dL/dn [G][m_max][3].
 * Weights: wq [W] (dL/dQ_j) and/or we [G] (dL/dE_g); either may be NULL. */
int orc_grad_batch(int n_grasps, int m_max, const int *counts,
                   const int *woff, const double *p, const double *n,
                   const double *t, const double *forces, const double *wq,
                   const double *we, const orc_params *prm, int nthreads,
                   double *dp, double *dn);

/* Relative KKT residual of an ADMM-form state for one QP, in FP64.  The ADMM
 * form has r = 9m+1 two-sided rows l <= A f <= u: per contact the 8 facets
 * (l = -inf, u = 0) then the normal bound (l = 0, u = fmax); last the gamma row
 * (l = gamma, u = +inf).  x[3m], z[r], y[r].
 *   rel = max( ||A x - z|| / (1 + max(||A x||, ||z||)),
 *              ||P x + q + A^T y|| / (1 + max(||P x||, ||A^T y||, ||q||)) )
 * (infinity norms).  out[0] = rel, out[1] = primal part, out[2] = dual part,
 * out[3] = worst violation of z in [l, u] or of the sign rule for y
 * (y > 0 only at z = u, y < 0 only at z = l), scaled like the primal part. */
void orc_admm_rel_kkt(int m, const double *G, const double *mu,
                      const double *t, const orc_params *prm, const double *x,
                      const double *z, const double *y, double *out);

/* Force-sensitivity estimate of one solved QP: 1 / lambda_min(Z^T P Z), where
 * Z spans the null space of the constraints whose multiplier exceeds
 * 1e-9 * max(1, max lam).  Large values flag minimisers that move a lot under
 * an O(u) perturbation of G (free internal-force directions). */
double orc_inv_reduced_curvature(int m, const double *G, const double *mu,
                                 const orc_params *prm, const double *lam);

#ifdef __cplusplus
}
#endif
#endif
