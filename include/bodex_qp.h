/*
 * bodex_qp.h -- C ABI of the MI355X (gfx950) batched contact-force QP library.
 *
 * The library solves, for every grasp g and every desired wrench direction
 * t_j of that grasp, the lower-level QP of BODex (arXiv 2412.16490,
 * Sec. IV-A, Eq. 7-9):
 *
 *     Q_j = min_f || G f - beta t_j ||^2 + eps ||f||^2
 *           s.t.  f_i inside the 8-facet pyramid that linearises the friction
 *                 cone of Eq. 1 (Sec. IV-A, last paragraph), 0 <= f_i1 <= fmax,
 *                 and sum_i f_i1 >= gamma (Eq. 9),
 *
 * where G = [G_1 .. G_m] is the grasp matrix of Eq. 2 built from contact
 * points p_i and inward normals n_i (Sec. III), with the torque rows scaled by
 * torque_scale.  It returns the optimal forces, Q_j, the grasp energy
 * E_g = sum_j Q_j (Eq. 3 restricted to the QP terms), and the gradient of a
 * weighted sum of E_g and Q_j with respect to p_i and n_i (Sec. IV-A: Q_j is
 * differentiable because G_i is).
 *
 * Method: ADMM in the ReLU-QP style (Sec. IV-B) -- one Cholesky-factorised
 * KKT matrix per grasp shared by all of its wrenches, an affine step plus a
 * clamp per iteration, periodic residual checks with per-grasp step-size
 * adaptation -- followed by an FP64 polish that re-solves the reduced KKT
 * system on the identified active set and corrects that set with dual
 * active-set steps, keeping the polished point only when its KKT conditions
 * hold.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Return value: 0 on success or a negative BODEX_E* code.  No C++ exception
 *    crosses this boundary.  bodex_qp_last_error() gives a message.
 *  * Device arrays are caller-owned, contiguous, 4-byte aligned, on the
 *    handle's device.  Host arrays (marked HOST) are read during the call only.
 *  * Work is enqueued on the handle's HIP stream; calls return once enqueued.
 *    Outputs are valid after the stream (or an event recorded on it) is
 *    synchronised.  Host arrays may be reused as soon as the call returns.
 *  * A handle is not thread-safe; use one handle per stream.  Handles are
 *    independent of each other.
 *  * Per-QP numerical trouble never fails a call: it is reported in status[].
 */
#ifndef BODEX_QP_H
#define BODEX_QP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BODEX_MAX_CONTACTS 8  /* m_max upper limit                       */
#define BODEX_MAX_WRENCHES 64 /* s_max upper limit (wrenches per grasp)   */

/* Error codes. */
#define BODEX_OK 0
#define BODEX_EINVAL -1     /* invalid argument (bad size, null pointer, ...) */
#define BODEX_EHIP -2       /* HIP runtime error; see bodex_qp_last_error     */
#define BODEX_EBUDGET -3    /* request exceeds the handle's device budget     */
#define BODEX_EINFEAS -4    /* gamma > m * fmax for some grasp: infeasible    */
#define BODEX_EUNSUP -5     /* unsupported size (s > s_max, m > m_max)        */
#define BODEX_ENODEV -6     /* no usable GPU device                           */

/* Per-QP status bits (status[w]). */
#define BODEX_ST_CONVERGED 0x01  /* final relative KKT residual <= tol_rel     */
#define BODEX_ST_MAX_ITER 0x02   /* ADMM stopped at max_iters above tol_rel   */
#define BODEX_ST_NONFINITE 0x04  /* non-finite input or iterate (QP isolated) */
#define BODEX_ST_FP64_CHOL 0x08  /* the grasp's KKT factor needed FP64        */
#define BODEX_ST_POLISH_REJ 0x10 /* polish ran but its point failed KKT       */
#define BODEX_ST_POLISHED 0x20   /* returned point is the accepted polish     */

/* Flags (bodex_qp_params.flags). */
#define BODEX_F_WARM_START 0x01   /* start ADMM from the state passed in       */
#define BODEX_F_POLISH 0x02       /* run the FP64 polish after ADMM            */
#define BODEX_F_ADAPTIVE_RHO 0x04 /* per-grasp rho adaptation                  */
#define BODEX_F_BATCHED 0x08      /* persistent cost-sorted launch (uneven m,s)*/
#define BODEX_F_GRAPH 0x10        /* capture launches in a hipGraph and replay */
                                  /* it while the batch shape is unchanged     */
#define BODEX_F_TIMING 0x20       /* record HIP events around each kernel      */
#define BODEX_F_SIGNED_DIST 0x40  /* E^c_d with the signed distance d_i (see   */
                                  /* bodex_qp_pose_gradient)                   */

/* Friction model (bodex_qp_params.friction_cone).
 * PYRAMID8: the 8-facet pyramid inscribed in the cone of Eq. 1, the
 *   linearisation of Sec. IV-A (facets at (2k+1) pi/8 with coefficient
 *   mu cos(pi/8)).
 * CIRCULAR: the exact cone |(f_2, f_3)| <= mu f_1 of Eq. 1 (the quadratically
 *   constrained form the paper linearises).  ADMM projects each contact's
 *   force onto the cone truncated at fmax (closed form); the FP64 polish is a
 *   barrier (interior-point) method warm-started from the ADMM point.  The
 *   ADMM state has 3 m_max + 1 rows of z and y (rows 3i..3i+2 contact i's
 *   force, row 3 m_max the normal-sum row).  bodex_qp_backward uses the
 *   polished forces the solve left in state.x. */
#define BODEX_CONE_PYRAMID8 0
#define BODEX_CONE_CIRCULAR 1

typedef struct {
    int m_max;            /* contacts per grasp, 1..8 (array padding); 1..5  */
                          /* with BODEX_CONE_CIRCULAR                        */
    int s_max;            /* wrenches per grasp, 1..64                        */
    float force_max;      /* fmax, upper bound of f_i1 (Eq. 1: 1.0)           */
    float gamma;          /* lower bound of sum_i f_i1 (Eq. 9); 0 = unused    */
    float beta;           /* desired-wrench magnitude (Eq. 7)                 */
    float eps_reg;        /* regulariser eps on ||f||^2                       */
    float torque_scale;   /* kappa: torque rows of G are kappa * (p x c)      */
    float tol_rel;        /* stop when relative KKT residual <= tol_rel       */
    int max_iters;        /* ADMM iteration cap                               */
    float rho0;           /* initial ADMM step size                           */
    float alpha;          /* over-relaxation, in (0, 2)                       */
    int check_every;      /* residual check / rho update period (iterations); */
                          /* with BODEX_F_POLISH and admm_tol 0 the pyramid's */
                          /* ADMM uses max(check_every, 20)                   */
    float rho_min;        /* clamp of the adapted rho                         */
    float rho_max;
    float rho_hysteresis; /* refactor only when rho changes by this factor    */
    float fp64_cond;      /* factor K in FP64 when cond estimate exceeds this */
    int polish_steps;     /* cap on active-set corrections in the polish      */
    int polish_chunk;     /* factorisations a QP takes in the one-lane FP64   */
                          /* polish before it is handed to the contact-       */
                          /* parallel polish (a group of lanes, one per       */
                          /* contact); 0 = every polish ends in the one-lane  */
                          /* kernel; -1 = chosen by the number of QPs (1 up   */
                          /* to 40,960, else 16).  A QP is                    */
                          /* also handed on at its next factorisation once at */
                          /* most 8 lanes of its wavefront still polish.      */
                          /* Used with BODEX_F_POLISH, the pyramid and        */
                          /* gamma = 0.                                       */
    unsigned flags;       /* BODEX_F_*                                        */
    int admm_waves;       /* ADMM kernel register budget as resident waves   */
                          /* per SIMD: 1, 2, 3 or 4 (0 = library default)     */
    float admm_tol;       /* ADMM stops a QP at this relative KKT residual;   */
                          /* the polish then lifts it to tol_rel (0 = the     */
                          /* friction model's default: 1e-1 for PYRAMID8,     */
                          /* 1e-4 for CIRCULAR, whose ADMM then also stops    */
                          /* after min(max_iters, 200) iterations; without    */
                          /* BODEX_F_POLISH ADMM always runs to tol_rel)      */
    int friction_cone;    /* BODEX_CONE_PYRAMID8 (default) or                 */
                          /* BODEX_CONE_CIRCULAR                              */
} bodex_qp_params;

/* One batch of grasps (CSR over wrenches). */
typedef struct {
    int n_grasps;              /* G >= 0                                      */
    int n_qps;                 /* W = wrench_offset[G]                        */
    const int *contact_count;  /* HOST [G], 1 <= m_g <= m_max                 */
    const int *wrench_offset;  /* HOST [G+1], nondecreasing, s_g <= s_max     */
    const float *points;       /* device [G][m_max][3]  p_i (object frame)    */
    const float *normals;      /* device [G][m_max][3]  n_i (normalised inside)*/
    const float *mu;           /* device [G][m_max]     friction, > 0         */
    const float *wrench_dir;   /* device [W][6]         t_j (beta applied)    */
} bodex_batch;

/* ADMM state, structure-of-arrays so that consecutive QPs are consecutive in
 * memory.  Rows of z, y per contact i: 8 pyramid facets (9i .. 9i+7), then
 * the normal bound (9i+8); row 9*m_max is the gamma row.  Unused rows of
 * grasps with fewer contacts hold zeros.  With BODEX_CONE_CIRCULAR z and y
 * have 3 m_max + 1 rows instead (see there). */
typedef struct {
    float *x;   /* device [3 m_max][W]      forces in (normal, d, e) order    */
    float *z;   /* device [9 m_max + 1][W]                                    */
    float *y;   /* device [9 m_max + 1][W]  dual variables                    */
    float *rho; /* device [G]               per-grasp ADMM step size          */
    float *r;   /* optional device [6][W]: the wrench residual G f - beta t */
                /* of the returned forces, formed in FP64 and rounded; the  */
                /* backward uses it (formed from the FP32 forces it loses   */
                /* its digits to cancellation when it is small).  NULL: not */
                /* written; the backward then recovers f* in FP64 (pyramid: */
                /* one more polish) or uses the FP32 forces (cone).         */
    /* Layout of the arrays above.  By default (stride 0, offsets NULL) a  */
    /* batch's QP w is column w of arrays with W columns and grasp g's rho */
    /* is rho[g].  A caller that keeps several requests' states in one     */
    /* pool (a serving loop) sets stride = the pool's column count and,    */
    /* per grasp of the batch, qp_offset[g] = the pool column of its first */
    /* QP (its s_g QPs follow) and grasp_offset[g] = its index in rho (of  */
    /* rho_len); columns of different grasps must not overlap.  The solve, */
    /* the backward and the descent then read and write the state in place */
    /* (no gather or scatter).  qp_offset and grasp_offset are HOST arrays, */
    /* read during the call; both or neither.                              */
    int stride;
    int rho_len;
    const int *qp_offset;
    const int *grasp_offset;
} bodex_state;

typedef struct {
    float *forces;          /* device [W][3 m_max]  optimal f (zero padded)   */
    float *qp_obj;          /* device [W]   Q_j = ||G f - beta t||^2+eps||f||^2 */
    float *energy;          /* device [G]   E_g = sum_j Q_j                   */
    float *kkt_rel;         /* device [W]   relative KKT residual of state    */
    int *iters;             /* device [W]   ADMM iterations used              */
    unsigned char *status;  /* device [W]   BODEX_ST_* bits                   */
    bodex_state state;      /* optional in/out state; all-NULL pointers make  */
                            /* the library use its own workspace              */
    float *polish_flops;    /* optional device [W]: algorithmic FP64 flops    */
                            /* the polish spent on each QP (0 without polish; */
                            /* NULL = not written), for roofline accounting   */
} bodex_result;

typedef struct bodex_qp bodex_qp_t;

/* Fill *p with the defaults: m_max 5, s_max 32, fmax 1, gamma 0, beta 1,
 * eps 1e-6, torque_scale 20, tol 1e-5, 500 iterations, rho0 0.3, alpha 1.6,
 * check every 10, rho in [1e-4, 1e4], hysteresis 5, fp64_cond 1e4, 128 polish
 * steps, polish_chunk -1, flags POLISH | ADAPTIVE_RHO, admm_waves 0,
 * admm_tol 0 (the model's default; with the polish on, ADMM only has to find the active set
 * roughly; the polish then solves each QP exactly). */
void bodex_qp_default_params(bodex_qp_params *p);

/* Create a handle on `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL = the default stream).  hbm_budget_bytes caps the library-owned
 * workspace (0 = 4 GiB).  The kernels are compiled for 4, 5, 6, 7 and 8
 * contacts (a batch runs on the smallest size >= m_max; the circular cone's
 * for 4 and 5).  Errors: EINVAL (bad params), EUNSUP (m_max above 5 with
 * BODEX_CONE_CIRCULAR), ENODEV, EHIP. */
int bodex_qp_create(const bodex_qp_params *p, int device, void *hip_stream,
                    size_t hbm_budget_bytes, bodex_qp_t **out);

/* Change the stream used by later calls (same device). */
int bodex_qp_set_stream(bodex_qp_t *h, void *hip_stream);

/* Forward solve of every QP in the batch.  With BODEX_F_WARM_START the ADMM
 * starts from out->state (which must then be non-NULL and hold a previous
 * state, e.g. from an earlier call on the same grasps); otherwise from zero.
 * Errors: EINVAL (null pointers, bad sizes, mu <= 0 is reported per QP as
 * non-finite), EUNSUP, EINFEAS, EBUDGET (workspace above budget), EHIP. */
int bodex_qp_solve(bodex_qp_t *h, const bodex_batch *in, bodex_result *out);

/* Descriptor ints the allocation-free solve can hold: 3 G + (tiles) + 6
 * <= 2^20 (a tile holds at least one grasp, so every batch of up to
 * 262,142 grasps fits). */
#define BODEX_STATIC_SCRATCH_INTS (1 << 20)

/* bodex_qp_solve without allocation, for callers that cannot allocate
 * device or pinned host memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The plain form's kernels with
 * the one-lane FP64 polish run to the end (polish_chunk is not used: the
 * contact-parallel polish needs workspace), so the results equal
 * bodex_qp_solve's with polish_chunk 0; the batch descriptor (contact counts,
 * wrench offsets, tile schedule) lives in a static device array of
 * BODEX_STATIC_SCRATCH_INTS ints (4 MiB per GPU, held until the process
 * ends; its address is taken per device at bodex_qp_create), staged through
 * a static pageable host buffer.  The caller passes the state (out->state:
 * x, z, y, rho all non-NULL; r optional); no library workspace is used.
 * Every call on one GPU shares that GPU's array and keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other threads)
 * race, so serialise them.  Calls no hipMalloc, hipFree or hipHostMalloc.
 * Errors: EINVAL (as bodex_qp_solve, or a NULL state pointer), EUNSUP
 * (BODEX_F_BATCHED or BODEX_F_GRAPH set; a batch beyond the scratch), EHIP. */
int bodex_qp_solve_static(bodex_qp_t *h, const bodex_batch *in, bodex_result *out);

/* Gradient of L = sum_g dL_dE[g] E_g + sum_w dL_dQ[w] Q_w with respect to
 * points and normals (Danskin's theorem: the feasible set does not depend on
 * p or n, so dQ/dG = 2 (G f* - beta t) f*^T, chained through Eq. 2 and the
 * tangent-basis construction).  f* is recomputed from `st` (the state a
 * solve wrote for the same batch); ADMM iterates are never stored.
 * dL_dE [G] and dL_dQ [W] are device arrays, either may be NULL.
 * Outputs dL_dpoints, dL_dnormals: device [G][m_max][3]; overwritten, or
 * added to when `accumulate` is non-zero.  The normal gradient has no radial
 * component (normals are normalised inside).  Errors: EINVAL, EHIP. */
int bodex_qp_backward(bodex_qp_t *h, const bodex_batch *in,
                      const bodex_state *st, const float *dL_dE,
                      const float *dL_dQ, float *dL_dpoints,
                      float *dL_dnormals, int accumulate);

/* Free library-owned memory and graphs.  Never frees caller arrays. */
int bodex_qp_destroy(bodex_qp_t *h);

/* Message of the last error on this handle (or of the last failed create when
 * h is NULL).  Valid until the next call on the handle. */
const char *bodex_qp_last_error(const bodex_qp_t *h);

/* Device bytes of a caller-held state for a batch (x, z, y, rho and the
 * residual r); the pyramid layout, an upper bound for the circular cone's. */
size_t bodex_qp_state_bytes(int n_grasps, int n_qps, int m_max);

/* The values the library takes for parameters whose rule it owns (see
 * admm_tol, check_every, max_iters and polish_chunk above), for a solve of
 * n_qps QPs with *p: ADMM's stopping tolerance, iteration cap and residual
 * check period, and the one-lane polish's factorisation budget (0: the
 * polish runs one lane per QP to the end, as for the circular cone, gamma > 0
 * or without BODEX_F_POLISH).  Needs no device.  Any output pointer may be
 * NULL; BODEX_EINVAL (message in bodex_qp_last_error(NULL)) for invalid
 * parameters. */
int bodex_qp_effective_params(const bodex_qp_params *p, int n_qps, float *admm_tol, int *max_iters,
                              int *check_every, int *polish_chunk);

/* Statistics of the last solve (host copies, filled after the stream is
 * synchronised by this call): number of graph replays, refactorisations,
 * launches.  Any pointer may be NULL.  Synchronises the handle's stream. */
int bodex_qp_last_stats(bodex_qp_t *h, int *launches, int *graph_replays,
                        int *tiles);

/* Kernel durations (milliseconds) of the last solve and backward on this
 * handle, measured with HIP events recorded on the handle's stream around each
 * kernel when BODEX_F_TIMING is set (otherwise reported as -1).  With
 * BODEX_F_GRAPH the events bracket the whole graph launch and are reported as
 * the ADMM time.  Synchronises on the events.  Any pointer may be NULL. */
int bodex_qp_kernel_times(bodex_qp_t *h, float *admm_ms, float *finalize_ms,
                          float *backward_ms);

/* Inputs of the fine-stage surrogate energies (Sec. IV-C, Eq. 10-11): one
 * entry per fingertip contact, arrays [G][m][...] contiguous in that order.
 * Unlike bodex_batch, the contact counts are a device array. */
typedef struct {
    int n_grasps;             /* G >= 0                                       */
    int m;                    /* contacts per grasp in the layout, 1..8       */
    const int *contact_count; /* device [G] contacts used (<= m); NULL = m    */
    const float *link_rot;    /* device [G][m][3][3] R_i of the fingertip's   */
                              /* link, row-major, invertible                  */
    const float *link_trans;  /* device [G][m][3] T_i                         */
    const float *hand_fine;   /* device [G][m][3] c^f_{i,w}: nearest point on */
                              /* the fingertip (fine stage, world frame)      */
    const float *obj_fine;    /* device [G][m][3] p^f_i: nearest object point */
    const float *obj_coarse;  /* device [G][m][3] p^c_i: object point from the*/
                              /* end of the coarse stage                      */
} bodex_fine_contacts;

/* Fine-stage energies with the Detach trick (Sec. IV-C, Eq. 10-11).  Per
 * contact, c_l = R^{-1} (c^f_w - T) is the fingertip point in its link frame,
 * held constant, and c' = R c_l + T; then
 *     q_surr[g] = Q'    = sum_i |c'_i - p^c_i|^2,
 *     e_dist[g] = E^f_d = sum_i |c'_i - p^f_i|^2
 * (device [G], required).  With dL_dR (device [G][m][3][3]) and dL_dT
 * (device [G][m][3]) -- both or neither -- also the gradient of
 * L = sum_g w_q[g] Q'_g + w_e[g] E^f_{d,g} with respect to the link
 * transforms, dL/dR_i = g_i c_l^T and dL/dT_i = g_i with
 * g_i = 2 w_q (c'_i - p^c_i) + 2 w_e (c'_i - p^f_i); w_q, w_e are device [G],
 * NULL = weight 0.  Gradients are overwritten, or added to when `accumulate`
 * is non-zero; contacts at or beyond contact_count[g] add nothing and get a
 * zero gradient.  Uses no workspace.  Errors: EINVAL (m outside 1..8,
 * G < 0, a required pointer NULL, only one gradient output, misaligned),
 * EHIP. */
int bodex_qp_detach_energy(bodex_qp_t *h, const bodex_fine_contacts *in,
                           const float *w_q, const float *w_e, float *q_surr,
                           float *e_dist, float *dL_dR, float *dL_dT,
                           int accumulate);

/* A floating hand over an analytic object, one per grasp: the step before
 * the QP in the coarse stage (Sec. IV-B forward kinematics for a hand whose
 * fingertips share the root transform; Sec. IV-C nearest-point query and
 * distance energy, here on analytic shapes).  Arrays [G][m][...] contiguous
 * in that order. */
typedef struct {
    int n_grasps;             /* G >= 0                                       */
    int m;                    /* fingertips per grasp in the layout, 1..8     */
    const int *contact_count; /* device [G] fingertips used (<= m); NULL = m  */
    const float *tip_local;   /* device [G][m][3] c_{i,l}: centre of the      */
                              /* fingertip's sphere in the hand frame         */
    const float *semi_axes;   /* device [G][3] the object: the solid ellipsoid */
                              /* sum_k (x_k / a_k)^2 <= 1 centred at the world */
                              /* origin (a sphere when equal); a_k > 0, not   */
                              /* checked (non-positive axes give NaN outputs) */
    float *hand_rot;          /* device [G][3][3] R, row-major rotation       */
    float *hand_trans;        /* device [G][3] T                              */
                              /* (both updated in place by bodex_qp_descend)  */
} bodex_hand;

/* Contacts of every fingertip: c_i = R c_{i,l} + T, the nearest point p_i of
 * the object's surface, its inward unit normal n_i and the signed distance
 * d_i of c_i (positive outside).  Computed in FP64 (the nearest point is the
 * root of the Lagrange condition, found by a monotone Newton iteration).
 * Where the nearest point is not unique (the medial ridge inside the object,
 * including a sphere's centre) one of them is returned.  Outputs points,
 * normals: device [G][m][3] (the layout of bodex_batch when m = m_max);
 * dist: device [G][m] or NULL.  Fingertips at or beyond contact_count[g] get
 * zeros.  Uses no workspace.  Errors: EINVAL (m outside 1..8, G < 0, a
 * required pointer NULL, misaligned), EHIP. */
int bodex_qp_contact_query(bodex_qp_t *h, const bodex_hand *in, float *points,
                           float *normals, float *dist);

/* Gradient with respect to the hand pose of
 *     L = (the caller's loss through the contacts) + w_dist E^c_d,
 *     E^c_d = sum_i (|c_i - p_i| - radius - offset)^2
 * (the coarse distance energy of Sec. IV-C; radius is the fingertip sphere's
 * radius alpha, offset the pre-grasp distance reduction of Sec. IV-D).  With
 * BODEX_F_SIGNED_DIST in the handle's flags the signed distance d_i takes
 * the place of |c_i - p_i|, so that a fingertip inside the object is pushed
 * out rather than held at distance alpha inside the surface.  On the surface
 * (d_i = 0) the unsigned form takes the outside branch of its derivative.  dL_dpoints, dL_dnormals: device [G][m][3], e.g.
 * from bodex_qp_backward; either may be NULL (no such term).  The contacts'
 * derivative is the exact Jacobian of the query (implicit function theorem;
 * zero where the nearest point is not unique).  Outputs (each optional):
 * e_dist [G] = E^c_d; dL_drot [G][3] = dL/domega for the world-frame
 * rotation vector omega of R(omega) = Exp(omega) R, i.e.
 * sum_i (R c_{i,l}) x dL/dc_i; dL_dtrans [G][3] = sum_i dL/dc_i.  Uses no
 * workspace.  Errors: EINVAL, EHIP. */
int bodex_qp_pose_gradient(bodex_qp_t *h, const bodex_hand *in,
                           const float *dL_dpoints, const float *dL_dnormals,
                           float w_dist, float radius, float offset,
                           float *e_dist, float *dL_drot, float *dL_dtrans);

/* Upper-level descent of the bilevel problem (Eq. 4-6 with the QPs of
 * Eq. 7-9) for floating hands on analytic objects. */
typedef struct {
    int iters;        /* gradient steps, >= 0                              */
    float w_qp;       /* weight of E_g = sum_j Q_j                         */
    float w_dist;     /* weight of E^c_d (see bodex_qp_pose_gradient)      */
    float radius;     /* fingertip sphere radius alpha                     */
    float offset;     /* distance reduction delta (pre-grasp)              */
    float step_rot;   /* eta_R: R <- Exp(-eta_R dL/domega) R               */
    float step_trans; /* eta_T: T <- T - eta_T dL/dT                       */
} bodex_descent;

/* `iters` steps of gradient descent on L = w_qp E_g + w_dist E^c_d over the
 * hand pose: per step, the contacts of the current pose (as
 * bodex_qp_contact_query), the QPs of every wrench at those contacts (as
 * bodex_qp_solve with the handle's parameters; from the second step on the
 * ADMM warm-starts from the previous step's state), the QP gradient (as
 * bodex_qp_backward with dL/dE_g = w_qp), the pose gradient (as
 * bodex_qp_pose_gradient) and the update of hand->hand_rot / hand_trans in
 * place.  `qp` gives the QP side: contact_count and wrench_offset (HOST), mu,
 * wrench_dir; its points and normals must be NULL (the library writes the
 * contacts into its workspace), and hand->contact_count must be NULL (the
 * counts are qp->contact_count); hand->m must equal the handle's m_max.
 * `out` receives the QP results of the last step and holds the state (its
 * state pointers may be NULL: the library's workspace); the first step
 * warm-starts only with BODEX_F_WARM_START.  loss_trace: optional device
 * [iters][G], L of each grasp at the pose before each step.  Everything is
 * enqueued on the handle's stream.  Errors: EINVAL, EUNSUP, EINFEAS,
 * EBUDGET, EHIP. */
int bodex_qp_descend(bodex_qp_t *h, const bodex_hand *hand,
                     const bodex_batch *qp, const bodex_descent *d,
                     bodex_result *out, float *loss_trace);

#ifdef __cplusplus
}
#endif
#endif /* BODEX_QP_H */
