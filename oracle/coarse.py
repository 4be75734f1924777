"""FP64 oracle of the step before the QP on analytic objects: a floating hand,
the nearest-point query on an ellipsoid (a sphere when the semi-axes are
equal), the coarse-stage distance energy and one upper-level descent step
(arXiv 2412.16490, Sec. IV-B and the coarse stage of Sec. IV-C).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

Per grasp: a hand pose (R, T) (a floating base with rigid fingers, so every
fingertip shares the root transform), fingertip sphere centres c_{i,l} in the
hand frame and an object, the solid ellipsoid sum_k (x_k / a_k)^2 <= 1 centred
at the origin of the world frame.

* c_{i,w} = R c_{i,l} + T (Sec. IV-B, forward kinematics of a floating hand).
* Nearest point p_i of the object's surface to c_{i,w}, its inward unit
  normal n_i and the signed distance d_i (positive outside).  With
  D = diag(a_k^2), every stationary point of |c - p|^2 on the surface is
  p = D (D + tI)^{-1} c for a root t of
      F(t) = sum_k a_k^2 c_k^2 / (a_k^2 + t)^2 - 1,
  and the nearest one is the root above -min_k a_k^2, where F decreases
  monotonically; it is bracketed by [-a0^2 + a0 |c_0|, -a0^2 + |a o c|] (axis
  0 of the smallest semi-axis) and found here by bisection to the last bit,
  in the shifted variable u = t + a0^2.
  Points with c_0 = 0 inside the object may have two nearest points (the
  ellipsoid's medial ridge): F stays negative above -a0^2, and the nearest
  point has p_k = a_k^2 c_k / (a_k^2 - a0^2) off axis 0 and the p_0 >= 0 that
  puts it on the surface.  The centre of a sphere is the extreme case; there
  the query returns p = a0 e_0.
* Coarse distance energy E^c_d = sum_i (|c_{i,w} - p_i| - alpha - delta)^2
  (Sec. IV-C; alpha the fingertip sphere's radius, delta the distance
  reduction of the pre-grasp stage, Sec. IV-D).  Its derivative with respect
  to c is u^T (I - dp/dc) with u = (c - p) / |c - p| (u = -n, the outward
  normal, when c lies on the surface).  Option signed=True: the signed
  distance d_i in place of |c_{i,w} - p_i| (a fingertip inside the object is
  then pushed out instead of being held at distance alpha inside).
* The derivative of the query: the paper approximates it by finite
  differences (its object is a mesh); on an analytic surface the exact
  Jacobian follows from the implicit function theorem applied to F(t, c) = 0:
      dt/dc = D M^2 c / (c^T D M^3 c),       M = (D + tI)^{-1},
      dp/dc = D M - D M^2 c (dt/dc)^T,
      n = -g / |g|,  g = M c,   dn/dc = -(I - g g^T / |g|^2) (M - M^2 c (dt/dc)^T) / |g|,
      dd/dc = -n^T.
  The tests pin it against central finite differences of the query itself.
* Upper-level loss L = w_qp sum_j Q_j + w_dist E^c_d (the QP energy of
  Eq. 3 plus the coarse distance energy; the robot-specific energies are not
  part of this path).  Per fingertip
      g_i = (dp/dc)^T dL/dp_i + (dn/dc)^T dL/dn_i + w_dist 2 r_i (dr_i/dc)^T,
  with r_i = |c_{i,w} - p_i| - alpha - delta (or d_i - alpha - delta),
  dL/dT = sum_i g_i and, for the rotation R(omega) = Exp(omega) R perturbed
  by a world-frame rotation vector, dL/domega = sum_i (R c_{i,l}) x g_i.
* Descent step: T <- T - eta_T dL/dT, R <- Exp(-eta_R dL/domega) R, with Exp
  the Rodrigues formula, which keeps R a rotation.
"""
from __future__ import annotations

import numpy as np

import oracle as _qp


def _axis0(a, c):
    """Axis of the smallest semi-axis; among equal ones the largest |c_k|."""
    amin = a.min()
    cand = [k for k in range(3) if a[k] == amin]
    return max(cand, key=lambda k: abs(c[k]))


def _root(a, c):
    """The root of F above -a0^2 by bisection, as u = t + a0^2 (so that the
    smallest denominator a0^2 + t = u carries no cancellation); returns
    (u, ridge) with ridge True when F < 0 on the whole interval (u = 0)."""
    a2 = a * a
    k0 = _axis0(a, c)
    off = a2 - a2[k0]  # a_k^2 - a0^2 >= 0, exact for k0
    lo = a[k0] * abs(c[k0])
    hi = np.sqrt(np.sum((a * c) ** 2))

    def F(u):
        s = 0.0
        for k in range(3):
            if c[k] != 0.0:
                s += (a[k] * c[k] / (off[k] + u)) ** 2
        return s - 1.0

    if c[k0] == 0.0:
        # F has no pole at u = 0: a root above it exists only if F > 0 there
        # (every axis as small as axis 0 has c_k = 0, see _axis0)
        if F(0.0) <= 0.0:
            return 0.0, True
        lo = 0.0
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if F(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi), False


def nearest_point(c, a):
    """Nearest surface point p, inward unit normal n, signed distance d (> 0
    outside) and the multiplier t, for a point c and semi-axes a (FP64)."""
    c = np.asarray(c, np.float64)
    a = np.asarray(a, np.float64)
    a2 = a * a
    k0 = _axis0(a, c)
    if not np.any(c):
        p = np.zeros(3)
        p[k0] = a[k0]
        n = np.zeros(3)
        n[k0] = -1.0
        return p, n, -a[k0], -a2[k0]
    u, ridge = _root(a, c)
    den = (a2 - a2[k0]) + u  # a_k^2 + t
    if ridge:
        p = np.zeros(3)
        for k in range(3):
            if k != k0:
                p[k] = a2[k] * c[k] / den[k]
        rest = np.sum((p / a) ** 2)
        p[k0] = a[k0] * np.sqrt(max(0.0, 1.0 - rest))
    else:
        p = a2 * c / den
    gp = p / a2  # half the gradient of sum (x/a)^2 at p: outward
    n = -gp / np.linalg.norm(gp)
    inside = np.sum((c / a) ** 2) < 1.0
    dist = np.linalg.norm(c - p)
    return p, n, (-dist if inside else dist), u - a2[k0]


def query_jacobian(c, a):
    """(dp/dc, dn/dc, dd/dc) at c; zero where the nearest point is not unique
    or not differentiable (the medial ridge, the centre)."""
    c = np.asarray(c, np.float64)
    a = np.asarray(a, np.float64)
    if not np.any(c):
        return np.zeros((3, 3)), np.zeros((3, 3)), np.zeros(3)
    p, n, d, t = nearest_point(c, a)
    a2 = a * a
    k0 = _axis0(a, c)
    den = (a2 - a2[k0]) + (t + a2[k0])
    if np.any(den <= 0.0):
        return np.zeros((3, 3)), np.zeros((3, 3)), np.zeros(3)
    M = 1.0 / den
    g = M * c
    dF_dc = a2 * M * M * c            # = (1/2) dF/dc
    dF_dt = np.sum(a2 * M ** 3 * c * c)  # = -(1/2) dF/dt
    dt_dc = dF_dc / dF_dt
    Jp = np.diag(a2 * M) - np.outer(a2 * M * M * c, dt_dc)
    Jg = np.diag(M) - np.outer(M * M * c, dt_dc)
    gn = np.linalg.norm(g)
    gh = g / gn
    Jn = -(np.eye(3) - np.outer(gh, gh)) @ Jg / gn
    return Jp, Jn, -n


def hand_points(R, T, cl):
    """c_{i,w} = R c_{i,l} + T for every fingertip: R [G,3,3], T [G,3], cl [G,M,3]."""
    R = np.asarray(R, np.float64)
    T = np.asarray(T, np.float64)
    cl = np.asarray(cl, np.float64)
    return np.einsum("gij,gmj->gmi", R, cl) + T[:, None, :]


def contact_query(R, T, cl, axes, counts=None):
    """Points, inward normals [G,M,3] and signed distances [G,M] of every live
    fingertip (padding fingertips: zeros)."""
    cw = hand_points(R, T, cl)
    G, M = cw.shape[:2]
    counts = np.full(G, M) if counts is None else np.asarray(counts)
    P = np.zeros((G, M, 3))
    N = np.zeros((G, M, 3))
    D = np.zeros((G, M))
    ax = np.asarray(axes, np.float64)
    for g in range(G):
        for i in range(int(counts[g])):
            P[g, i], N[g, i], D[g, i], _ = nearest_point(cw[g, i], ax[g])
    return P, N, D


def rodrigues(w):
    """Exp of the skew matrix of the rotation vector w (Rodrigues' formula)."""
    w = np.asarray(w, np.float64)
    th = np.linalg.norm(w)
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if th == 0.0:
        return np.eye(3)
    return np.eye(3) + np.sin(th) / th * K + (1.0 - np.cos(th)) / th ** 2 * (K @ K)


def dist_term(c, p, n, d, Jp, signed=False):
    """(distance, its gradient with respect to c) of one fingertip for E^c_d:
    |c - p| and u^T (I - dp/dc) (the paper's form), or with signed=True the
    signed distance d and dd/dc = -n."""
    if signed:
        return d, -np.asarray(n, np.float64)
    v = np.asarray(c, np.float64) - np.asarray(p, np.float64)
    nv = np.linalg.norm(v)
    u = v / nv if nv > 0.0 else -np.asarray(n, np.float64)
    return nv, (np.eye(3) - Jp).T @ u


def pose_gradient(R, T, cl, axes, dLdp=None, dLdn=None, w_dist=0.0, radius=0.0, offset=0.0, counts=None,
                  signed=False):
    """(E^c_d [G], dL/domega [G,3], dL/dT [G,3]) for
    L = (the caller's loss through p, n) + w_dist E^c_d."""
    R = np.asarray(R, np.float64)
    cl = np.asarray(cl, np.float64)
    cw = hand_points(R, T, cl)
    G, M = cw.shape[:2]
    counts = np.full(G, M) if counts is None else np.asarray(counts)
    ax = np.asarray(axes, np.float64)
    E = np.zeros(G)
    dw = np.zeros((G, 3))
    dT = np.zeros((G, 3))
    for g in range(G):
        for i in range(int(counts[g])):
            p, n, d, _ = nearest_point(cw[g, i], ax[g])
            Jp, Jn, Jd = query_jacobian(cw[g, i], ax[g])
            dist, Jdist = dist_term(cw[g, i], p, n, d, Jp, signed)
            if not np.any(Jd):  # no derivative of the query here (ridge, centre)
                Jdist = np.zeros(3)
            r = dist - radius - offset
            E[g] += r * r
            gi = 2.0 * w_dist * r * Jdist
            if dLdp is not None:
                gi = gi + Jp.T @ np.asarray(dLdp[g, i], np.float64)
            if dLdn is not None:
                gi = gi + Jn.T @ np.asarray(dLdn[g, i], np.float64)
            dT[g] += gi
            dw[g] += np.cross(R[g] @ cl[g, i], gi)
    return E, dw, dT


def descent_step(R, T, dw, dT, step_rot, step_trans):
    """T - eta_T dL/dT and Exp(-eta_R dL/domega) R."""
    R = np.asarray(R, np.float64)
    Rn = np.stack([rodrigues(-step_rot * np.asarray(dw[g], np.float64)) @ R[g] for g in range(R.shape[0])])
    return Rn, np.asarray(T, np.float64) - step_trans * np.asarray(dT, np.float64)


def _solve_qps(counts, woff, P, N, mu, wrench, prm, cone):
    """The QPs at the contacts: the pyramid oracle, or with cone=True the
    circular-cone oracle (the same kappa, beta, eps, fmax and gamma)."""
    if not cone:
        return _qp.solve_batch(counts, woff, P, N, mu, wrench, prm)
    from oracle import cone as _cone
    prm = prm or _qp.params()
    return _cone.solve_batch(counts, woff, P, N, mu, wrench, kappa=prm.kappa, beta=prm.beta, eps=prm.eps,
                             fmax=prm.fmax, gamma=prm.gamma)


def loss(R, T, cl, axes, counts, woff, mu, wrench, w_qp=1.0, w_dist=0.0, radius=0.0, offset=0.0, prm=None,
         cone=False, signed=False):
    """L per grasp at the pose (R, T), with the pyramid QP oracle (or the
    circular-cone one); also the contacts and the QP solution."""
    P, N, D = contact_query(R, T, cl, axes, counts)
    res = _solve_qps(counts, woff, P, N, mu, wrench, prm, cone)
    live = np.arange(P.shape[1])[None, :] < np.asarray(counts)[:, None]
    dist = D if signed else np.linalg.norm(hand_points(R, T, cl) - P, axis=2)
    Ec = np.sum(np.where(live, (dist - radius - offset) ** 2, 0.0), axis=1)
    return w_qp * res["energy"] + w_dist * Ec, P, N, res


def descend(R, T, cl, axes, counts, woff, mu, wrench, iters, w_qp=1.0, w_dist=0.0, radius=0.0, offset=0.0,
            step_rot=0.0, step_trans=0.0, prm=None, cone=False, signed=False):
    """`iters` upper-level gradient steps; returns the final (R, T) and the
    loss [iters, G] at each pose before its step.  The QP gradient is
    Danskin's (a function of the optimal forces only), so the same chain rule
    serves the pyramid and the circular cone."""
    R = np.asarray(R, np.float64).copy()
    T = np.asarray(T, np.float64).copy()
    trace = []
    for _ in range(iters):
        L, P, N, res = loss(R, T, cl, axes, counts, woff, mu, wrench, w_qp, w_dist, radius, offset, prm, cone,
                            signed)
        trace.append(L)
        G = P.shape[0]
        dP, dN = _qp.grad_batch(counts, woff, P, N, wrench, res["forces"], we=np.full(G, float(w_qp)), prm=prm)
        _, dw, dT = pose_gradient(R, T, cl, axes, dP, dN, w_dist, radius, offset, counts, signed)
        R, T = descent_step(R, T, dw, dT, step_rot, step_trans)
    return R, T, np.array(trace)
