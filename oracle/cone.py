"""FP64 oracle of the contact-force QP with the exact circular friction cone
(arXiv 2412.16490: Eq. 7-9 with the cone of Eq. 1, the quadratically
constrained form that Sec. IV-A replaces by the 8-facet pyramid).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

For one grasp with grasp matrix G (Eq. 2, torque rows scaled by kappa) and
one desired wrench direction t:

    Q* = min_f ||G f - beta t||^2 + eps ||f||^2
         s.t. per contact i:  ||(f_i2, f_i3)|| <= mu_i f_i1,  f_i1 <= fmax
              sum_i f_i1 >= gamma            (only when gamma > 0)

(f_i1 >= 0 is implied by the cone.)  The objective is strictly convex, so f*
is unique.  Method: the barrier method (Boyd & Vandenberghe, Convex
Optimization, Sec. 11.3): minimise t_b Q(f) + phi(f) by Newton's method with
a backtracking line search that keeps f strictly feasible, for t_b growing
geometrically until the duality-gap bound nu / t_b is below `gap` (nu = 2
per cone + 1 per bound + 1 for the sum row); each centering stops when half
the squared Newton decrement is below `newton_tol` or below the rounding
level of the merit value t_b Q + phi (the line search cannot resolve less).
The Newton system is solved after symmetric diagonal scaling; should it still
be singular to working precision, the iteration stops at the current point
(t_barrier reports how far it got).  The barrier is
    phi(f) = - sum_i log(mu_i^2 f_i1^2 - f_i2^2 - f_i3^2) - sum_i log(fmax - f_i1)
             - log(sum_i f_i1 - gamma).
At the end the barrier also gives a dual point (per-contact cone multipliers
s_i in the dual cone, bound multipliers, the sum-row multiplier) whose dual
value certifies Q* from below; `solve` returns it with the primal point.
"""
from __future__ import annotations

import numpy as np

from oracle import grasp_matrix


def _barrier(f, mu, fmax, gamma, use_gam):
    """phi, its gradient and Hessian; None when f is not strictly feasible."""
    m = mu.shape[0]
    F = f.reshape(m, 3)
    s = mu ** 2 * F[:, 0] ** 2 - F[:, 1] ** 2 - F[:, 2] ** 2
    b = fmax - F[:, 0]
    if np.any(s <= 0) or np.any(F[:, 0] <= 0) or np.any(b <= 0):
        return None
    sg = F[:, 0].sum() - gamma if use_gam else 1.0
    if sg <= 0:
        return None
    phi = -np.sum(np.log(s)) - np.sum(np.log(b)) - (np.log(sg) if use_gam else 0.0)
    g = np.zeros(3 * m)
    H = np.zeros((3 * m, 3 * m))
    for i in range(m):
        ds = np.array([2 * mu[i] ** 2 * F[i, 0], -2 * F[i, 1], -2 * F[i, 2]])
        d2s = np.diag([2 * mu[i] ** 2, -2.0, -2.0])
        sl = slice(3 * i, 3 * i + 3)
        g[sl] += -ds / s[i]
        H[sl, sl] += np.outer(ds, ds) / s[i] ** 2 - d2s / s[i]
        g[3 * i] += 1.0 / b[i]
        H[3 * i, 3 * i] += 1.0 / b[i] ** 2
    if use_gam:
        idx = np.arange(0, 3 * m, 3)
        g[idx] -= 1.0 / sg
        H[np.ix_(idx, idx)] += 1.0 / sg ** 2
    return phi, g, H


def solve(G, mu, t, beta=1.0, eps=1e-6, fmax=1.0, gamma=0.0, gap=1e-13, t0=1.0, growth=20.0,
          newton_tol=1e-14, max_newton=200):
    """Returns dict: f (3m), q (objective), dual (s [m,3], nu [m], lam_g),
    t_barrier, newton (total Newton steps)."""
    G = np.asarray(G, np.float64)
    mu = np.asarray(mu, np.float64)
    t = np.asarray(t, np.float64)
    m = mu.shape[0]
    n = 3 * m
    use_gam = gamma > 0.0
    if use_gam and not gamma < m * fmax:
        raise ValueError("gamma >= m fmax: no strictly feasible point")
    P = 2.0 * (G.T @ G + eps * np.eye(n))
    q = -2.0 * beta * (G.T @ t)

    def Q(f):
        r = G @ f - beta * t
        return r @ r + eps * (f @ f)

    f1 = fmax / 2 if not use_gam else 0.5 * (gamma / m + fmax)
    f = np.zeros(n)
    f[0::3] = f1
    nu = 3 * m + (1 if use_gam else 0)
    tb = t0
    steps = 0
    floor = False
    while True:
        # centering: Newton on tb Q + phi
        for _ in range(max_newton):
            phi, gb, Hb = _barrier(f, mu, fmax, gamma, use_gam)
            grad = tb * (P @ f + q) + gb
            hess = tb * P + Hb
            # symmetric diagonal scaling before the solve (the barrier's
            # diagonal spans many orders of magnitude at large tb)
            sc = 1.0 / np.sqrt(np.diag(hess))
            try:
                d = -sc * np.linalg.solve(hess * np.outer(sc, sc), grad * sc)
            except np.linalg.LinAlgError:
                floor = True  # rounding floor: stop at the current point
                break
            dec2 = -grad @ d
            steps += 1
            val = tb * Q(f) + phi
            # stop when centred, or when the decrement is below what the
            # rounding of the merit value can resolve
            if dec2 / 2 <= max(newton_tol, 64 * np.finfo(float).eps * abs(val)):
                break
            a = 1.0
            while True:
                bn = _barrier(f + a * d, mu, fmax, gamma, use_gam)
                if bn is not None and tb * Q(f + a * d) + bn[0] <= val + 0.25 * a * (grad @ d):
                    break
                a *= 0.5
                if a < 1e-20:
                    break
            if a < 1e-20:
                break
            f = f + a * d
        if floor or nu / tb < gap:
            break
        tb *= growth
    # dual point from the barrier: s_i = -(1/tb) grad of the cone term (in the
    # dual cone ||s_t|| <= s_1 / mu), nu_i = 1 / (tb (fmax - f_i1)),
    # lam_g = 1 / (tb (sum f_1 - gamma))
    F = f.reshape(m, 3)
    s_c = mu ** 2 * F[:, 0] ** 2 - F[:, 1] ** 2 - F[:, 2] ** 2
    S = np.stack([2 * mu ** 2 * F[:, 0], -2 * F[:, 1], -2 * F[:, 2]], axis=1) / (tb * s_c[:, None])
    nub = 1.0 / (tb * (fmax - F[:, 0]))
    lam_g = 1.0 / (tb * (F[:, 0].sum() - gamma)) if use_gam else 0.0
    return {"f": f, "q": Q(f), "dual": (S, nub, lam_g), "t_barrier": tb, "newton": steps}


def solve_batch(counts, woff, p, n, mu, t, kappa=20.0, beta=1.0, eps=1e-6, fmax=1.0, gamma=0.0, qps=None,
                **kw):
    """Every (or the listed) QP of a CSR batch; forces [W][3 m_max] (zero
    padded), objectives [W], energies [G] (over all wrenches of a grasp, only
    when qps is None)."""
    counts = np.asarray(counts)
    woff = np.asarray(woff)
    G_n = counts.shape[0]
    M = p.shape[1]
    W = int(woff[-1])
    qlist = np.arange(W) if qps is None else np.asarray(qps)
    gidx = np.searchsorted(woff, qlist, side="right") - 1
    forces = np.zeros((W, 3 * M))
    qobj = np.full(W, np.nan)
    cache = {}
    for w, g in zip(qlist, gidx):
        m = int(counts[g])
        if g not in cache:
            cache[g] = grasp_matrix(np.asarray(p[g, :m], np.float64), np.asarray(n[g, :m], np.float64), kappa)
        r = solve(cache[g], np.asarray(mu[g, :m], np.float64), np.asarray(t[w], np.float64), beta=beta, eps=eps,
                  fmax=fmax, gamma=gamma, **kw)
        forces[w, :3 * m] = r["f"]
        qobj[w] = r["q"]
    energy = None
    if qps is None:
        energy = np.array([qobj[woff[g]:woff[g + 1]].sum() for g in range(G_n)])
    return {"forces": forces, "qobj": qobj, "energy": energy}
