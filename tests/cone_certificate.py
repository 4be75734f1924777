"""Optimality certificate for circular-cone QP answers (Eq. 7-9 with the cone
of Eq. 1), independent of how they were computed: a point f minimises the
convex objective Q over the feasible set C exactly when it is a fixed point of
the projected-gradient map f = Pi_C(f - a grad Q(f)) for any a > 0.

Pi_C has a closed form per contact (the cone truncated at fmax is, in the
(axial, radial) half-plane of the contact's force, the triangle (0,0),
(fmax,0), (fmax, mu fmax), so its projection is the closest point of that
triangle).  With the normal-sum row sum_i f_i1 >= gamma the set is the product
of the contacts' cones cut by a half-space a.f >= gamma; its projection is
Pi(y + nu a) for the nu >= 0 at which the cut holds with equality (or nu = 0
when the product projection already satisfies it), found by Brent's method on
the bracket [0, hi] since a.Pi(y + nu a) is nondecreasing in nu.
"""
import numpy as np
from scipy.optimize import brentq


def _closest_on_segment(p, a, b):
    d = b - a
    s = np.clip((p - a) @ d / (d @ d), 0.0, 1.0)
    return a + s * d


def triangle_projection(a, r, mu, fmax):
    """Closest point to (a, r) in the triangle (0,0), (fmax, 0), (fmax, mu fmax)."""
    p = np.array([a, r])
    O, B, V = np.array([0.0, 0.0]), np.array([fmax, 0.0]), np.array([fmax, mu * fmax])
    inside = r <= mu * a + 1e-300 and a <= fmax and r >= 0
    if inside:
        return p
    cands = [_closest_on_segment(p, O, B), _closest_on_segment(p, B, V), _closest_on_segment(p, O, V)]
    return min(cands, key=lambda c: np.sum((c - p) ** 2))


def project_contact(f, mu, fmax):
    rt = np.hypot(f[1], f[2])
    a2, r2 = triangle_projection(f[0], rt, mu, fmax)
    if rt > 0:
        return np.array([a2, f[1] * r2 / rt, f[2] * r2 / rt])
    return np.array([a2, 0.0, 0.0])


def _project_all(y, mu, fmax):
    """project_contact applied to every contact of y (vectorised, the same
    case analysis: the point itself when inside, else the closest of the
    triangle's three edges)."""
    f = y.reshape(-1, 3)
    a, rt = f[:, 0], np.hypot(f[:, 1], f[:, 2])
    best_a, best_r = a.copy(), rt.copy()
    best_d = np.full(a.shape, np.inf)
    for (oa, orr), (da, dr) in (((0.0, 0.0), (fmax, 0.0 * mu)), ((fmax, 0.0 * mu), (0.0, mu * fmax)),
                                ((0.0, 0.0), (fmax, mu * fmax))):
        s = np.clip(((a - oa) * da + (rt - orr) * dr) / (da * da + dr * dr), 0.0, 1.0)
        ca, cr = oa + s * da, orr + s * dr
        d = (ca - a) ** 2 + (cr - rt) ** 2
        take = d < best_d
        best_a, best_r, best_d = np.where(take, ca, best_a), np.where(take, cr, best_r), np.where(take, d, best_d)
    inside = (rt <= mu * a + 1e-300) & (a <= fmax) & (rt >= 0)
    best_a, best_r = np.where(inside, a, best_a), np.where(inside, rt, best_r)
    scale = np.where(rt > 0, best_r / np.where(rt > 0, rt, 1.0), 0.0)
    return np.stack([best_a, f[:, 1] * scale, f[:, 2] * scale], axis=1).reshape(-1)


def project_set(y, mu, fmax, gamma=0.0):
    mu = np.asarray(mu, np.float64)
    f = _project_all(y, mu, fmax)
    if gamma <= 0.0 or f[0::3].sum() >= gamma:
        return f
    a = np.zeros(len(y))
    a[0::3] = 1.0
    def excess(nu):
        return _project_all(y + nu * a, mu, fmax)[0::3].sum() - gamma

    hi = 1.0
    while excess(hi) < 0.0:
        hi *= 2.0
    nu = brentq(excess, 0.0, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=200)
    f = _project_all(y + nu * a, mu, fmax)
    return f if f[0::3].sum() >= gamma else _project_all(y + np.nextafter(nu, np.inf) * a, mu, fmax)


def fixed_point_residual(G, mu, t, f, beta=1.0, eps=1e-6, fmax=1.0, gamma=0.0, step=1.0):
    """max |Pi(f - a grad Q(f)) - f| with a = step / lambda_max(P).

    With step = 1 the map is a contraction and the residual certifies the
    objective; along internal-force directions (null space of G, curvature
    2 eps) it moves a point by only ~2 eps / lambda_max of its error, so a
    large step (step = 1e6 takes a near 1 / (2 eps)) is what makes the
    residual bound the force error there."""
    m = len(mu)
    P = 2 * (G.T @ G + eps * np.eye(3 * m))
    grad = P @ f - 2 * beta * G.T @ t
    a = step / np.linalg.eigvalsh(P)[-1]
    return float(np.abs(project_set(f - a * grad, mu, fmax, gamma) - f).max())


def fista(G, mu, t, beta=1.0, eps=1e-6, fmax=1.0, gamma=0.0, iters=10000):
    """The minimiser by accelerated projected gradient (FISTA with the
    closed-form projection, restarted whenever the momentum step points
    uphill), from f = 0: a method that shares nothing with a barrier
    method, whose limit is the minimiser whatever the curvature along
    internal-force directions (10,000 iterations reach it to rounding on
    the 4- and 5-contact workloads)."""
    m = len(mu)
    P = 2 * (G.T @ G + eps * np.eye(3 * m))
    q = -2 * beta * G.T @ t
    L = np.linalg.eigvalsh(P)[-1]
    x = np.zeros(3 * m)
    y = x.copy()
    tk = 1.0
    for _ in range(iters):
        xn = project_set(y - (P @ y + q) / L, mu, fmax, gamma)
        if (y - xn) @ (xn - x) > 0:
            tk = 1.0
        tn = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * tk * tk))
        y = xn + (tk - 1.0) / tn * (xn - x)
        x, tk = xn, tn
    return x


def certify_batch(grasp_matrix, b, forces, qps, beta=1.0, gamma=0.0, eps=1e-6, fmax=1.0, kappa=20.0,
                  steps=(1.0,)):
    """Largest fixed-point residual over the listed QPs of a CSR batch, one
    per step scale; forces [W][3 m_max]."""
    woff = np.asarray(b.woff)
    gidx = np.searchsorted(woff, qps, side="right") - 1
    cache = {}
    worst = np.zeros(len(steps))
    for w, g in zip(qps, gidx):
        m = int(b.counts[g])
        if g not in cache:
            cache[g] = grasp_matrix(b.points[g, :m].astype(np.float64), b.normals[g, :m].astype(np.float64), kappa)
        for k, st in enumerate(steps):
            worst[k] = max(worst[k], fixed_point_residual(cache[g], b.mu[g, :m].astype(np.float64),
                                                          b.wrench[w].astype(np.float64), forces[w, :3 * m], beta,
                                                          eps, fmax, gamma, st))
    return worst
