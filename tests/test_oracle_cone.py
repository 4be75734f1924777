"""Pins of the circular-cone oracle (Eq. 7-9 with the cone of Eq. 1) against
what the mathematics fixes, independently of the barrier method it uses:

* one contact at the object's origin: G = [R; 0] with R orthonormal, so the
  QP is (1 + eps) |f - w|^2 + const with w = R^T t_f / (1 + eps) and f* is the
  Euclidean projection of w onto the truncated cone -- computed here as the
  closest point of a triangle in the (axial, radial) half-plane, one case per
  region of the plane (inside, cone surface, apex, normal bound, rim);
* contacts whose desired wrench only pulls: f* = 0 and Q* = beta^2 |t|^2
  (the gradient at 0 lies in the polar cone);
* the sandwich: the inscribed 8-facet pyramid (mu cos(pi/8) facets) is inside
  the cone, the circumscribed one (facets tangent to the cone) contains it,
  so Q*_inscribed >= Q*_cone >= Q*_circumscribed -- both from the active-set
  pyramid oracle, which shares nothing with this one;
* relaxation: where the optimum of the problem without the cone (bounded
  least squares, scipy's BVLS) satisfies the cone, it is the optimum;
* the projected-gradient fixed point f = Pi(f - a grad Q(f)) (optimality);
* weak duality: any dual point in the dual cone bounds Q* from below;
* feasibility of the returned point.
"""
import numpy as np
import pytest

import oracle
from oracle import cone
from paper_2412_16490_amd import workload as wl

import cone_certificate as cc

EPS = 1e-6
C8 = np.cos(np.pi / 8)


_project_contact = cc.project_contact


def _frame(n):
    G = oracle.grasp_matrix(np.zeros((1, 3)), n[None, :], 20.0)
    return G[:3, :3]  # columns nhat, d, e


@pytest.mark.parametrize("w", [
    (0.5, 0.1, -0.05),     # inside
    (0.3, 0.6, 0.2),       # above the cone surface
    (-0.4, 0.1, 0.0),      # in the polar cone: the apex
    (-0.2, 0.02, 0.01),    # apex
    (1.7, 0.1, 0.05),      # beyond the normal bound
    (1.5, 0.9, -0.6),      # beyond the rim
    (0.9, 0.3, 0.1),       # near the rim, on the surface side
])
def test_single_contact_at_origin_is_a_projection(w):
    rng = np.random.default_rng(3)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    mu = 0.5
    w = np.asarray(w, float)
    R = _frame(n)
    t = np.concatenate([(1 + EPS) * (R @ w), [0.1, -0.2, 0.05]])
    G = oracle.grasp_matrix(np.zeros((1, 3)), n[None, :], 20.0)
    r = cone.solve(G, np.array([mu]), t, eps=EPS)
    f_exp = _project_contact(w, mu, 1.0)
    np.testing.assert_allclose(r["f"], f_exp, atol=1e-8)
    q_exp = np.sum((G @ f_exp - t) ** 2) + EPS * f_exp @ f_exp
    assert r["q"] == pytest.approx(q_exp, rel=1e-11, abs=1e-14)


def test_pulling_wrench_gives_zero_force():
    rng = np.random.default_rng(5)
    n0 = np.array([0.3, -0.5, 0.8])
    n0 /= np.linalg.norm(n0)
    m = 4
    N = n0 + 0.1 * rng.standard_normal((m, 3))
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    mu = np.full(m, 0.6)
    ang = np.arccos(np.clip(N @ n0, -1, 1))
    assert np.all(np.cos(ang) >= mu * np.sin(ang))  # -G_i^T t in the dual cone
    G = oracle.grasp_matrix(np.zeros((m, 3)), N, 20.0)
    t = np.concatenate([-n0, np.zeros(3)])
    r = cone.solve(G, mu, t, eps=EPS)
    assert np.abs(r["f"]).max() < 1e-9
    assert r["q"] == pytest.approx(1.0, abs=1e-9)


def _grasps(n=6, seed=16491):
    b = wl.config(1, n)
    out = []
    for g in range(b.n_grasps):
        m = b.counts[g]
        G = oracle.grasp_matrix(b.points[g, :m].astype(float), b.normals[g, :m].astype(float), 20.0)
        for j in range(3):
            out.append((G, b.mu[g, :m].astype(float), b.wrench[b.woff[g] + j].astype(float)))
    return out


@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_sandwich_between_inscribed_and_circumscribed_pyramids(gamma):
    for G, mu, t in _grasps():
        q_cone = cone.solve(G, mu, t, gamma=gamma)["q"]
        prm = oracle.params(gamma=gamma)
        q_in = oracle.qp_solve(G, mu, t, prm)[2]
        q_out = oracle.qp_solve(G, mu / C8, t, prm)[2]
        assert q_out - 1e-11 <= q_cone <= q_in + 1e-11, (q_out, q_cone, q_in)


@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_returned_point_is_feasible(gamma):
    for G, mu, t in _grasps(4):
        f = cone.solve(G, mu, t, gamma=gamma)["f"].reshape(-1, 3)
        assert np.all(np.hypot(f[:, 1], f[:, 2]) <= mu * f[:, 0] + 1e-12)
        assert np.all(f[:, 0] <= 1.0 + 1e-12)
        assert f[:, 0].sum() >= gamma - 1e-12


@pytest.mark.parametrize("m,mu_v", [(1, 1.5), (2, 3.0)])
def test_relaxation_optimum_that_is_feasible_is_the_optimum(m, mu_v):
    # wrenches that forces inside the cone produce: where the optimum without
    # the cone (bounded least squares, scipy's BVLS) lies inside the cone, it
    # is the optimum with it
    sp = pytest.importorskip("scipy.optimize")
    rng = np.random.default_rng(11)
    hits = 0
    for k in range(40):
        p, n = wl.ellipsoid_contacts(rng, 1, m)
        G = oracle.grasp_matrix(p[0].astype(float), n[0].astype(float), 20.0)
        mu = np.full(m, mu_v)
        f_in = np.zeros(3 * m)
        f_in[0::3] = rng.uniform(0.2, 0.8, m)
        ang = rng.uniform(0, 2 * np.pi, m)
        rad = rng.uniform(0, 0.4, m) * 0.6 * f_in[0::3]
        f_in[1::3], f_in[2::3] = rad * np.cos(ang), rad * np.sin(ang)
        t = G @ f_in
        A = np.vstack([G, np.sqrt(EPS) * np.eye(3 * m)])
        rhs = np.concatenate([t, np.zeros(3 * m)])
        lo = np.full(3 * m, -np.inf)
        hi = np.full(3 * m, np.inf)
        lo[0::3] = 0.0
        hi[0::3] = 1.0
        res = sp.lsq_linear(A, rhs, bounds=(lo, hi), method="bvls", tol=1e-15)
        f = res.x.reshape(m, 3)
        if np.all(np.hypot(f[:, 1], f[:, 2]) < mu * f[:, 0] * (1 - 1e-6)):
            hits += 1
            r = cone.solve(G, mu, t, eps=EPS)
            q_rel = np.sum((G @ res.x - t) ** 2) + EPS * res.x @ res.x
            assert r["q"] == pytest.approx(q_rel, rel=1e-9, abs=1e-13)
            np.testing.assert_allclose(r["f"], res.x, atol=1e-7)
    assert hits >= 20


def test_projected_gradient_fixed_point():
    # the barrier leaves a weakly active constraint (small multiplier lam) at
    # a distance of about 1 / (t_b lam) inside the boundary: 1e-7 covers
    # multipliers down to ~1e-7 at the final t_b
    for G, mu, t in _grasps(5):
        m = mu.shape[0]
        r = cone.solve(G, mu, t)
        f = r["f"]
        P = 2 * (G.T @ G + EPS * np.eye(3 * m))
        grad = P @ f - 2 * G.T @ t
        a = 1.0 / np.linalg.eigvalsh(P)[-1]
        y = f - a * grad
        fp = np.concatenate([_project_contact(y[3 * i:3 * i + 3], mu[i], 1.0) for i in range(m)])
        assert np.abs(fp - f).max() <= 1e-7


@pytest.mark.parametrize("gamma,beta", [(0.5, 1.0), (1.0, 0.0), (2.0, 1.0)])
def test_projected_gradient_fixed_point_with_the_normal_sum_row(gamma, beta):
    for G, mu, t in _grasps(4):
        r = cone.solve(G, mu, t, gamma=gamma, beta=beta)
        assert cc.fixed_point_residual(G, mu, t, r["f"], beta=beta, gamma=gamma) <= 1e-7
        assert cc.fixed_point_residual(G, mu, t, r["f"], beta=beta, gamma=gamma, step=1e6) <= 1e-5


def test_the_certificate_rejects_a_perturbed_point():
    for G, mu, t in _grasps(2):
        f = cone.solve(G, mu, t, gamma=0.5)["f"]
        worst = max(cc.fixed_point_residual(G, mu, t, f + 1e-4 * np.eye(len(f))[k], gamma=0.5) for k in range(len(f)))
        assert worst > 1e-6
        # the sum row: dropping it from the certificate is noticed when it binds
        f2 = cone.solve(G, mu, t, gamma=2.0, beta=0.0)["f"]
        assert cc.fixed_point_residual(G, mu, t, f2, beta=0.0, gamma=2.0) <= 1e-7
        assert cc.fixed_point_residual(G, mu, t, f2, beta=0.0, gamma=0.0, step=1e6) > 1e-3


def test_unit_step_is_blind_to_internal_forces_and_fista_is_not():
    # an error along an internal-force direction (G v = 0: only the 2 eps
    # curvature sees it) passes the unit-step fixed point; the distance to
    # the accelerated projected-gradient limit sees it
    for G, mu, t in _grasps(2)[::3]:
        f = cone.solve(G, mu, t)["f"]
        v = np.linalg.svd(G)[2][-1]  # a null vector of G (3 m > 6)
        fb = f + 1e-3 * v
        if np.all(np.hypot(fb[1::3], fb[2::3]) < mu * fb[0::3]) and np.all(fb[0::3] < 1.0):
            assert cc.fixed_point_residual(G, mu, t, fb) <= 1e-7
        assert cc.fixed_point_residual(G, mu, t, fb, step=1e6) > 1e-4
        assert np.abs(cc.fista(G, mu, t, iters=4000) - fb).max() > 5e-4


@pytest.mark.parametrize("w,gamma,beta,iters,tol", [(503, 0.0, 1.0, 10000, 1e-7), (103, 0.0, 1.0, 10000, 1e-7),
                                                    (285, 0.0, 1.0, 10000, 1e-7), (72, 0.0, 1.0, 60000, 1e-6),
                                                    (45, 1.0, 1.0, 3000, 1e-7), (117, 1.0, 1.0, 3000, 1e-7)])
def test_forces_match_the_projected_gradient_limit(w, gamma, beta, iters, tol):
    # forces pinned by a method that shares nothing with the barrier, on the
    # QPs of the uneven workload's first 40 grasps whose barrier points sit
    # closest to a weakly active cone (largest large-step residual), a
    # force-closure QP (Q* ~ eps |f|^2: the minimiser is fixed only by the
    # 2 eps curvature, so the first-order method needs longer), and QPs whose
    # normal-sum row binds
    b = wl.config(3, 40)
    g = int(np.searchsorted(b.woff, w, side="right") - 1)
    m = int(b.counts[g])
    G = oracle.grasp_matrix(b.points[g, :m].astype(float), b.normals[g, :m].astype(float), 20.0)
    mu, t = b.mu[g, :m].astype(float), b.wrench[w].astype(float)
    f = cone.solve(G, mu, t, gamma=gamma, beta=beta)["f"]
    assert np.abs(f - cc.fista(G, mu, t, beta=beta, gamma=gamma, iters=iters)).max() <= tol


def test_weak_duality_lower_bound():
    # a coarser barrier run gives a dual point; its dual value bounds Q*
    # from below and is close to it
    for G, mu, t in _grasps(4):
        m = mu.shape[0]
        q_star = cone.solve(G, mu, t)["q"]
        r = cone.solve(G, mu, t, gap=1e-6)
        S, nu, _ = r["dual"]
        assert np.all(S[:, 0] >= mu * np.hypot(S[:, 1], S[:, 2]) - 1e-15) and np.all(nu >= 0)
        P = 2 * (G.T @ G + EPS * np.eye(3 * m))
        q = -2 * G.T @ t
        c = S.copy()
        c[:, 0] -= nu
        c = c.reshape(-1)
        D = t @ t - 0.5 * (c - q) @ np.linalg.solve(P, c - q) - nu.sum()
        assert D <= q_star + 1e-12
        assert q_star - D <= 1e-5


def test_a_wrong_friction_coefficient_fails_the_projection_pin():
    # the projection pin is sensitive to a 1% error in mu
    n = np.array([0.0, 0.6, 0.8])
    w = np.array([0.3, 0.6, 0.2])
    G = oracle.grasp_matrix(np.zeros((1, 3)), n[None, :], 20.0)
    t = np.concatenate([(1 + EPS) * (_frame(n) @ w), np.zeros(3)])
    f_bad = cone.solve(G, np.array([0.5 * 1.01]), t, eps=EPS)["f"]
    assert np.abs(f_bad - _project_contact(w, 0.5, 1.0)).max() > 1e-4
