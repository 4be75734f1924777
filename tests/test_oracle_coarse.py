"""Pins of the coarse-stage oracle on analytic objects (floating hand, nearest
point on an ellipsoid, E^c_d, pose gradient and descent step; Sec. IV-B and
the coarse stage of Sec. IV-C) against what the mathematics fixes:

* spheres: the nearest point, normal and signed distance in closed form;
* ellipsoids: the returned point is on the surface, no point of a dense
  parametric sample of the surface is nearer, and c - p is normal to the
  surface (brute force and first-order optimality), inside and outside;
* the medial ridge and the centre: the distance equals the brute-force minimum;
* the query's Jacobians against central differences of the query itself, and
  the signed distance's gradient is a unit vector;
* the Rodrigues exponential against scipy's rotation-vector conversion;
* the pose gradient against central differences of the whole loss through the
  QP oracle (translation and world-frame rotation vector), and a planted error
  (the normal's Jacobian dropped) fails that check;
* a small descent step lowers the loss by the first-order amount.
"""
import numpy as np
import pytest

import oracle
from oracle import coarse as oc
from paper_2412_16490_amd import workload as wl


def _surface_sample(a, n=400):
    th = np.linspace(0.0, np.pi, n)
    ph = np.linspace(-np.pi, np.pi, 2 * n)
    T, P = np.meshgrid(th, ph, indexing="ij")
    return np.stack([a[0] * np.sin(T) * np.cos(P), a[1] * np.sin(T) * np.sin(P), a[2] * np.cos(T)], -1).reshape(-1, 3)


def _brute_distance(S, a, c):
    """Minimum distance from c to the surface: the best point of the dense
    sample, refined by a Nelder-Mead search over the angles around it."""
    opt = pytest.importorskip("scipy.optimize")
    k = np.argmin(np.linalg.norm(S - c, axis=1))
    q = S[k] / a
    th0, ph0 = np.arccos(np.clip(q[2], -1, 1)), np.arctan2(q[1], q[0])

    def dist(v):
        th, ph = v
        x = np.array([a[0] * np.sin(th) * np.cos(ph), a[1] * np.sin(th) * np.sin(ph), a[2] * np.cos(th)])
        return np.linalg.norm(x - c)

    r = opt.minimize(dist, [th0, ph0], method="Nelder-Mead", options={"xatol": 1e-13, "fatol": 1e-16,
                                                                     "maxiter": 4000})
    return min(r.fun, np.linalg.norm(S[k] - c))


def test_sphere_closed_form():
    rng = np.random.default_rng(0)
    r = 0.04
    for scale in (0.01, 0.03, 0.05, 0.2):
        for _ in range(10):
            c = rng.standard_normal(3)
            c *= scale / np.linalg.norm(c)
            p, n, d, _ = oc.nearest_point(c, [r, r, r])
            u = c / np.linalg.norm(c)
            np.testing.assert_allclose(p, r * u, atol=1e-15)
            np.testing.assert_allclose(n, -u, atol=1e-14)
            assert d == pytest.approx(scale - r, abs=1e-15)


@pytest.mark.parametrize("a", [(0.03, 0.05, 0.07), (0.08, 0.02, 0.05), (0.04, 0.04, 0.07)])
def test_ellipsoid_nearest_point_by_brute_force(a):
    a = np.asarray(a)
    S = _surface_sample(a)
    rng = np.random.default_rng(1)
    for k in range(40):
        c = rng.standard_normal(3) * (0.5 if k % 2 else 1.5) * a
        p, n, d, _ = oc.nearest_point(c, a)
        assert np.sum((p / a) ** 2) == pytest.approx(1.0, abs=1e-13)
        brute = _brute_distance(S, a, c)
        assert abs(d) <= brute + 1e-14
        assert abs(d) >= brute - 1e-11
        inside = np.sum((c / a) ** 2) < 1
        assert (d < 0) == inside
        # first-order optimality: c - p along the normal, on its outer side
        v = c - p
        assert np.linalg.norm(np.cross(v, n)) <= 1e-12 * max(np.linalg.norm(v), 1e-3)
        assert np.dot(v, -n) * np.sign(d) >= -1e-15
        assert np.dot(n, p / a ** 2) < 0  # inward


def test_medial_ridge_and_centre():
    a = np.array([0.03, 0.05, 0.07])
    S = _surface_sample(a, 500)
    # c_0 = 0 deep inside: two nearest points (+- along the smallest axis)
    for c in (np.array([0.0, 0.004, -0.003]), np.array([0.0, 0.0, 0.001]), np.zeros(3)):
        p, n, d, _ = oc.nearest_point(c, a)
        brute = _brute_distance(S, a, c)
        assert np.sum((p / a) ** 2) == pytest.approx(1.0, abs=1e-12)
        assert -d == pytest.approx(brute, abs=1e-11)
        assert -d == pytest.approx(np.linalg.norm(c - p), abs=1e-15)
        assert p[0] > 0
    # a sphere's centre: every surface point is nearest; the query picks one
    p, n, d, _ = oc.nearest_point(np.zeros(3), [0.05, 0.05, 0.05])
    assert d == -0.05 and np.linalg.norm(p) == pytest.approx(0.05) and np.dot(n, p) < 0


def _fd_query(c, a, h=1e-7):
    Jp = np.zeros((3, 3))
    Jn = np.zeros((3, 3))
    Jd = np.zeros(3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        p1, n1, d1, _ = oc.nearest_point(c + e, a)
        p0, n0, d0, _ = oc.nearest_point(c - e, a)
        Jp[:, k] = (p1 - p0) / (2 * h)
        Jn[:, k] = (n1 - n0) / (2 * h)
        Jd[k] = (d1 - d0) / (2 * h)
    return Jp, Jn, Jd


@pytest.mark.parametrize("a", [(0.03, 0.05, 0.07), (0.05, 0.05, 0.05), (0.02, 0.08, 0.03)])
def test_query_jacobian_matches_central_differences(a):
    a = np.asarray(a)
    rng = np.random.default_rng(2)
    for k in range(30):
        c = rng.standard_normal(3) * (0.6 if k % 3 == 0 else 1.4) * a
        if abs(c[np.argmin(a)]) < 0.2 * a.min():
            continue  # keep central differences away from the ridge
        Jp, Jn, Jd = oc.query_jacobian(c, a)
        fp, fn, fd = _fd_query(c, a)
        assert np.abs(Jp - fp).max() <= 1e-7
        assert np.abs(Jn - fn).max() <= 1e-7 / a.min()
        assert np.abs(Jd - fd).max() <= 1e-7
        assert np.linalg.norm(Jd) == pytest.approx(1.0, abs=1e-12)


def test_rodrigues_matches_scipy():
    Rot = pytest.importorskip("scipy.spatial.transform").Rotation
    rng = np.random.default_rng(3)
    for scale in (0.0, 1e-9, 1e-3, 0.5, 3.0):
        w = rng.standard_normal(3) * scale
        np.testing.assert_allclose(oc.rodrigues(w), Rot.from_rotvec(w).as_matrix(), atol=1e-15)


def _loss(hb, R, T, w_dist=200.0, radius=0.01, offset=0.005, cone=False, signed=False):
    L, _, _, _ = oc.loss(R, T, hb.tip_local, hb.semi_axes, hb.counts, hb.woff, hb.mu, hb.wrench,
                         w_qp=1.0, w_dist=w_dist, radius=radius, offset=offset, cone=cone, signed=signed)
    return L


def _grad(hb, R, T, w_dist=200.0, radius=0.01, offset=0.005, drop_normals=False, cone=False, signed=False):
    L, P, N, res = oc.loss(R, T, hb.tip_local, hb.semi_axes, hb.counts, hb.woff, hb.mu, hb.wrench,
                           w_qp=1.0, w_dist=w_dist, radius=radius, offset=offset, cone=cone, signed=signed)
    dP, dN = oracle.grad_batch(hb.counts, hb.woff, P, N, hb.wrench, res["forces"], we=np.ones(hb.n_grasps))
    _, dw, dT = oc.pose_gradient(R, T, hb.tip_local, hb.semi_axes, dP, None if drop_normals else dN,
                                 w_dist, radius, offset, hb.counts, signed=signed)
    return dw, dT


def _fd_pose(hb, R, T, h=1e-6, cone=False, signed=False):
    G = hb.n_grasps
    dw = np.zeros((G, 3))
    dT = np.zeros((G, 3))
    kw = dict(cone=cone, signed=signed)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        Tp, Tm = T + e, T - e
        dT[:, k] = (_loss(hb, R, Tp, **kw) - _loss(hb, R, Tm, **kw)) / (2 * h)
        Rp = np.stack([oc.rodrigues(e) @ R[g] for g in range(G)])
        Rm = np.stack([oc.rodrigues(-e) @ R[g] for g in range(G)])
        dw[:, k] = (_loss(hb, Rp, T, **kw) - _loss(hb, Rm, T, **kw)) / (2 * h)
    return dw, dT


def test_distance_energy_closed_form_on_a_sphere():
    # a fingertip at distance rho from the centre of a sphere of radius a:
    # |c - p| = |a - rho| (Sec. IV-C), signed distance rho - a
    a, alpha, delta = 0.05, 0.01, 0.002
    R, T = np.eye(3)[None], np.zeros((1, 3))
    for rho in (0.012, 0.04, 0.05, 0.07):
        cl = np.array([[[0.0, rho, 0.0]]])
        E, _, _ = oc.pose_gradient(R, T, cl, [[a, a, a]], w_dist=1.0, radius=alpha, offset=delta)
        assert E[0] == pytest.approx((abs(a - rho) - alpha - delta) ** 2, rel=1e-12, abs=1e-18)
        Es, _, _ = oc.pose_gradient(R, T, cl, [[a, a, a]], w_dist=1.0, radius=alpha, offset=delta, signed=True)
        assert Es[0] == pytest.approx((rho - a - alpha - delta) ** 2, rel=1e-12, abs=1e-18)
        # dE/dT along the radius: 2 r d|c-p|/drho with d|c-p|/drho = sign(rho - a)
        _, _, dT = oc.pose_gradient(R, T, cl, [[a, a, a]], w_dist=1.0, radius=alpha, offset=delta)
        sg = 1.0 if rho >= a else -1.0
        assert dT[0, 1] == pytest.approx(2 * (abs(a - rho) - alpha - delta) * sg, rel=1e-10)


@pytest.mark.parametrize("shape,mc,inside,signed", [("ellipsoid", None, 0.0, False), ("sphere", None, 0.0, False),
                                                   ("mixed", (4, 5), 0.0, False),
                                                   ("ellipsoid", None, 0.4, False), ("mixed", (4, 5), 0.4, False),
                                                   ("ellipsoid", None, 0.4, True), ("sphere", None, 0.4, True)])
def test_pose_gradient_matches_central_differences_through_the_qp(shape, mc, inside, signed):
    hb = wl.hand_batch(11, 6, m_choices=mc, s=8, shape=shape, inside=inside)
    R, T = hb.rot.astype(np.float64), hb.trans.astype(np.float64)
    if inside:
        _, _, D = oc.contact_query(R, T, hb.tip_local, hb.semi_axes, hb.counts)
        assert (D < 0).sum() >= 3
    dw, dT = _grad(hb, R, T, signed=signed)
    fw, fT = _fd_pose(hb, R, T, signed=signed)
    for g in range(hb.n_grasps):
        assert np.linalg.norm(dT[g] - fT[g]) <= 1e-5 * max(np.linalg.norm(fT[g]), 1.0)
        assert np.linalg.norm(dw[g] - fw[g]) <= 1e-5 * max(np.linalg.norm(fw[g]), 1.0)


def test_pose_gradient_through_the_circular_cone_matches_central_differences():
    # the same chain rule with the cone oracle's forces (Danskin's gradient
    # depends on the QP only through f*)
    hb = wl.hand_batch(14, 3, s=4)
    R, T = hb.rot.astype(np.float64), hb.trans.astype(np.float64)
    dw, dT = _grad(hb, R, T, cone=True)
    fw, fT = _fd_pose(hb, R, T, cone=True)
    for g in range(hb.n_grasps):
        assert np.linalg.norm(dT[g] - fT[g]) <= 1e-5 * max(np.linalg.norm(fT[g]), 1.0)
        assert np.linalg.norm(dw[g] - fw[g]) <= 1e-5 * max(np.linalg.norm(fw[g]), 1.0)


def test_the_two_distance_forms_differ_only_inside():
    for inside in (0.0, 0.4):
        hb = wl.hand_batch(15, 6, s=4, inside=inside)
        R, T = hb.rot.astype(np.float64), hb.trans.astype(np.float64)
        gu = _grad(hb, R, T)
        gs = _grad(hb, R, T, signed=True)
        scale = max(np.abs(gs[0]).max(), np.abs(gs[1]).max())
        diff = max(np.abs(gu[0] - gs[0]).max(), np.abs(gu[1] - gs[1]).max()) / scale
        if inside:
            assert diff > 1e-2
        else:
            assert diff < 1e-12  # two routes to the same derivative outside


def test_dropped_normal_jacobian_fails_the_difference_check():
    hb = wl.hand_batch(12, 6, s=8)
    R, T = hb.rot.astype(np.float64), hb.trans.astype(np.float64)
    dw, dT = _grad(hb, R, T, drop_normals=True)
    fw, fT = _fd_pose(hb, R, T)
    err = max(np.linalg.norm(dT[g] - fT[g]) / max(np.linalg.norm(fT[g]), 1.0) for g in range(hb.n_grasps))
    assert err > 1e-2


def test_small_descent_step_lowers_the_loss_to_first_order():
    hb = wl.hand_batch(13, 8, s=8)
    R, T = hb.rot.astype(np.float64), hb.trans.astype(np.float64)
    dw, dT = _grad(hb, R, T)
    L0 = _loss(hb, R, T)
    eta = 1e-7
    R1, T1 = oc.descent_step(R, T, dw, dT, eta, eta)
    L1 = _loss(hb, R1, T1)
    pred = eta * (np.sum(dw * dw, axis=1) + np.sum(dT * dT, axis=1))
    assert np.all(L1 < L0)
    np.testing.assert_allclose(L0 - L1, pred, rtol=2e-2)
