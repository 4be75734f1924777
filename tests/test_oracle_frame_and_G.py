"""Pins of the oracle's contact frame and grasp matrix (Sec. III, Eq. 2).

The frame must be orthonormal with n = d x e (Sec. III); the grasp matrix must
map a contact force to the wrench it exerts: the force itself in the upper
three rows and the (scaled) moment about the object origin below.  Checked with
identities that hold for any correct implementation, not by re-deriving the
oracle's formula.
"""
import numpy as np
import pytest


def _dirs(seed, k):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_frame_orthonormal_right_handed(orc):
    ns = np.concatenate([_dirs(1, 500), np.eye(3), -np.eye(3),
                         [[1e-9, 0, 1], [0, 1e-9, -1], [0.6, 0.8, 0.0],
                          [0.6, 0.8, -0.0], [-1e-12, 1e-12, 1]]])
    for n in ns:
        nh, d, e = orc.frame(n)
        np.testing.assert_allclose(nh, n / np.linalg.norm(n), atol=1e-15)
        F = np.stack([nh, d, e])
        np.testing.assert_allclose(F @ F.T, np.eye(3), atol=2e-15)
        # Sec. III: n = d x e
        np.testing.assert_allclose(np.cross(d, e), nh, atol=2e-15)


def test_frame_normalises_scaled_normals(orc):
    for n in _dirs(2, 50):
        a = orc.frame(n)
        b = orc.frame(7.3 * n)
        for u, v in zip(a, b):
            np.testing.assert_allclose(u, v, atol=1e-15)


def test_frame_is_continuous_off_the_seam(orc):
    # away from n_z = 0 the tangents vary smoothly with n
    for n in _dirs(3, 50):
        if abs(n[2]) < 0.05:
            continue
        d0 = orc.frame(n)[1]
        d1 = orc.frame(n + 1e-7 * np.array([1.0, -2.0, 0.5]))[1]
        assert np.linalg.norm(d1 - d0) < 1e-4


@pytest.mark.parametrize("m", [1, 2, 4, 5, 8])
def test_grasp_matrix_is_force_and_moment(orc, m):
    rng = np.random.default_rng(10 + m)
    p = rng.uniform(-0.1, 0.1, size=(m, 3))
    n = _dirs(20 + m, m)
    kappa = 20.0
    G = orc.grasp_matrix(p, n, kappa)
    assert G.shape == (6, 3 * m)
    f = rng.standard_normal(3 * m)
    w = G @ f
    F = np.zeros(3)
    T = np.zeros(3)
    for i in range(m):
        nh, d, e = orc.frame(n[i])
        Fi = f[3 * i] * nh + f[3 * i + 1] * d + f[3 * i + 2] * e
        F += Fi
        T += np.cross(p[i], Fi)
    np.testing.assert_allclose(w[:3], F, atol=1e-14)
    np.testing.assert_allclose(w[3:], kappa * T, atol=1e-14)
    # the first column of each block is the unit normal (normal force first)
    for i in range(m):
        np.testing.assert_allclose(G[:3, 3 * i], n[i], atol=1e-15)


def test_grasp_matrix_torque_scale_is_linear(orc):
    rng = np.random.default_rng(5)
    p = rng.uniform(-0.1, 0.1, size=(4, 3))
    n = _dirs(6, 4)
    G1 = orc.grasp_matrix(p, n, 1.0)
    G20 = orc.grasp_matrix(p, n, 20.0)
    np.testing.assert_allclose(G20[:3], G1[:3], atol=0)
    np.testing.assert_allclose(G20[3:], 20.0 * G1[3:], rtol=1e-15, atol=1e-18)
    # a contact at the origin exerts no moment
    G0 = orc.grasp_matrix(np.zeros((1, 3)), n[:1], 20.0)
    assert np.abs(G0[3:]).max() == 0.0


def test_grasp_matrix_translation_identity(orc):
    # Moving every contact by c changes the moment by kappa * (c x F): the
    # lower block must satisfy G_lower(p + c) = G_lower(p) + kappa [c]_x G_upper.
    rng = np.random.default_rng(8)
    p = rng.uniform(-0.1, 0.1, size=(5, 3))
    n = _dirs(9, 5)
    c = np.array([0.01, -0.02, 0.03])
    k = 20.0
    Ga = orc.grasp_matrix(p, n, k)
    Gb = orc.grasp_matrix(p + c, n, k)
    cx = np.array([[0, -c[2], c[1]], [c[2], 0, -c[0]], [-c[1], c[0], 0]])
    np.testing.assert_allclose(Gb[3:], Ga[3:] + k * cx @ Ga[:3], atol=1e-14)
