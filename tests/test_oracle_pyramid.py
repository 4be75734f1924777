"""Pins of the oracle's constraint rows: the 8-facet pyramid that linearises
the friction cone of Eq. 1 (Sec. IV-A), the normal-force bound of Eq. 1 and the
normal-sum row of Eq. 9.

Reading used (inscribed pyramid): its 8 edge rays lie on the cone
f2^2 + f3^2 = mu^2 f1^2 at tangent angles k*pi/4, so every pyramid force is a
valid Eq. 1 force.
"""
import numpy as np
import pytest


def _facets(orc, mu):
    C, b = orc.constraints([mu], 1.0, 0.0)
    return C[:8], b[:8], C[8], b[8]


@pytest.mark.parametrize("mu", [0.3, 0.5, 0.8, 1.2])
def test_edges_on_cone_and_on_two_facets(orc, mu):
    F, bF, _, _ = _facets(orc, mu)
    assert np.all(bF == 0.0)
    for k in range(8):
        th = k * np.pi / 4
        v = np.array([1.0, mu * np.cos(th), mu * np.sin(th)])
        # Eq. 1 with equality: on the cone surface
        assert abs(v[1] ** 2 + v[2] ** 2 - mu ** 2 * v[0] ** 2) < 1e-14
        s = F @ v
        assert np.all(s <= 1e-14)          # inside every facet
        assert np.sum(np.abs(s) < 1e-14) == 2  # exactly on two facets


@pytest.mark.parametrize("mu", [0.3, 0.5, 0.8])
def test_pyramid_inside_cone_and_covers_inscribed_octagon(orc, mu):
    F, _, _, _ = _facets(orc, mu)
    rng = np.random.default_rng(0)
    # any pyramid point is a valid Eq. 1 force (inscribed reading)
    pts = rng.uniform(-1, 1, size=(20000, 3))
    pts[:, 0] = np.abs(pts[:, 0])
    pts[:, 1:] *= 1.2 * mu          # sample around the cone, some points outside
    inside = np.all(pts @ F.T <= 0, axis=1)
    v = pts[inside]
    assert 1000 < len(v) < len(pts)
    assert np.all(v[:, 1] ** 2 + v[:, 2] ** 2 <= mu ** 2 * v[:, 0] ** 2 * (1 + 1e-12))
    # and the pyramid contains the cone shrunk by cos(pi/8) (its inscribed circle)
    ang = rng.uniform(0, 2 * np.pi, 5000)
    c8 = np.cos(np.pi / 8)
    w = np.stack([np.ones_like(ang), mu * c8 * np.cos(ang), mu * c8 * np.sin(ang)], 1)
    assert np.all(w @ F.T <= 1e-12)


@pytest.mark.parametrize("mu", [0.3, 0.5, 0.8])
def test_facet_gram_closed_form(orc, mu):
    F, _, B, bB = _facets(orc, mu)
    # sum_k a_k a_k^T = diag(8 mu^2 cos^2(pi/8), 4, 4): the sums of cos, sin and
    # sin*cos over the 8 facet angles vanish.
    c8 = np.cos(np.pi / 8)
    np.testing.assert_allclose(F.T @ F, np.diag([8 * mu ** 2 * c8 ** 2, 4, 4]), atol=1e-14)
    np.testing.assert_allclose(B, [1.0, 0.0, 0.0])
    assert bB == 1.0


def test_facets_imply_nonnegative_normal(orc):
    # opposite facets k and k+4 sum to (-2 mu cos(pi/8), 0, 0): f1 >= 0 follows
    F, _, _, _ = _facets(orc, 0.5)
    for k in range(4):
        s = F[k] + F[k + 4]
        assert s[0] < 0 and abs(s[1]) < 1e-15 and abs(s[2]) < 1e-15


def test_gamma_row(orc):
    C, b = orc.constraints([0.5, 0.6, 0.7], 1.0, 0.0)
    assert C.shape == (27, 9)           # gamma = 0: implied row dropped
    C, b = orc.constraints([0.5, 0.6, 0.7], 1.0, 0.4)
    assert C.shape == (28, 9)
    np.testing.assert_allclose(C[-1], [-1, 0, 0, -1, 0, 0, -1, 0, 0])
    assert b[-1] == -0.4
    # rows of different contacts act on disjoint variables
    assert np.all(C[:9, 3:] == 0) and np.all(C[9:18, :3] == 0)
