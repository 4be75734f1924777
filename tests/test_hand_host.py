"""The solver's coarse-stage query arithmetic compiled for the host (the same
header the GPU kernels use) against the oracle: nearest point, normal and
signed distance (its Newton iteration against the oracle's bisection), the
Jacobian-transposed products against the oracle's implicit-function Jacobians,
the medial ridge and the centre, and the Rodrigues exponential."""
import ctypes
import os

import numpy as np
import pytest

import host_build

from oracle import coarse as oc

HERE = os.path.dirname(os.path.abspath(__file__))
_D = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def host(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("hand_host") / "libhand_host.so")
    host_build.build(os.path.join(HERE, "hand_host.cpp"), out)
    L = ctypes.CDLL(out)
    L.host_nearest.restype = ctypes.c_int
    return L


def _p(a):
    return np.ascontiguousarray(a, np.float64).ctypes.data_as(_D)


def _query(host, c, a):
    c = np.ascontiguousarray(c, np.float64)
    a = np.ascontiguousarray(a, np.float64)
    p, n, d = np.zeros(3), np.zeros(3), ctypes.c_double()
    jac = host.host_nearest(_p(c), _p(a), p.ctypes.data_as(_D), n.ctypes.data_as(_D), ctypes.byref(d))
    return p, n, d.value, jac


AXES = [(0.03, 0.05, 0.07), (0.08, 0.02, 0.05), (0.04, 0.04, 0.07), (0.05, 0.05, 0.05), (0.02, 0.02, 0.02)]


@pytest.mark.parametrize("a", AXES)
def test_query_matches_oracle(host, a):
    a = np.asarray(a)
    rng = np.random.default_rng(4)
    for k in range(300):
        scale = [0.3, 0.9, 1.02, 1.5, 5.0][k % 5]
        c = rng.standard_normal(3) * scale * a
        p, n, d, jac = _query(host, c, a)
        po, no, do, _ = oc.nearest_point(c, a)
        assert np.abs(p - po).max() <= 1e-14 * a.max()
        assert np.abs(n - no).max() <= 1e-12
        assert abs(d - do) <= 1e-15 * max(abs(do), a.max())


def test_ridge_centre_and_surface(host):
    a = np.array([0.03, 0.05, 0.07])
    cases = [np.array([0.0, 0.004, -0.003]), np.array([0.0, 0.0, 0.001]), np.zeros(3),
             np.array([0.0, 0.04, 0.0]), np.array([0.03, 0.0, 0.0]), np.array([0.0, 0.05, 0.0])]
    for c in cases:
        p, n, d, jac = _query(host, c, a)
        po, no, do, _ = oc.nearest_point(c, a)
        np.testing.assert_allclose(p, po, atol=1e-15)
        np.testing.assert_allclose(n, no, atol=1e-13)
        assert d == pytest.approx(do, abs=1e-15)
    p, n, d, jac = _query(host, np.zeros(3), [0.05, 0.05, 0.05])
    assert d == -0.05 and jac == 0


@pytest.mark.parametrize("a", AXES)
def test_chain_matches_oracle_jacobians(host, a):
    a = np.asarray(a)
    rng = np.random.default_rng(5)
    for k in range(200):
        c = rng.standard_normal(3) * [0.5, 1.1, 2.0, 4.0][k % 4] * a
        vp, vn = rng.standard_normal(3), rng.standard_normal(3)
        ws = rng.standard_normal()
        out = np.zeros(3)
        host.host_chain(_p(c), _p(a), _p(vp), _p(vn), ctypes.c_double(ws), out.ctypes.data_as(_D))
        Jp, Jn, Jd = oc.query_jacobian(c, a)
        ref = Jp.T @ vp + Jn.T @ vn + ws * Jd
        scale = np.abs(Jp.T @ vp).max() + np.abs(Jn.T @ vn).max() + abs(ws)
        assert np.abs(out - ref).max() <= 1e-12 * scale


def test_rodrigues_matches_oracle(host):
    rng = np.random.default_rng(6)
    for s in (0.0, 1e-9, 1e-7, 1e-5, 1e-3, 0.3, 2.0):
        w = rng.standard_normal(3) * s
        E = np.zeros(9)
        host.host_rodrigues(_p(w), E.ctypes.data_as(_D))
        np.testing.assert_allclose(E.reshape(3, 3), oc.rodrigues(w), atol=2e-16)
