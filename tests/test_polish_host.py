"""The solver's FP64 polish compiled for the host (the same header the GPU
kernels use) against the oracle: from a cold start (no warm rows) and from a
deliberately poor warm guess it must reach the oracle's minimiser, and the
run-time facet coefficients must equal cos/sin of (2k+1) pi / 8."""
import ctypes
import os

import numpy as np
import pytest

import host_build
import oracle
from paper_2412_16490_amd import workload as wl

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def host(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("polish_host") / "libpolish_host.so")
    host_build.build(os.path.join(HERE, "polish_host.cpp"), out)
    lib = ctypes.CDLL(out)
    return lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def test_facet_coefficients(host):
    for k in range(8):
        c, s = ctypes.c_double(), ctypes.c_double()
        host.host_facet_cs(k, ctypes.byref(c), ctypes.byref(s))
        phi = (2 * k + 1) * np.pi / 8
        assert abs(c.value - np.cos(phi)) < 1e-15 and abs(s.value - np.sin(phi)) < 1e-15


def _solve(host, b, g, y0, gamma=0.0, fmax=1.0):
    m = int(b.counts[g])
    s = int(b.woff[g + 1] - b.woff[g])
    p, pp = _d(b.points[g, :m])
    n, pn = _d(b.normals[g, :m])
    mu, pm = _d(b.mu[g, :m])
    t, pt = _d(b.wrench[b.woff[g]:b.woff[g + 1]])
    y = np.ascontiguousarray(y0, dtype=np.float32)
    x = np.zeros((s, 15))
    st = np.zeros(s, np.int32)
    steps = np.zeros(s, np.int32)
    host.host_polish_grasp(m, pp, pn, pm, pt, s, ctypes.c_double(20.0), ctypes.c_double(1.0),
                           ctypes.c_double(1e-6), ctypes.c_double(fmax), ctypes.c_double(gamma),
                           y.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), 200,
                           x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           st.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return x[:, :3 * m], st, steps


@pytest.mark.parametrize("cfg,ng,gamma,fmax", [(1, 12, 0.0, 1.0), (3, 12, 0.0, 1.0), (0, 8, 0.0, 1.0),
                                               (1, 8, 2.0, 1.0), (3, 8, 0.5, 0.4)])
def test_polish_reaches_oracle_minimiser(host, cfg, ng, gamma, fmax):
    b = wl.config(cfg, ng)
    ref = oracle.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench,
                             oracle.params(gamma=gamma, fmax=fmax))
    rng = np.random.default_rng(5)
    for g in range(b.n_grasps):
        s = int(b.woff[g + 1] - b.woff[g])
        m = int(b.counts[g])
        fr = ref["forces"][b.woff[g]:b.woff[g + 1], :3 * m]
        cold = np.zeros((s, 46))
        poor = np.where(rng.random((s, 46)) < 0.3, rng.random((s, 46)), 0.0)   # random rows "active"
        poor[:, 45] = -rng.random(s)
        for y0 in (cold, poor):
            x, st, steps = _solve(host, b, g, y0, gamma, fmax)
            assert np.all(st == 0), (g, st)
            assert np.abs(x - fr).max() <= 1e-8 * fmax, (g, np.abs(x - fr).max())


def _valid_rows(rng):
    """A random active row set of one contact that the polish can hold: up to
    three rows, independent (no bound row together with two opposite facets,
    whose tangential parts are parallel)."""
    while True:
        n = int(rng.integers(0, 4))
        rows = sorted(rng.choice(9, size=n, replace=False).tolist())
        facets = [k for k in rows if k < 8]
        if 8 in rows and len(facets) == 2 and abs(facets[0] - facets[1]) == 4:
            continue
        return rows


def test_one_row_change_matches_the_matrix_from_every_contact(host):
    # a row joining or leaving contact ci changes eps I + G Pi G^T by a
    # rank-one term; the matrix formed from the old factor plus that term must
    # equal the one formed from every contact's projector
    b = wl.config(1, 40)
    rng = np.random.default_rng(11)
    worst = 0.0
    for g in range(b.n_grasps):
        m = int(b.counts[g])
        p, pp = _d(b.points[g, :m])
        n, pn = _d(b.normals[g, :m])
        mu, pm = _d(b.mu[g, :m])
        for trial in range(6):
            rows = [_valid_rows(rng) for _ in range(m)]
            ci = int(rng.integers(0, m))
            if not rows[ci]:
                continue
            kk = int(rng.choice(rows[ci]))
            full = sum(sum(1 << (9 * i + k) for k in rows[i]) for i in range(m))
            less = full & ~(1 << (9 * ci + kk))
            for join in (0, 1):
                before, after = (less, full) if join else (full, less)
                a, pa = _d(np.zeros(21))
                c, pc = _d(np.zeros(21))
                rc = host.host_matrix_change(m, pp, pn, pm, ctypes.c_double(20.0), ctypes.c_double(1e-6),
                                             ctypes.c_ulonglong(before), ctypes.c_ulonglong(after), ci, kk, join,
                                             pa, pc)
                assert rc == 0
                err = np.abs(a - c).max() / np.abs(c).max()
                worst = max(worst, err)
                assert err <= 1e-12, (g, trial, join, err)
    print("worst relative difference %.2e" % worst)


def test_one_row_change_pin_fails_with_the_wrong_direction(host):
    # planted error on the oracle side of the comparison: the change's
    # direction taken without projecting out the contact's other rows
    # differs from the matrix from every contact, so the pin above can fail
    b = wl.config(1, 4)
    g, m = 0, int(b.counts[0])
    G = oracle.grasp_matrix(b.points[g, :m], b.normals[g, :m])
    mu = b.mu[g, :m] * np.cos(np.pi / 8)
    rows = {0: [1, 2]}
    def rowc(i, k):
        if k == 8:
            return np.array([1.0, 0.0, 0.0])
        phi = (2 * k + 1) * np.pi / 8
        return np.array([-mu[i], np.cos(phi), np.sin(phi)])
    def M_of(rs):
        M = 1e-6 * np.eye(6)
        for i in range(m):
            C = np.array([rowc(i, k) for k in rs.get(i, [])]).reshape(-1, 3)
            Pi = np.eye(3) - (C.T @ np.linalg.pinv(C @ C.T) @ C if len(C) else 0.0)
            Gi = G[:, 3 * i:3 * i + 3]
            M += Gi @ Pi @ Gi.T
        return M
    before, after = M_of({0: [1]}), M_of(rows)
    c = rowc(0, 2)
    v = G[:, 0:3] @ (c / np.linalg.norm(c))        # wrong: not projected
    assert np.abs((before - np.outer(v, v)) - after).max() > 1e-6 * np.abs(after).max()
    r1 = rowc(0, 1)
    Q = np.eye(3) - np.outer(r1, r1) / (r1 @ r1)
    e = Q @ c
    v = G[:, 0:3] @ (e / np.linalg.norm(e))        # right: projected
    assert np.abs((before - np.outer(v, v)) - after).max() <= 1e-12 * np.abs(after).max()


def _counts(host, b, g, y0, force_retry, first_cap=200):
    m = int(b.counts[g])
    s = int(b.woff[g + 1] - b.woff[g])
    p, pp = _d(b.points[g, :m])
    n, pn = _d(b.normals[g, :m])
    mu, pm = _d(b.mu[g, :m])
    t, pt = _d(b.wrench[b.woff[g]:b.woff[g + 1]])
    y = np.ascontiguousarray(y0, dtype=np.float32)
    cnt = np.zeros((s, 4), np.int32)
    x = np.zeros((s, 15))
    bad = host.host_polish_counts(m, pp, pn, pm, pt, s, ctypes.c_double(20.0), ctypes.c_double(1e-6),
                                  y.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(force_retry),
                                  cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                  x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(first_cap))
    return bad, cnt, x[:, :3 * m]


def test_polish_factors_once_then_changes_one_row_at_a_time(host):
    b = wl.config(1, 24)
    rng = np.random.default_rng(13)
    tot = upd = 0
    for g in range(b.n_grasps):
        s = int(b.woff[g + 1] - b.woff[g])
        y0 = np.where(rng.random((s, 46)) < 0.3, rng.random((s, 46)), 0.0)
        bad, cnt, _ = _counts(host, b, g, y0, False)
        assert bad == 0
        tot += int(np.sum(cnt[:, 0] - 1))
        upd += int(np.sum(cnt[:, 1]))
        assert np.all(cnt[:, 1] <= cnt[:, 0] - 1)
    print("factorisations after the first: %d, one-row changes: %d" % (tot, upd))
    assert tot > 0 and upd >= 0.99 * tot


def test_retry_on_fresh_factorisations_reaches_the_minimiser(host):
    # the path a QP takes when its acceptance check fails after one-row
    # changes (forced here): it restarts from its last set with fresh
    # factorisations only and must still end at the oracle's minimiser
    b = wl.config(1, 16)
    ref = oracle.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench, oracle.params())
    rng = np.random.default_rng(17)
    retried = 0
    for g in range(b.n_grasps):
        s = int(b.woff[g + 1] - b.woff[g])
        m = int(b.counts[g])
        y0 = np.where(rng.random((s, 46)) < 0.3, rng.random((s, 46)), 0.0)
        bad0, c0, x0 = _counts(host, b, g, y0, False)
        bad1, c1, x1 = _counts(host, b, g, y0, True)
        assert bad0 == 0 and bad1 == 0
        fr = ref["forces"][b.woff[g]:b.woff[g + 1], :3 * m]
        assert np.abs(x1 - fr).max() <= 1e-8, (g, np.abs(x1 - fr).max())
        used = c0[:, 1] > 0
        # a retried QP factors afresh at least once more and makes no further one-row changes
        assert np.all(c1[used, 0] > c0[used, 0]) and np.all(c1[used, 1] == c0[used, 1])
        assert np.all(c1[~used] == c0[~used])
        retried += int(used.sum())
    assert retried > 0


@pytest.mark.parametrize("mode", ["breakdown", "step cap"])
def test_retry_after_a_failed_attempt_reaches_the_minimiser(host, mode):
    # a QP whose attempt with one-row changes ends in a ratio-test breakdown
    # (forced once) or runs out of steps (a first-attempt cap of 4
    # factorisations) is taken once more from its last set with fresh
    # factorisations and a cap of its own, and ends at the oracle's minimiser
    b = wl.config(1, 16)
    ref = oracle.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench, oracle.params())
    rng = np.random.default_rng(19)
    retried = 0
    for g in range(b.n_grasps):
        s = int(b.woff[g + 1] - b.woff[g])
        m = int(b.counts[g])
        y0 = np.where(rng.random((s, 46)) < 0.3, rng.random((s, 46)), 0.0)
        bad0, c0, x0 = _counts(host, b, g, y0, 0)
        if mode == "breakdown":
            bad1, c1, x1 = _counts(host, b, g, y0, 2)
            hit = c0[:, 1] > 0  # QPs that made a one-row change: the forced breakdown hits them
        else:
            bad1, c1, x1 = _counts(host, b, g, y0, 3, first_cap=4)
            hit = (c0[:, 0] > 4) & (c0[:, 1] > 0)
        assert bad0 == 0 and bad1 == 0
        fr = ref["forces"][b.woff[g]:b.woff[g + 1], :3 * m]
        assert np.abs(x1 - fr).max() <= 1e-8, (g, np.abs(x1 - fr).max())
        assert np.all(c1[~hit] == c0[~hit])
        retried += int(hit.sum())
    assert retried > 0


def test_restart_from_the_empty_set_after_a_breakdown(host):
    # a QP whose first ratio test breaks down (forced once) before any
    # one-row change has no last set to retry from: it restarts from the
    # empty active set (the unconstrained minimiser, from which the dual
    # active-set steps are the textbook method) with fresh factorisations,
    # and ends at the oracle's minimiser
    b = wl.config(1, 16)
    ref = oracle.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench, oracle.params())
    rng = np.random.default_rng(23)
    hit_total = 0
    for g in range(b.n_grasps):
        s = int(b.woff[g + 1] - b.woff[g])
        m = int(b.counts[g])
        y0 = np.where(rng.random((s, 46)) < 0.3, rng.random((s, 46)), 0.0)
        bad0, c0, x0 = _counts(host, b, g, y0, 0)
        bad1, c1, x1 = _counts(host, b, g, y0, 4)
        assert bad0 == 0 and bad1 == 0
        fr = ref["forces"][b.woff[g]:b.woff[g + 1], :3 * m]
        assert np.abs(x1 - fr).max() <= 1e-8, (g, np.abs(x1 - fr).max())
        hit = c0[:, 3] > 0  # QPs that reach a ratio test: the forced breakdown hits them
        assert np.all(c1[~hit] == c0[~hit])
        assert np.all(c1[hit, 0] > 1)
        hit_total += int(hit.sum())
    assert hit_total > 0
