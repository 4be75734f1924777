"""The chunked FP64 polish compiled for the host (the headers the GPU kernels
use): the one-lane polish stops after a budget of factorisations, saves its
state to a spill record, and the contact-parallel polish (one thread per
contact standing in for one lane per contact) continues from the record.
Whatever the budget -- 0 hands every QP on at its first factorisation -- the
result must be the oracle's minimiser, and a QP the group finishes keeps the
counts of its first part."""
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
    out = str(tmp_path_factory.mktemp("gpolish_host") / "libgpolish_host.so")
    host_build.build(os.path.join(HERE, "gpolish_host.cpp"), out, extra=["-pthread"])
    return ctypes.CDLL(out)


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _run(host, b, g, y0, budget, force_break=0, shared_factor=0):
    m = int(b.counts[g])
    s = min(int(b.woff[g + 1] - b.woff[g]), 6)
    p, pp = _d(b.points[g, :m])
    n, pn = _d(b.normals[g, :m])
    mu, pm = _d(b.mu[g, :m])
    t, pt = _d(b.wrench[b.woff[g]:b.woff[g] + s])
    y = np.ascontiguousarray(y0[:s], dtype=np.float32)
    x = np.zeros((s, 15))
    st = np.zeros(s, np.int32)
    hd = np.zeros(s, np.int32)
    cnt = np.zeros((s, 4), np.int32)
    I = ctypes.POINTER(ctypes.c_int)
    bad = host.host_chunked_polish(m, pp, pn, pm, pt, s, ctypes.c_double(20.0), ctypes.c_double(1e-6),
                                   y.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(budget),
                                   x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), st.ctypes.data_as(I),
                                   hd.ctypes.data_as(I), cnt.ctypes.data_as(I), int(force_break),
                                   int(shared_factor))
    return bad, x[:, :3 * m], st, hd, cnt


@pytest.mark.parametrize("cfg,ng", [(1, 12), (3, 12), (0, 6)])
@pytest.mark.parametrize("budget", [0, 1, 4, 12])
def test_chunked_polish_reaches_the_minimiser(host, cfg, ng, budget):
    b = wl.config(cfg, ng)
    ref = oracle.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench, oracle.params())
    rng = np.random.default_rng(23 + budget)
    handed = 0
    for g in range(b.n_grasps):
        s = int(b.woff[g + 1] - b.woff[g])
        m = int(b.counts[g])
        y0 = np.where(rng.random((s, 46)) < 0.3, rng.random((s, 46)), 0.0)
        bad, x, st, hd, cnt = _run(host, b, g, y0, budget)
        assert bad == 0, st
        fr = ref["forces"][b.woff[g]:b.woff[g] + len(st), :3 * m]
        assert np.abs(x - fr).max() <= 1e-8, (g, np.abs(x - fr).max())
        if budget == 0:
            assert np.all(hd == 1)
        # a QP handed on had used up its budget; one kept was done within it
        assert np.all(cnt[hd == 1, 0] > budget)
        assert np.all(cnt[hd == 0, 0] <= budget)
        handed += int(hd.sum())
    assert handed > 0


@pytest.mark.parametrize("budget", [0, 2])
def test_group_restart_from_the_empty_set_after_a_breakdown(host, budget):
    # the first ratio test breaks down (forced once): with budget 0 in the
    # contact-parallel polish, which restarts from the empty active set;
    # with budget 2 wherever the QP reaches its first step
    b = wl.config(1, 8)
    ref = oracle.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench, oracle.params())
    rng = np.random.default_rng(29)
    hit = 0
    for g in range(b.n_grasps):
        s = int(b.woff[g + 1] - b.woff[g])
        m = int(b.counts[g])
        y0 = np.where(rng.random((s, 46)) < 0.3, rng.random((s, 46)), 0.0)
        bad0, x0, st0, hd0, c0 = _run(host, b, g, y0, budget)
        bad, x, st, hd, cnt = _run(host, b, g, y0, budget, force_break=1)
        assert bad0 == 0 and bad == 0, st
        fr = ref["forces"][b.woff[g]:b.woff[g] + len(st), :3 * m]
        assert np.abs(x - fr).max() <= 1e-8, (g, np.abs(x - fr).max())
        hit += int(np.sum(c0[:, 3] > 0))
    assert hit > 0


@pytest.mark.parametrize("budget", [0, 3])
def test_group_factor_in_memory_matches_the_register_form(host, budget):
    # the GPU kernel keeps each group's 6x6 factor once in LDS (Sym6Shared)
    # instead of in every lane's registers: the chol6 routines through that
    # accessor do the same arithmetic, so the results are bit-identical
    b = wl.config(1, 10)
    rng = np.random.default_rng(31)
    handed = 0
    for g in range(b.n_grasps):
        s = int(b.woff[g + 1] - b.woff[g])
        y0 = np.where(rng.random((s, 46)) < 0.3, rng.random((s, 46)), 0.0)
        r0 = _run(host, b, g, y0, budget)
        r1 = _run(host, b, g, y0, budget, shared_factor=1)
        assert r0[0] == 0 and r1[0] == 0
        for a0, a1 in zip(r0[1:], r1[1:]):
            assert np.array_equal(a0, a1)
        handed += int(r0[3].sum())
    assert handed > 0
