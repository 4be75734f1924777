"""Parity of the HIP solver (through the C ABI) with the FP64 oracle.

Sizes: the full 4-contact sphere workload (64 grasps, 384 QPs), subsets of the
5-contact ellipsoid workload that span many tiles and end in a ragged tile,
the mixed 4/5-contact uneven-wrench workload, and the full 8192-grasp
ellipsoid workload in its benchmark launch with sampled QPs checked one by one.
"""
import numpy as np
import pytest

import oracle
from paper_2412_16490_amd import api
from paper_2412_16490_amd import workload as wl
from gpu_common import (check_energy, check_forward, check_state_kkt, oracle_params, run_gpu)

pytestmark = pytest.mark.gpu


def _ref(b, prm=None):
    return oracle.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench,
                              prm=prm or oracle_params())


def test_sphere_m4_s6_full():
    b = wl.config(0)
    gpu = run_gpu(b, tol_rel=1e-6)
    ref = _ref(b)
    print("sphere:", check_forward(b, gpu, ref), "iters mean", gpu["iters"].mean())
    check_energy(b, gpu, ref)
    check_state_kkt(b, gpu, 1e-5, range(b.n_qps))


@pytest.mark.parametrize("ng", [1, 3, 37, 256])
def test_ellipsoid_m5_s16_subsets(ng):
    b = wl.config(1, ng)
    gpu = run_gpu(b)
    ref = _ref(b)
    print("ellipsoid %d:" % ng, check_forward(b, gpu, ref), "iters mean", gpu["iters"].mean())
    check_energy(b, gpu, ref)
    check_state_kkt(b, gpu, 1e-5, range(0, b.n_qps, max(1, b.n_qps // 200)))


@pytest.mark.parametrize("admm_tol", [1e-5, 1e-3, 1e-2, 0.0, 1e30])
def test_admm_tolerance_does_not_change_the_result(admm_tol):
    # ADMM run to tol_rel (1e-5), to 1e-3 or 1e-2, to the pyramid's default
    # (0: 1e-1), or stopped at its first check (1e30): the polish reaches the
    # same minimiser
    b = wl.config(1, 96)
    gpu = run_gpu(b, admm_tol=admm_tol)
    ref = _ref(b)
    print("admm_tol %g:" % admm_tol, check_forward(b, gpu, ref), "iters mean", gpu["iters"].mean())
    check_energy(b, gpu, ref)


def test_polish_flop_count_is_reported():
    import torch
    b = wl.config(1, 32)
    p = api.default_params(m_max=5, s_max=16)
    s = api.Solver(p)
    db = api.DeviceBatch(b)
    r = api.new_result(db.n_grasps, db.n_qps, 5, polish_flops=True)
    s.solve(db, result=r)
    torch.cuda.synchronize()
    fl = r["polish_flops"].cpu().numpy()
    # at least the warm start, one factorisation, one equality solve and the
    # acceptance check of a 5-contact QP
    assert np.all(fl >= 3 * 249 * 5 + 150 * 5 + 231 * 5 + 100 + 530 * 5 + 144)
    r2 = api.new_result(db.n_grasps, db.n_qps, 5)          # no flop output: still fine
    s.solve(db, result=r2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r2["forces"].cpu().numpy(), r["forces"].cpu().numpy())
    s.close()


@pytest.mark.parametrize("gamma,beta", [(0.0, 1.0), (0.5, 1.0), (1.0, 0.0)])
def test_force_axis_wrenches(gamma, beta):
    # the paper's force-closure energy: the six unit force-axis wrenches per
    # grasp (Sec. IV-A), with the normal-sum row of Eq. 9; beta = 0 is the
    # QP baseline of the comparison in Sec. V
    b = wl.force_axis_batch(wl.config(1, 128))
    gpu = run_gpu(b, gamma=gamma, beta=beta)
    ref = _ref(b, oracle_params(gamma=gamma, beta=beta))
    print("force axes gamma %g beta %g:" % (gamma, beta), check_forward(b, gpu, ref, beta=beta))
    check_energy(b, gpu, ref, beta=beta)


def test_mixed_m45_uneven_s():
    b = wl.config(3, 300)
    gpu = run_gpu(b)
    ref = _ref(b)
    print("mixed:", check_forward(b, gpu, ref))
    check_energy(b, gpu, ref)
    check_state_kkt(b, gpu, 1e-5, range(0, b.n_qps, 37))


def test_mixed_batched_form_matches_oracle():
    b = wl.config(3, 300)
    gpu = run_gpu(b, flags=api.default_params().flags | api.F_BATCHED)
    ref = _ref(b)
    check_forward(b, gpu, ref)
    check_energy(b, gpu, ref)


def test_full_ellipsoid_m5_s16_every_qp():
    # the headline shape in its benchmark launch: all 131,072 QPs element by
    # element against the oracle
    b = wl.config(1)
    print("full ellipsoid m5 s16: 131,072 QPs, every QP against the oracle", flush=True)
    gpu = run_gpu(b)
    ref = _ref(b)
    print("full:", check_forward(b, gpu, ref), "iters mean", gpu["iters"].mean())
    check_energy(b, gpu, ref)
    assert np.all(gpu["kkt_rel"] <= 1e-5)
    check_state_kkt(b, gpu, 1e-5, range(0, b.n_qps, 97))


def test_full_mixed_batched_graph_every_qp():
    # the 50,000-grasp uneven batch in the launch configuration the benchmark
    # times: the persistent cost-sorted launch captured in a graph, replayed;
    # all 951,279 QPs element by element against the oracle
    import torch
    b = wl.config(3)
    print("full mixed batched graph: 50,000 grasps, every QP against the oracle", flush=True)
    p = api.default_params(m_max=5, s_max=32)
    p.flags |= api.F_BATCHED | api.F_GRAPH
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = api.Solver(p, stream=stream.cuda_stream)
        db = api.DeviceBatch(b)
        st = api.new_state(db.n_grasps, db.n_qps, 5)
        r = api.new_result(db.n_grasps, db.n_qps, 5)
        s.solve(db, state=st, result=r)
        s.solve(db, state=st, result=r)
        stats = s.stats()
        stream.synchronize()
        s.close()
    assert stats["graph_replays"] == 1 and stats["launches"] == 1
    gpu = {k: v.cpu().numpy() for k, v in r.items()}
    ref = _ref(b)
    print("full mixed batched:", check_forward(b, gpu, ref))
    check_energy(b, gpu, ref)
    assert np.all(gpu["kkt_rel"] <= 1e-5)


def test_largest_swept_batch_sampled():
    # 131,072 grasps x 16 wrenches (2.1 M QPs, the largest batch the
    # benchmark sweeps): sampled grasps against the oracle, every QP checked
    # for convergence
    b = wl.uniform_batch(16491, 131072, 5, 16, name="sweep")
    gpu = run_gpu(b)
    rng = np.random.default_rng(13)
    grasps = np.sort(rng.choice(b.n_grasps, 48, replace=False))
    grasps = np.unique(np.concatenate([grasps, [0, b.n_grasps - 1]]))
    sub = b.subset(grasps)
    ref = _ref(sub)
    qps = np.concatenate([np.arange(b.woff[g], b.woff[g + 1]) for g in grasps])
    sub_gpu = {k: gpu[k][qps] for k in ("forces", "qp_obj", "status", "kkt_rel", "iters")}
    sub_gpu["energy"] = gpu["energy"][grasps]
    print("2.1M QPs sampled:", check_forward(sub, sub_gpu, ref))
    check_energy(sub, sub_gpu, ref)
    assert np.all(gpu["status"] & api.ST_CONVERGED)
    assert np.all(np.isfinite(gpu["forces"]))


def test_gamma_and_bounds_parity():
    b = wl.config(1, 40)
    for gamma, fmax, beta in [(0.5, 1.0, 1.0), (1.2, 0.5, 2.0)]:
        gpu = run_gpu(b, gamma=gamma, force_max=fmax, beta=beta)
        ref = _ref(b, oracle_params(gamma=gamma, fmax=fmax, beta=beta))
        check_forward(b, gpu, ref, beta=beta, fmax=fmax)


def test_small_contact_counts_in_m5_layout():
    # grasps with 1 and 2 contacts (the brute-force sizes) inside a 5-contact layout
    rng = np.random.default_rng(3)
    b = wl.config(1, 24)
    b.counts[:] = rng.integers(1, 3, size=24)
    for g in range(24):
        m = b.counts[g]
        b.points[g, m:] = 0
        b.normals[g, m:] = [0, 0, 1]
    gpu = run_gpu(b)
    ref = _ref(b)
    check_forward(b, gpu, ref)
    check_energy(b, gpu, ref)


def test_extreme_sizes():
    # 64 wrenches per grasp (the largest s), single-contact grasps, and a
    # 4-contact layout (m_max = 4 kernels) in one test
    b64 = wl.uniform_batch(777, 9, 5, 64, name="s64")
    gpu = run_gpu(b64)
    ref = _ref(b64)
    print("s=64:", check_forward(b64, gpu, ref))
    check_energy(b64, gpu, ref)
    b1 = wl.uniform_batch(778, 40, 1, 7, name="m1")
    gpu = run_gpu(b1)
    ref = _ref(b1)
    print("m=1:", check_forward(b1, gpu, ref))
    check_energy(b1, gpu, ref)
    b4 = wl.uniform_batch(779, 70, 4, 13, name="m4")
    gpu = run_gpu(b4)
    ref = _ref(b4)
    print("m=4 layout:", check_forward(b4, gpu, ref))
    check_energy(b4, gpu, ref)


def test_empty_batch_is_a_no_op():
    import torch
    b = wl.uniform_batch(780, 4, 5, 3)
    e = b.subset([])
    p = api.default_params(m_max=5, s_max=8)
    s = api.Solver(p)
    db = api.DeviceBatch(e)
    r = s.solve(db)
    torch.cuda.synchronize()
    assert r["forces"].shape[0] == 0 and s.stats()["launches"] == 0
    s.close()


def test_graph_replay_matches_direct_launch():
    # capture on a side stream, replay several times with eager work between,
    # and compare every replay with a direct launch
    import torch
    b = wl.config(3, 500)
    s_max = int(np.max(np.diff(b.woff)))
    db = api.DeviceBatch(b)
    direct = run_gpu(b, flags=api.default_params().flags | api.F_BATCHED)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        p = api.default_params(m_max=5, s_max=s_max)
        p.flags |= api.F_BATCHED | api.F_GRAPH
        s = api.Solver(p, stream=side.cuda_stream)
        st = api.new_state(db.n_grasps, db.n_qps, 5)
        r = api.new_result(db.n_grasps, db.n_qps, 5)       # same buffers every call
        replays = 0
        for rep in range(4):
            s.solve(db, state=st, result=r)
            replays += s.stats()["graph_replays"]
            junk = torch.randn(1000, device="cuda").sum()   # eager work in between
            side.synchronize()
            assert torch.isfinite(junk)
            np.testing.assert_array_equal(r["forces"].cpu().numpy(), direct["forces"])
            np.testing.assert_array_equal(r["qp_obj"].cpu().numpy(), direct["qp_obj"])
            np.testing.assert_array_equal(r["energy"].cpu().numpy(), direct["energy"])
            np.testing.assert_array_equal(r["status"].cpu().numpy(), direct["status"])
        assert replays == 3
        s.close()


def test_kernel_timing_flag():
    import torch
    b = wl.config(1, 64)
    p = api.default_params(m_max=5, s_max=16)
    p.flags |= api.F_TIMING
    s = api.Solver(p)
    db = api.DeviceBatch(b)
    st = api.new_state(db.n_grasps, db.n_qps, 5)
    s.solve(db, state=st)
    s.backward(db, st, dL_dE=torch.ones(db.n_grasps, device="cuda"))
    kt = s.kernel_times()
    assert kt["admm_ms"] > 0 and kt["finalize_ms"] > 0 and kt["backward_ms"] > 0
    s.close()


@pytest.mark.parametrize("chunk", [0, 1, 3, 12, 40])
@pytest.mark.parametrize("cfg,ng", [(1, 300), (3, 300), (0, 64)])
def test_chunked_polish_budgets(chunk, cfg, ng):
    # the one-lane polish with a budget of `chunk` factorisations, the
    # contact-parallel polish for the QPs it hands on (0: none handed on,
    # 1: nearly all, 40: none needs it), the outputs of those QPs formed by
    # the second finalize pass: the same minimiser either way
    b = wl.config(cfg, ng)
    print("chunked polish: %s, %d grasps, chunk %d" % (b.name, ng, chunk), flush=True)
    gpu = run_gpu(b, polish_chunk=chunk, tol_rel=1e-6 if cfg == 0 else 1e-5)
    ref = _ref(b)
    print("chunk %d:" % chunk, check_forward(b, gpu, ref))
    check_energy(b, gpu, ref)
    check_state_kkt(b, gpu, 1e-6 if cfg == 0 else 1e-5, range(0, b.n_qps, 7))
