"""torch.autograd wrapper and the continuous-batching server."""
import numpy as np
import pytest

import oracle
from paper_2412_16490_amd import api
from paper_2412_16490_amd import workload as wl

pytestmark = pytest.mark.gpu


def test_autograd_energy_gradient_matches_oracle():
    import torch
    from paper_2412_16490_amd.autograd import BodexQPEnergy
    b = wl.config(2, 48)
    P = torch.tensor(b.points, device="cuda", requires_grad=True)
    N = torch.tensor(b.normals, device="cuda", requires_grad=True)
    mu = torch.tensor(b.mu, device="cuda")
    t = torch.tensor(b.wrench, device="cuda")
    E, Q, F = BodexQPEnergy.apply(P, N, mu, t, b.woff, b.counts, None)
    rng = np.random.default_rng(2)
    we = torch.tensor(rng.standard_normal(b.n_grasps), dtype=torch.float32, device="cuda")
    wq = torch.tensor(rng.standard_normal(b.n_qps), dtype=torch.float32, device="cuda")
    loss = (we * E).sum() + (wq * Q).sum()
    loss.backward()
    P0, N0 = b.points.astype(np.float64), b.normals.astype(np.float64)
    ref = oracle.solve_batch(b.counts, b.woff, P0, N0, b.mu, b.wrench)
    rp, rn = oracle.grad_batch(b.counts, b.woff, P0, N0, b.wrench, ref["forces"],
                               wq=wq.cpu().numpy().astype(np.float64),
                               we=we.cpu().numpy().astype(np.float64))
    gp, gn = P.grad.cpu().numpy(), N.grad.cpu().numpy()
    for g in range(b.n_grasps):
        assert np.linalg.norm(gp[g] - rp[g]) <= 1e-3 * max(np.linalg.norm(rp[g]), 1e-4)
        assert np.linalg.norm(gn[g] - rn[g]) <= 1e-3 * max(np.linalg.norm(rn[g]), 1e-4)
    np.testing.assert_allclose(E.detach().cpu().numpy(), ref["energy"], rtol=1e-5, atol=1e-6)
    assert not F.requires_grad


def _stream(n, steps=4, seed=123):
    return list(wl.request_stream(seed=seed, rate=1000.0, duration=10.0, size_range=(16, 256),
                                  steps=steps, max_requests=n))


def test_served_results_equal_alone_and_in_mix():
    from paper_2412_16490_amd.serve import Server
    reqs = _stream(6)
    srv = Server(m_max=5, s_max=32, budget_bytes=1 << 30)
    srv.keep_results = True
    stats = srv.run(reqs, realtime=False)
    mixed = srv.results
    srv.close()
    assert stats["requests"] == 6
    assert stats["ticks"] < 6 * 4          # requests shared ticks
    for r in reqs[:3]:
        alone = Server(m_max=5, s_max=32, budget_bytes=1 << 30)
        alone.keep_results = True
        alone.run([r], realtime=False)
        a = alone.results[r.rid]
        alone.close()
        m = mixed[r.rid]
        np.testing.assert_allclose(a["qp_obj"], m["qp_obj"], rtol=1e-5, atol=1e-8)
        np.testing.assert_allclose(a["forces"], m["forces"], atol=1e-4)
        np.testing.assert_allclose(a["energy"], m["energy"], rtol=1e-5, atol=1e-8)
        np.testing.assert_allclose(a["grad_points"], m["grad_points"], rtol=1e-4, atol=1e-6)


def test_served_step_matches_oracle_after_random_walk():
    # the last step of a served request solves the QPs of the walked points
    from paper_2412_16490_amd.serve import Server
    reqs = _stream(2, steps=3, seed=7)
    srv = Server(m_max=5, s_max=32, budget_bytes=1 << 30)
    srv.keep_results = True
    srv.run(reqs, realtime=False)
    for r in reqs:
        b = r.batch
        pts = b.points.copy()
        for k in range(r.steps - 1):        # points of the last step
            pts = pts + r.walk[k]
        ref = oracle.solve_batch(b.counts, b.woff, pts, b.normals, b.mu, b.wrench)
        got = srv.results[r.rid]
        s = np.diff(b.woff)
        err = np.abs(got["energy"] - ref["energy"]) / np.maximum(ref["energy"], 1e-2 * s)
        assert err.max() <= 1e-5
    srv.close()


def test_budget_admission_queues_instead_of_failing():
    from paper_2412_16490_amd.serve import POOL_SHARE, Server, _StatePool, request_bytes
    reqs = _stream(5, steps=2, seed=11)
    biggest = max(request_bytes(r.batch.n_grasps, r.batch.n_qps, 5) for r in reqs)
    most_qps = max(r.batch.n_qps for r in reqs)
    bq, bg = _StatePool.bytes_per(5)
    # room for about one request at a time, in the per-request budget and in
    # the state pool
    budget = int(1.05 * max(biggest / (1 - POOL_SHARE), (bq + bg / 4) * most_qps / POOL_SHARE))
    srv = Server(m_max=5, s_max=32, budget_bytes=budget)
    stats = srv.run(reqs, realtime=False)
    assert stats["requests"] == 5
    assert stats["peak_device_bytes"] <= budget - int(POOL_SHARE * budget)
    srv.close()


def test_state_pool_layout_equals_the_plain_state():
    # the solve and the backward on a state pool (per-grasp column offsets,
    # grasps scattered over the pool in another order) give the same bits as
    # on a plain state, warm-started the same way
    import torch
    b = wl.config(3, 120)
    db = api.DeviceBatch(b)
    G, W = db.n_grasps, db.n_qps
    s = api.Solver(api.default_params(m_max=5, s_max=32))
    sw = api.Solver(api.default_params(m_max=5, s_max=32, flags_set=api.F_WARM_START))
    plain = api.new_state(G, W, 5)
    cap_q, cap_g = 3 * W, 3 * G
    pool = api.new_state(cap_g, cap_q, 5)
    rng = np.random.default_rng(5)
    order = rng.permutation(G)
    s_of = np.diff(b.woff)
    qoff = np.zeros(G, np.int32)
    col = 7
    for g in order:             # grasps placed in a shuffled order with gaps
        qoff[g] = col
        col += int(s_of[g]) + int(rng.integers(0, 4))
    assert col <= cap_q
    goff = (2 * rng.permutation(G) + 1).astype(np.int32)
    pooled = dict(pool, qp_offset=qoff, grasp_offset=goff)
    outs = []
    for st, solver_cold in ((plain, s), (pooled, s)):
        r1 = solver_cold.solve(db, state=st)
        r2 = sw.solve(db, state=st)            # a warm-started second step
        gp, gn = sw.backward(db, st, dL_dE=torch.ones(G, device="cuda"))
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy() for t in (r1["forces"], r2["forces"], r2["qp_obj"], r2["iters"],
                                               r2["status"], gp, gn)])
    for a_, b_ in zip(*outs):
        np.testing.assert_array_equal(a_, b_)
    # the pooled columns hold the plain state's columns
    cols = np.concatenate([qoff[g] + np.arange(s_of[g]) for g in range(G)])
    np.testing.assert_array_equal(pool["x"][:, cols].cpu().numpy(), plain["x"].cpu().numpy())
    np.testing.assert_array_equal(pool["rho"][goff].cpu().numpy(), plain["rho"].cpu().numpy())
    s.close()
    sw.close()


def test_autotuner_picks_a_converged_configuration(tmp_path):
    from paper_2412_16490_amd import autotune
    b = wl.config(3, 400)
    db = api.DeviceBatch(b)
    best, table = autotune.tune(db, reps=1, grid={"admm_waves": [1, 2], "check_every": [10],
                                                    "batched": [0, 1]},
                                cache_path=str(tmp_path / "cache.json"))
    assert len(table) == 4 and all(t["converged"] for t in table)
    assert best in [t["knobs"] for t in table]
    best2, _ = autotune.tune(db, cache_path=str(tmp_path / "cache.json"))   # cached
    assert best2 == best
    p = autotune.apply(api.default_params(m_max=5, s_max=32), best)
    ref = oracle.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench)
    from gpu_common import run_gpu, check_forward
    gpu = run_gpu(b, admm_waves=p.admm_waves, check_every=p.check_every, flags=p.flags)
    check_forward(b, gpu, ref)
