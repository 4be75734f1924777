"""GPU parity of the exact circular friction cone (Eq. 1 in place of the
8-facet pyramid of Sec. IV-A) against the FP64 cone oracle, through the C ABI.

Tolerances are those of the pyramid path: objective
|Q_gpu - Q*| <= 1e-5 max(Q*, 1e-2 beta^2 |t|^2), forces 1e-4 fmax, energy
1e-5 max(E*, 1e-2 s beta^2), gradients 1e-3 relative (norm-wise per grasp,
floor 1e-4).  The cone's FP64 barrier polish reaches the oracle's own
precision (forces to ~1e-6, objectives to ~1e-10) on every QP, so no instance
is exempted.
"""
import numpy as np
import pytest

import oracle
from oracle import cone as oc
from paper_2412_16490_amd import api
from paper_2412_16490_amd import workload as wl

import cone_certificate as cc

pytestmark = pytest.mark.gpu


def _solve(b, state=None, gamma=0.0, beta=1.0, backward=False, residual=True, **kw):
    import torch
    p = api.default_params(m_max=b.m_max, s_max=int(np.max(np.diff(b.woff))))
    p.friction_cone = api.CONE_CIRCULAR
    p.gamma = gamma
    p.beta = beta
    for k, v in kw.items():
        setattr(p, k, v)
    s = api.Solver(p)
    db = api.DeviceBatch(b)
    st = state if state is not None else api.new_state(db.n_grasps, db.n_qps, db.m_max, cone=True,
                                                       residual=residual)
    res = api.new_result(db.n_grasps, db.n_qps, db.m_max, polish_flops=True)
    s.solve(db, state=st, result=res)
    out = {k: v.cpu().numpy() for k, v in res.items()}
    if backward:
        gp, gn = s.backward(db, st, dL_dE=torch.ones(db.n_grasps, device="cuda"))
        out["dP"] = gp.cpu().numpy().astype(np.float64)
        out["dN"] = gn.cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    out["state"] = st
    s.close()
    return out


def _check(b, gpu, ref, qps=None, beta=1.0):
    W = b.n_qps
    qps = np.arange(W) if qps is None else np.asarray(qps)
    st = gpu["status"][qps]
    assert np.all(st & api.ST_CONVERGED), "unconverged: %s" % qps[(st & api.ST_CONVERGED) == 0][:10]
    assert np.all(st & api.ST_POLISHED), "unpolished: %d" % np.sum((st & api.ST_POLISHED) == 0)
    Qs = ref["qobj"][qps]
    tn = np.sum(b.wrench[qps].astype(np.float64) ** 2, axis=1)
    qerr = np.abs(gpu["qp_obj"][qps] - Qs) / np.maximum(Qs, 1e-2 * beta ** 2 * tn)
    assert qerr.max() <= 1e-5, "objective error %.3e at QP %d" % (qerr.max(), qps[np.argmax(qerr)])
    M = b.m_max
    ferr = np.abs(gpu["forces"][qps] - ref["forces"][qps][:, :3 * M]).max(axis=1)
    print("cone check: %d QPs, objective error max %.2e, force error max %.2e" % (len(qps), qerr.max(), ferr.max()),
          flush=True)
    assert ferr.max() <= 1e-4, "force error %.3e at QP %d" % (ferr.max(), qps[np.argmax(ferr)])
    return qerr.max(), ferr.max()


def _oracle(b, gamma=0.0, beta=1.0, qps=None):
    """The cone oracle's answers, each certified optimal independently of the
    barrier method: the projected-gradient fixed point with the closed-form
    projection holds to 1e-7."""
    ref = oc.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench, gamma=gamma, beta=beta, qps=qps)
    qlist = np.arange(b.n_qps) if qps is None else np.asarray(qps)
    r1, = cc.certify_batch(oracle.grasp_matrix, b, ref["forces"], qlist, beta=beta, gamma=gamma)
    assert r1 <= 1e-7, r1
    return ref


def test_cone_sphere_m4_s6_full():
    b = wl.config(0)
    print("cone parity: sphere m4 s6, %d QPs" % b.n_qps, flush=True)
    gpu = _solve(b)
    ref = _oracle(b)
    qe, fe = _check(b, gpu, ref)
    E = np.array([ref["qobj"][b.woff[g]:b.woff[g + 1]].sum() for g in range(b.n_grasps)])
    s = np.diff(b.woff)
    assert np.all(np.abs(gpu["energy"] - E) <= 1e-5 * np.maximum(E, 1e-2 * s))
    print("objective %.2e force %.2e" % (qe, fe))


@pytest.mark.parametrize("gamma", [0.0, 2.0])
def test_cone_ellipsoid_m5_s16_subset(gamma):
    b = wl.config(1, 40)
    print("cone parity: ellipsoid m5 s16, 40 grasps, gamma %g" % gamma, flush=True)
    gpu = _solve(b, gamma=gamma)
    ref = _oracle(b, gamma=gamma)
    _check(b, gpu, ref)
    # the polish reports its flops
    assert np.all(gpu["polish_flops"] > 0)


def test_cone_mixed_contact_counts():
    b = wl.config(3, 60)
    print("cone parity: mixed m4/m5, uneven s, %d QPs" % b.n_qps, flush=True)
    gpu = _solve(b)
    ref = _oracle(b)
    _check(b, gpu, ref)


def test_cone_between_the_pyramids():
    # on the same grasps the exact cone's energy lies between the inscribed
    # pyramid's (the solver's default model) and the circumscribed one's
    b = wl.config(1, 64)
    gpu_c = _solve(b)
    p = api.default_params(m_max=5, s_max=16)
    s = api.Solver(p)
    db = api.DeviceBatch(b)
    r_in = s.solve(db, state=api.new_state(db.n_grasps, db.n_qps, 5))
    import torch
    torch.cuda.synchronize()
    e_in = r_in["energy"].cpu().numpy()
    s.close()
    b_out = wl.Batch(b.points, b.normals, (b.mu / np.cos(np.pi / 8)).astype(np.float32), b.wrench, b.counts, b.woff)
    s2 = api.Solver(api.default_params(m_max=5, s_max=16))
    db2 = api.DeviceBatch(b_out)
    r_out = s2.solve(db2, state=api.new_state(db2.n_grasps, db2.n_qps, 5))
    torch.cuda.synchronize()
    e_out = r_out["energy"].cpu().numpy()
    s2.close()
    e_c = gpu_c["energy"]
    tol = 1e-5 * np.maximum(e_c, 1e-2 * 16)
    assert np.all(e_c <= e_in + tol) and np.all(e_c >= e_out - tol)
    print("mean energy: inscribed %.4e cone %.4e circumscribed %.4e" % (e_in.mean(), e_c.mean(), e_out.mean()))


def test_cone_full_size_sampled():
    b = wl.config(1)
    gpu = _solve(b)
    rng = np.random.default_rng(5)
    qps = np.unique(np.concatenate([rng.integers(0, b.n_qps, 200), [0, b.n_qps - 1]]))
    ref = _oracle(b, qps=qps)
    _check(b, gpu, ref, qps=qps)
    assert np.all(gpu["status"] & api.ST_CONVERGED)


def test_cone_warm_start_keeps_the_result():
    b = wl.config(1, 24)
    g1 = _solve(b)
    p_flags = api.default_params().flags | api.F_WARM_START
    g2 = _solve(b, state=g1["state"], flags=p_flags)
    assert np.all(g2["status"] & api.ST_POLISHED)
    assert np.all(g2["iters"] <= 10)  # the warm state converges at the first check
    np.testing.assert_allclose(g2["qp_obj"], g1["qp_obj"], rtol=1e-5, atol=1e-7)


def test_cone_qp_baseline_beta0():
    # beta = 0 with the normal-sum row: the force-sum-only baseline
    b = wl.force_axis_batch(wl.config(1, 16))
    gpu = _solve(b, gamma=1.0, beta=0.0)
    ref = _oracle(b, gamma=1.0, beta=0.0)
    Qs = ref["qobj"]
    assert np.all(np.abs(gpu["qp_obj"] - Qs) <= 1e-5 * np.maximum(Qs, 1e-2))
    assert np.all(np.abs(gpu["forces"] - ref["forces"][:, :15]).max(axis=1) <= 1e-4)


def test_cone_backward_matches_oracle_gradient():
    # Danskin's theorem makes the gradient a function of f* alone (chained
    # through Eq. 2 and the tangent basis): against the oracle's gradient at
    # the oracle's minimiser.  The solve stores the residual G f* - beta t
    # formed in FP64 (state.r); formed from the FP32 forces instead it loses
    # its digits on grasps with a small residual (checked below against the
    # chain rule applied to the FP32 forces themselves)
    b = wl.config(2, 48)
    gpu = _solve(b, backward=True)
    P0, N0 = b.points.astype(np.float64), b.normals.astype(np.float64)
    ref = _oracle(b)
    _check(b, gpu, ref)
    rel = lambda a, r: np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-4)
    rp, rn = oracle.grad_batch(b.counts, b.woff, P0, N0, b.wrench, ref["forces"][:, :3 * b.m_max],
                               we=np.ones(b.n_grasps))
    ep = max(rel(gpu["dP"][g], rp[g]) for g in range(b.n_grasps))
    en = max(rel(gpu["dN"][g], rn[g]) for g in range(b.n_grasps))
    print("cone grad rel err (exact forces) points %.2e normals %.2e" % (ep, en))
    assert ep <= 1e-3 and en <= 1e-3
    # without the stored residual: the chain rule on the FP32 forces
    gpu2 = _solve(b, backward=True, residual=False)
    f_gpu = gpu2["forces"].astype(np.float64)
    rp2, rn2 = oracle.grad_batch(b.counts, b.woff, P0, N0, b.wrench, f_gpu, we=np.ones(b.n_grasps))
    ep2 = max(rel(gpu2["dP"][g], rp2[g]) for g in range(b.n_grasps))
    en2 = max(rel(gpu2["dN"][g], rn2[g]) for g in range(b.n_grasps))
    print("cone grad rel err (own FP32 forces, no residual) points %.2e normals %.2e" % (ep2, en2))
    assert ep2 <= 1e-3 and en2 <= 1e-3


def test_cone_retry_after_a_failed_polish():
    """polish_steps = 0: the barrier polish reaches its Newton-step cap before
    the first step, so the retry from the point half way to the cone axis
    runs as well and fails the same way.  Each QP keeps the ADMM point (forces
    and objective equal to those of the same solve without the polish), is
    marked rejected, and its polish work counts the start of both attempts:
    two merit gradients each, 140 m + 20 FP64 flops apiece."""
    b = wl.config(1, 16)
    print("cone retry: ellipsoid m5 s16, 16 grasps, polish_steps 0", flush=True)
    same = dict(tol_rel=1e-4, admm_tol=1e-4, max_iters=200)
    gpu = _solve(b, polish_steps=0, **same)
    off = _solve(b, flags=api.default_params().flags & ~api.F_POLISH, **same)
    st = gpu["status"]
    assert np.all(st & api.ST_POLISH_REJ) and not np.any(st & api.ST_POLISHED)
    assert np.array_equal(gpu["forces"], off["forces"])
    assert np.array_equal(gpu["qp_obj"], off["qp_obj"])
    m = np.repeat(b.counts, np.diff(b.woff)).astype(np.float64)
    assert np.allclose(gpu["polish_flops"], 4.0 * (140.0 * m + 20.0), rtol=1e-6, atol=0.0)


def test_cone_rejects_bad_model_value():
    import ctypes
    p = api.default_params()
    p.friction_cone = 7
    h = ctypes.c_void_p()
    assert api.lib().bodex_qp_create(ctypes.byref(p), 0, None, 0, ctypes.byref(h)) == api.EINVAL


def test_cone_backward_with_the_normal_sum_row():
    # gamma > 0: the gradient against the oracle's at its minimiser
    b = wl.config(2, 24)
    gpu = _solve(b, gamma=1.0, backward=True)
    ref = _oracle(b, gamma=1.0)
    _check(b, gpu, ref)
    P0, N0 = b.points.astype(np.float64), b.normals.astype(np.float64)
    rp, rn = oracle.grad_batch(b.counts, b.woff, P0, N0, b.wrench, ref["forces"][:, :3 * b.m_max],
                               we=np.ones(b.n_grasps))
    rel = lambda a, r: np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-4)
    ep = max(rel(gpu["dP"][g], rp[g]) for g in range(b.n_grasps))
    en = max(rel(gpu["dN"][g], rn[g]) for g in range(b.n_grasps))
    print("cone gamma 1 grad rel err points %.2e normals %.2e" % (ep, en))
    assert ep <= 1e-3 and en <= 1e-3
