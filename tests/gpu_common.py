"""Helpers shared by the GPU tests: run the HIP solver, run the oracle on the
same inputs, and compare with the stated tolerances.

Tolerances (FP32 GPU vs FP64 oracle):
  objective  |Q_gpu - Q*| <= 1e-5 * max(Q*, 1e-2 beta^2 ||t||^2)
  forces     max |f_gpu - f*| <= 1e-4 * fmax
  energy     |E_gpu - E*| <= 1e-5 * max(E*, 1e-2 s beta^2)
  gradient   ||g_gpu - g*||_2 <= 1e-3 * max(||g*||_2, 1e-4)   (per grasp, points and normals)
  KKT        oracle-recomputed relative KKT residual of the returned state <= tol
The floor on the objective covers FP32 evaluation of ||r||^2 for tiny Q*.
"""
import numpy as np

import oracle
from paper_2412_16490_amd import api


def run_gpu(batch, state=True, **params):
    import torch
    p = api.default_params(m_max=batch.m_max, s_max=max(1, int(np.max(np.diff(batch.woff)))))
    for k, v in params.items():
        setattr(p, k, v)
    solver = api.Solver(p)
    db = api.DeviceBatch(batch)
    st = api.new_state(db.n_grasps, db.n_qps, db.m_max) if state else None
    res = solver.solve(db, state=st)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in res.items()}
    if st is not None:
        out["state"] = {k: v.cpu().numpy() for k, v in st.items()}
    out["stats"] = solver.stats()
    solver.close()
    return out


def oracle_params(p=None, **kw):
    d = dict(kappa=20.0, beta=1.0, eps=1e-6, fmax=1.0, gamma=0.0)
    d.update(kw)
    return oracle.params(**d)


def check_forward(batch, gpu, ref, beta=1.0, fmax=1.0, qps=None, require_polished=True):
    """Element-wise comparison; returns a dict of worst errors."""
    W = batch.n_qps
    qps = np.arange(W) if qps is None else np.asarray(qps)
    st = gpu["status"][qps]
    assert np.all(st & api.ST_CONVERGED), "unconverged QPs: %s" % qps[(st & api.ST_CONVERGED) == 0][:10]
    assert not np.any(st & api.ST_NONFINITE)
    if require_polished:
        assert np.all(st & api.ST_POLISHED), "unpolished QPs: %d" % np.sum((st & api.ST_POLISHED) == 0)
    Qs = ref["qobj"][qps]
    tnorm2 = np.sum(batch.wrench[qps].astype(np.float64) ** 2, axis=1)
    qerr = np.abs(gpu["qp_obj"][qps] - Qs) / np.maximum(Qs, 1e-2 * beta ** 2 * tnorm2)
    assert qerr.max() <= 1e-5, "objective error %.3e at QP %d" % (qerr.max(), qps[np.argmax(qerr)])
    M = batch.m_max
    ferr = np.abs(gpu["forces"][qps] - ref["forces"][qps][:, :3 * M]).max(axis=1) / fmax
    assert ferr.max() <= 1e-4, "force error %.3e at QP %d" % (ferr.max(), qps[np.argmax(ferr)])
    return {"qerr": float(qerr.max()), "ferr": float(ferr.max())}


def check_energy(batch, gpu, ref, grasps=None, beta=1.0):
    grasps = np.arange(batch.n_grasps) if grasps is None else np.asarray(grasps)
    s = np.diff(batch.woff)[grasps]
    E = ref["energy"][grasps]
    err = np.abs(gpu["energy"][grasps] - E) / np.maximum(E, 1e-2 * s * beta ** 2)
    assert err.max() <= 1e-5, "energy error %.3e" % err.max()
    return float(err.max())


def check_state_kkt(batch, gpu, tol, qps, prm=None):
    """Recompute the relative KKT residual of the returned state in FP64."""
    prm = prm or oracle_params()
    M = batch.m_max
    st = gpu["state"]
    worst = 0.0
    for w in qps:
        g = int(np.searchsorted(batch.woff, w, side="right") - 1)
        m = int(batch.counts[g])
        G = oracle.grasp_matrix(batch.points[g, :m], batch.normals[g, :m], prm.kappa)
        x = st["x"][:3 * m, w].astype(np.float64)
        rows = list(range(9 * m)) + [9 * M]
        z = st["z"][rows, w].astype(np.float64)
        y = st["y"][rows, w].astype(np.float64)
        o = oracle.admm_rel_kkt(G, batch.mu[g, :m], batch.wrench[w], x, z, y, prm)
        assert o[0] <= tol, "oracle rel KKT %.3e > %.1e at QP %d" % (o[0], tol, w)
        assert o[3] <= 1e-6, "state bound/sign violation %.3e at QP %d" % (o[3], w)
        worst = max(worst, o[0])
    return worst
