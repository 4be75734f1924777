"""Parity of the ReLU-QP solver itself (Sec. IV-B: ADMM with the per-grasp
factorised KKT system, its residual checks and rho updates), with the FP64
polish switched off, against the FP64 oracle through the C ABI.

With the polish off the returned point is the ADMM iterate stopped at the
relative KKT residual tol_rel (or at max_iters).  A relative KKT residual of
1e-5 does not fix the objective to 1e-5: the duality gap it allows is about
|y|_1 r_p + |x|_1 r_d, ~1e-3 relative on these workloads, which is why the
solver's default path ends with the exact FP64 polish.  For every QP the
kernel marks converged the returned state is therefore checked against what
it certifies:

* the oracle recomputes the relative KKT residual of the returned FP32 state
  (x, z, y) in FP64: it must be <= tol_rel (the kernel's own FP64 check of
  the same state decided the flag, so only rounding may differ);
* the returned duals y are a valid dual point (weak duality): the dual
  function D(y) = beta^2 |t|^2 - (q + A^T y)^T P^{-1} (q + A^T y) / 2 -
  sigma_C(y) (sigma_C the support function of the row bounds [l, u]) is
  finite and D(y) <= Q*;
* the objective is within what the state certifies: Q* - V <= Q(x) <= Q* +
  (Q(x) - D(y)), where V = lambda*^T (C x - b)^+ prices the returned point's
  constraint violation with the oracle's multipliers (for any x, Q(x) - Q* >=
  grad Q(x*)^T (x - x*) = -lambda*^T (C x - b) >= -V), with the floor
  1e-5 max(Q*, 1e-2 beta^2 |t|^2) for rounding;
* the wrench: |G (x - x*)|^2 <= Q(x) - Q* + V <= (Q(x) - D(y)) + V (the
  same expansion, the quadratic term being |G d|^2 + eps |d|^2), + 1e-4;
* the returned objective is Q of the returned forces.

The converged fraction, the gap and the objective, wrench and force errors
are reported.  Also here: the FP64 factorisation taken when a grasp's
conditioning bound exceeds fp64_cond, forced on every grasp.
"""
import numpy as np
import pytest

import oracle
from paper_2412_16490_amd import api
from paper_2412_16490_amd import workload as wl
from gpu_common import check_energy, check_forward, check_state_kkt, oracle_params, run_gpu

pytestmark = pytest.mark.gpu

def _admm_rows(mu, fmax, gamma):
    """The ADMM form's rows for one grasp: per contact the 8 facets
    (l = -inf, u = 0) and the normal bound [0, fmax], then the normal-sum
    row [gamma, +inf)."""
    m = len(mu)
    C, _ = oracle.constraints(mu, fmax, 0.0)  # 8 facets then f_1 <= fmax, per contact
    srow = np.zeros((1, 3 * m))
    srow[0, 0::3] = 1.0
    A = np.vstack([C[:9 * m], srow])
    lo = np.tile(np.r_[np.full(8, -np.inf), 0.0], m)
    hi = np.tile(np.r_[np.zeros(8), fmax], m)
    return A, np.r_[lo, gamma], np.r_[hi, np.inf]


def _support(y, lo, hi):
    """sup over z in [lo, hi] of y.z (inf where unbounded in y's direction)."""
    with np.errstate(invalid="ignore"):
        v = np.where(y > 0, y * hi, np.where(y < 0, y * lo, 0.0))
    return float(np.sum(v))


def _check_admm_only(b, gpu, tol, prm=None, min_converged=0.9):
    prm = prm or oracle_params()
    st = gpu["status"]
    assert not np.any(st & api.ST_POLISHED)
    conv = np.flatnonzero(st & api.ST_CONVERGED)
    frac = len(conv) / b.n_qps
    # the oracle's FP64 relative KKT of every converged QP's returned state
    kk = check_state_kkt(b, gpu, tol * (1 + 1e-6) + 1e-12, conv, prm)
    M = b.m_max
    S = gpu["state"]
    gaps, qerrs, gerrs, ferrs = [], [], [], []
    for w in conv:
        g = int(np.searchsorted(b.woff, w, side="right") - 1)
        m = int(b.counts[g])
        G = oracle.grasp_matrix(b.points[g, :m].astype(np.float64), b.normals[g, :m].astype(np.float64), prm.kappa)
        mu = b.mu[g, :m].astype(np.float64)
        t = b.wrench[w].astype(np.float64)
        fs, lam, Qs, info = oracle.qp_solve(G, mu, t, prm)
        assert info["status"] == 0
        C, cb = oracle.constraints(mu, prm.fmax, prm.gamma)
        A, lo, hi = _admm_rows(mu, prm.fmax, prm.gamma)
        x = S["x"][:3 * m, w].astype(np.float64)
        y = S["y"][list(range(9 * m)) + [9 * M], w].astype(np.float64)
        P = 2 * (G.T @ G + prm.eps * np.eye(3 * m))
        q = -2 * prm.beta * G.T @ t
        c = prm.beta ** 2 * t @ t
        v = q + A.T @ y
        D = c - 0.5 * v @ np.linalg.solve(P, v) - _support(y, lo, hi)
        Qx = float(np.sum((G @ x - prm.beta * t) ** 2) + prm.eps * x @ x)
        V = float(lam @ np.maximum(C @ x - cb, 0.0))
        floor = 1e-5 * max(Qs, 1e-2 * prm.beta ** 2 * (t @ t))
        assert np.isfinite(D) and D <= Qs + 1e-12 * (1 + Qs), "weak duality fails at QP %d: %g > %g" % (w, D, Qs)
        gap = Qx - D
        Qg = float(gpu["qp_obj"][w])
        assert abs(Qg - Qx) <= 1e-5 * max(Qx, 1e-2 * prm.beta ** 2 * (t @ t)), w
        assert Qs - V - floor <= Qg <= Qs + max(gap, 0.0) + floor, \
            "objective %.9g outside [%.9g, %.9g] at QP %d" % (Qg, Qs - V, Qs + gap, w)
        gerr = np.linalg.norm(G @ (x - fs))
        assert gerr <= np.sqrt(max(gap + V, 0.0)) + 1e-4, "wrench error %.3e, gap %.3e, V %.3e at QP %d" % (
            gerr, gap, V, w)
        gaps.append(max(gap, V) / max(Qs, 1e-2))
        qerrs.append(abs(Qg - Qs) / max(Qs, 1e-2))
        gerrs.append(gerr)
        ferrs.append(np.abs(x - fs).max())
    pct = lambda a, k: float(np.percentile(a, k)) if len(a) else 0.0
    print("ADMM only, tol %g: converged %d/%d (%.4f), iters mean %.1f max %d; worst oracle KKT %.2e; relative gap "
          "median %.1e max %.1e; relative objective error median %.1e max %.1e; wrench error max %.1e; force error "
          "median %.1e max %.1e" % (tol, len(conv), b.n_qps, frac, gpu["iters"].mean(), gpu["iters"].max(), kk,
                                     pct(gaps, 50), pct(gaps, 100), pct(qerrs, 50), pct(qerrs, 100),
                                     pct(gerrs, 100), pct(ferrs, 50), pct(ferrs, 100)), flush=True)
    assert frac >= min_converged
    # the rest either ran to the cap and say so, or stopped on the kernel's
    # FP32 residual check at tol while the FP64 evaluation of the returned
    # state lands just above it (a rounding margin)
    un = np.flatnonzero((st & api.ST_CONVERGED) == 0)
    cap = (st[un] & api.ST_MAX_ITER) != 0
    assert np.all(gpu["iters"][un][cap] == 500)
    edge = un[~cap]
    print("unconverged: %d at the cap, %d stopped by the FP32 check with FP64 residual up to %.2e"
          % (int(cap.sum()), len(edge), gpu["kkt_rel"][edge].max(initial=0)), flush=True)
    assert np.all(gpu["kkt_rel"][edge] <= 4 * tol)
    return frac


def test_admm_only_sphere_m4_s6():
    # the 4-contact workload's own stopping rule: 1e-6 or 500 iterations
    b = wl.config(0)
    print("ADMM only: sphere m4 s6, 384 QPs, tol 1e-6", flush=True)
    gpu = run_gpu(b, tol_rel=1e-6, max_iters=500, flags=api.F_ADAPTIVE_RHO)
    _check_admm_only(b, gpu, 1e-6)


@pytest.mark.parametrize("ng", [3, 64, 300])
def test_admm_only_ellipsoid_m5_s16_subsets(ng):
    b = wl.config(1, ng)
    print("ADMM only: ellipsoid m5 s16, %d grasps, tol 1e-5" % ng, flush=True)
    gpu = run_gpu(b, tol_rel=1e-5, max_iters=500, flags=api.F_ADAPTIVE_RHO)
    _check_admm_only(b, gpu, 1e-5)


def test_admm_only_mixed_m45():
    b = wl.config(3, 200)
    print("ADMM only: mixed m4/5, 200 grasps, tol 1e-5", flush=True)
    gpu = run_gpu(b, tol_rel=1e-5, max_iters=500, flags=api.F_ADAPTIVE_RHO)
    _check_admm_only(b, gpu, 1e-5)


def test_fp64_factorisation_on_every_grasp():
    # fp64_cond = 1 lies below every grasp's conditioning bound, so every
    # grasp's KKT matrix is factored in FP64; ADMM alone and the polished
    # path both keep parity
    b = wl.config(1, 96)
    print("FP64 factor forced: ellipsoid m5 s16, 96 grasps", flush=True)
    gpu = run_gpu(b, tol_rel=1e-5, max_iters=500, flags=api.F_ADAPTIVE_RHO, fp64_cond=1.0)
    assert np.all(gpu["status"] & api.ST_FP64_CHOL), "grasps without the FP64 factor"
    _check_admm_only(b, gpu, 1e-5)
    gpu2 = run_gpu(b, fp64_cond=1.0)
    assert np.all(gpu2["status"] & api.ST_FP64_CHOL)
    ref = oracle.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench, prm=oracle_params())
    print("FP64 factor, polished:", check_forward(b, gpu2, ref), flush=True)
    check_energy(b, gpu2, ref)
    # the default bound takes FP64 on no grasp of this workload
    gpu3 = run_gpu(b)
    assert not np.any(gpu3["status"] & api.ST_FP64_CHOL)
