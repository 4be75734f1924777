"""Pin of the oracle's QP solver by brute-force active-set enumeration.

For a strictly convex QP (eps > 0) the minimiser is the solution of the
equality-constrained problem on some linearly independent subset of its active
rows.  Enumerating every such subset, solving its KKT system, discarding
primal-infeasible candidates and keeping the lowest objective therefore yields
the exact minimiser -- by a route that shares nothing with the oracle's dual
active-set iteration.  Feasible only for m <= 2 (19 rows, ~4e4 subsets).
"""
import itertools

import numpy as np
import pytest


def brute_force(P, q, C, b, tol=1e-11):
    n = P.shape[0]
    nc = C.shape[0]
    best_x, best_v = None, np.inf
    for k in range(0, min(n, nc) + 1):
        combos = np.array(list(itertools.combinations(range(nc), k)), dtype=np.int64)
        if k == 0:
            x = np.linalg.solve(P, -q)[None]
        else:
            CS = C[combos]                                   # [N, k, n]
            sv = np.linalg.svd(CS, compute_uv=False)         # [N, k]
            keep = sv[:, -1] > 1e-9 * sv[:, 0]
            combos, CS = combos[keep], CS[keep]
            if len(combos) == 0:
                continue
            N = len(combos)
            K = np.zeros((N, n + k, n + k))
            K[:, :n, :n] = P
            K[:, :n, n:] = np.transpose(CS, (0, 2, 1))
            K[:, n:, :n] = CS
            rhs = np.zeros((N, n + k))
            rhs[:, :n] = -q
            rhs[:, n:] = b[combos]
            x = np.linalg.solve(K, rhs[..., None])[..., 0][:, :n]
        feas = np.all(x @ C.T <= b + tol, axis=1)
        if not feas.any():
            continue
        xf = x[feas]
        v = 0.5 * np.einsum("ni,ij,nj->n", xf, P, xf) + xf @ q
        j = int(np.argmin(v))
        if v[j] < best_v:
            best_v, best_x = v[j], xf[j]
    return best_x


def _instance(orc, seed, m):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-0.05, 0.05, size=(m, 3))
    n = rng.standard_normal((m, 3))
    mu = rng.uniform(0.2, 1.0, size=m)
    t = rng.standard_normal(6)
    t /= np.linalg.norm(t)
    beta = [0.3, 1.0, 3.0][seed % 3]
    fmax = [1.0, 0.5][seed % 2]
    gamma = [0.0, 0.0, 0.2 * m * fmax][seed % 3]
    return p, n, mu, t, orc.params(kappa=20.0, beta=beta, eps=1e-6, fmax=fmax, gamma=gamma)


SEEDS_M1 = list(range(100, 130))
SEEDS_M2 = list(range(200, 216))


@pytest.mark.parametrize("m,seed", [(1, s) for s in SEEDS_M1] + [(2, s) for s in SEEDS_M2])
def test_oracle_equals_bruteforce(orc, m, seed):
    p, n, mu, t, prm = _instance(orc, seed, m)
    G = orc.grasp_matrix(p, n, prm.kappa)
    P = 2 * (G.T @ G + prm.eps * np.eye(3 * m))
    q = -2 * prm.beta * G.T @ t
    C, b = orc.constraints(mu, prm.fmax, prm.gamma)
    xb = brute_force(P, q, C, b)
    f, lam, Q, info = orc.qp_solve(G, mu, t, prm)
    assert info["status"] == 0
    np.testing.assert_allclose(f, xb, atol=1e-9, rtol=0)
    Qb = np.sum((G @ xb - prm.beta * t) ** 2) + prm.eps * xb @ xb
    assert abs(Q - Qb) <= 1e-10 * max(1.0, Qb)


def test_bruteforce_detects_a_planted_error(orc):
    # A solver that ignores the friction pyramid (keeps only the bound rows)
    # must be caught by the enumeration: the comparison is not vacuous.
    p, n, mu, t, prm = _instance(orc, 3, 2)
    prm.beta = 1.0
    G = orc.grasp_matrix(p, n, prm.kappa)
    P = 2 * (G.T @ G + prm.eps * np.eye(6))
    q = -2 * prm.beta * G.T @ t
    C, b = orc.constraints(mu, prm.fmax, 0.0)
    xb = brute_force(P, q, C, b)
    bound_rows = [8, 17]
    x_wrong = brute_force(P, q, C[bound_rows], b[bound_rows])
    assert np.abs(x_wrong - xb).max() > 1e-3
