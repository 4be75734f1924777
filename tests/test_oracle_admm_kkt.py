"""Pins of the oracle's relative-KKT measure for ADMM-form states.

ADMM form: r = 9m+1 two-sided rows l <= A f <= u (per contact 8 facets with
u = 0 then the normal bound [0, fmax]; last the normal-sum row [gamma, inf)).
The measure (OSQP-style, eps_abs = eps_rel) must vanish at the exact optimum
mapped into this form, and must respond to each kind of defect.
"""
import numpy as np

from paper_2412_16490_amd import workload as wl


def _to_admm(orc, G, mu, t, prm):
    m = len(mu)
    f, lam, Q, info = orc.qp_solve(G, mu, t, prm)
    C, b = orc.constraints(mu, prm.fmax, prm.gamma)
    r = 9 * m + 1
    z = np.zeros(r)
    y = np.zeros(r)
    for i in range(m):
        z[9 * i:9 * i + 8] = C[9 * i:9 * i + 8] @ f
        z[9 * i + 8] = f[3 * i]
        y[9 * i:9 * i + 9] = lam[9 * i:9 * i + 9]      # facets and upper bound
    z[9 * m] = f[0::3].sum()
    if prm.gamma > 0:
        y[9 * m] = -lam[9 * m]                          # lower-active sum row
    z = np.minimum(z, np.r_[np.tile(np.r_[np.zeros(8), prm.fmax], m), np.inf])
    return f, z, y


def test_exact_optimum_has_zero_residual(orc):
    b = wl.config(1, 16)
    for g in range(16):
        G = orc.grasp_matrix(b.points[g], b.normals[g], 20.0)
        for gamma in (0.0, 0.4):
            prm = orc.params(gamma=gamma)
            for w in range(b.woff[g], b.woff[g] + 4):
                f, z, y = _to_admm(orc, G, b.mu[g], b.wrench[w], prm)
                out = orc.admm_rel_kkt(G, b.mu[g], b.wrench[w], f, z, y, prm)
                assert out[0] < 1e-11 and out[3] < 1e-11, out


def test_residual_responds_to_defects(orc):
    b = wl.config(1, 2)
    G = orc.grasp_matrix(b.points[0], b.normals[0], 20.0)
    prm = orc.params()
    t = b.wrench[0]
    f, z, y = _to_admm(orc, G, b.mu[0], t, prm)
    # primal defect: z off A f by delta in one row
    z2 = z.copy()
    z2[3] -= 1e-3
    o = orc.admm_rel_kkt(G, b.mu[0], t, f, z2, y, prm)
    nAx = max(np.abs(z).max(), 1e-3)
    assert abs(o[1] - 1e-3 / (1 + max(nAx, np.abs(z2).max()))) < 1e-9
    # dual defect: a perturbed multiplier breaks stationarity
    y2 = y.copy()
    y2[8] += 1e-3
    assert orc.admm_rel_kkt(G, b.mu[0], t, f, z, y2, prm)[2] > 1e-5
    # sign defect: a positive multiplier on a facet row with slack
    y3 = y.copy()
    facet = np.array([r for r in range(len(z) - 1) if r % 9 != 8])
    k = int(facet[np.argmin(z[facet])])
    assert z[k] < -1e-2
    y3[k] = 0.5
    assert orc.admm_rel_kkt(G, b.mu[0], t, f, z, y3, prm)[3] > 1e-3
    # bound defect: z outside [l, u]
    z4 = z.copy()
    z4[8] = -0.1
    assert orc.admm_rel_kkt(G, b.mu[0], t, f, z4, y, prm)[3] > 0.05
