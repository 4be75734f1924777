"""Pin of the oracle's energy gradient by central finite differences.

E_g = sum_j Q_j is C^1 in (p, n) (Danskin: the feasible set does not depend on
G; eps > 0 makes each minimiser unique), with dQ/dG = 2 (G f* - beta t) f*^T
(Sec. IV-A: Q_j is differentiable through G_i).  The analytic chain through
Eq. 2, the tangent basis and the normalisation of n is compared with central
differences of the oracle's own energy in FP64 (h = 1e-4), on 64 seeded grasps
of the 5-contact / 16-wrench ellipsoid workload.

Finite differences are only as good as the energy's smoothness at scale h: its
curvature can reach ||r||^2/eps near active-set switches.  A grasp whose
comparison fails at h = 1e-4 is re-checked at h = 1e-5 and 1e-6; the test
fails if a grasp fails at every step size, and it also demands agreement to
1e-5 for every grasp at h = 1e-6 (the FD error must vanish as h -> 0).
Normal z-coordinates within 2h of the basis seam n_z = 0 are skipped.
"""
import numpy as np
import pytest

from paper_2412_16490_amd import workload as wl


def _energy(orc, b, P, N):
    out = orc.solve_batch(b.counts, b.woff, P, N, b.mu, b.wrench, nthreads=0)
    return out["energy"]


def _fd(orc, b, h):
    """Central differences of every grasp's energy in every p and n coordinate."""
    G, M = b.n_grasps, b.m_max
    P0 = b.points.astype(np.float64)
    N0 = b.normals.astype(np.float64)
    dP = np.zeros((G, M, 3))
    dN = np.zeros((G, M, 3))
    for which, base, out in (("p", P0, dP), ("n", N0, dN)):
        for i in range(M):
            for c in range(3):
                plus = base.copy()
                minus = base.copy()
                plus[:, i, c] += h
                minus[:, i, c] -= h
                if which == "p":
                    ep = _energy(orc, b, plus, N0)
                    em = _energy(orc, b, minus, N0)
                else:
                    ep = _energy(orc, b, P0, plus)
                    em = _energy(orc, b, P0, minus)
                out[:, i, c] = (ep - em) / (2 * h)
    return dP, dN


def _rel_ok(a, b, skip=None):
    a = a.copy()
    b = b.copy()
    if skip is not None:
        a[skip] = 0
        b[skip] = 0
    return np.linalg.norm(a - b) <= 1e-3 * max(np.linalg.norm(b), 1e-4)


def test_gradient_matches_central_differences(orc):
    b = wl.config(2, 64)
    P0 = b.points.astype(np.float64)
    N0 = b.normals.astype(np.float64)
    out = orc.solve_batch(b.counts, b.woff, P0, N0, b.mu, b.wrench)
    gP, gN = orc.grad_batch(b.counts, b.woff, P0, N0, b.wrench, out["forces"],
                            we=np.ones(b.n_grasps))
    pending = set(range(b.n_grasps))
    report = {}
    for h in (1e-4, 1e-5, 1e-6):
        fP, fN = _fd(orc, b, h)
        for g in sorted(pending):
            seam = np.zeros((b.m_max, 3), bool)
            seam[:, 2] = np.abs(N0[g, :, 2]) < 2 * h
            if _rel_ok(gP[g], fP[g]) and _rel_ok(gN[g], fN[g], seam):
                pending.discard(g)
                if h != 1e-4:
                    report[g] = h
    assert not pending, "grasps failing FD at every h: %s" % sorted(pending)
    # the large majority must pass at the nominal step (measured: 11 of 64
    # need a smaller h on this seed)
    assert len(report) <= 16, report
    # and every grasp converges as h -> 0: at h = 1e-6 the agreement is far
    # inside the 1e-3 bar for all 64 grasps
    fP, fN = _fd(orc, b, 1e-6)
    for g in range(b.n_grasps):
        seam = np.zeros((b.m_max, 3), bool)
        seam[:, 2] = np.abs(N0[g, :, 2]) < 2e-6
        a, c = gN[g].copy(), fN[g].copy()
        a[seam] = c[seam] = 0
        assert np.linalg.norm(gP[g] - fP[g]) <= 1e-5 * max(np.linalg.norm(fP[g]), 1e-4)
        assert np.linalg.norm(a - c) <= 1e-5 * max(np.linalg.norm(c), 1e-4)


def test_gradient_weights_are_linear(orc):
    b = wl.config(2, 6)
    P0 = b.points.astype(np.float64)
    N0 = b.normals.astype(np.float64)
    out = orc.solve_batch(b.counts, b.woff, P0, N0, b.mu, b.wrench)
    rng = np.random.default_rng(0)
    wq = rng.standard_normal(b.n_qps)
    we = rng.standard_normal(b.n_grasps)
    a = orc.grad_batch(b.counts, b.woff, P0, N0, b.wrench, out["forces"], wq=wq)
    c = orc.grad_batch(b.counts, b.woff, P0, N0, b.wrench, out["forces"], we=we)
    s = orc.grad_batch(b.counts, b.woff, P0, N0, b.wrench, out["forces"], wq=wq, we=we)
    np.testing.assert_allclose(s[0], a[0] + c[0], atol=1e-13)
    np.testing.assert_allclose(s[1], a[1] + c[1], atol=1e-13)
    # normal gradients carry no radial component (n is normalised inside)
    radial = np.einsum("gmc,gmc->gm", s[1], N0) / np.linalg.norm(N0, axis=-1)
    assert np.abs(radial).max() < 1e-12


def test_fd_check_detects_a_planted_error(orc):
    # Dropping the basis-Jacobian terms of the normal gradient (a plausible
    # mistake) must fail the comparison.
    b = wl.config(2, 4)
    P0 = b.points.astype(np.float64)
    N0 = b.normals.astype(np.float64)
    out = orc.solve_batch(b.counts, b.woff, P0, N0, b.mu, b.wrench)
    gP, gN = orc.grad_batch(b.counts, b.woff, P0, N0, b.wrench, out["forces"],
                            we=np.ones(b.n_grasps))
    fP, fN = _fd(orc, b, 1e-4)
    # rebuild dN with only the nhat column's own terms
    bad = np.zeros_like(gN)
    for g in range(b.n_grasps):
        G = orc.grasp_matrix(P0[g], N0[g], 20.0)
        Gb = np.zeros_like(G)
        for w in range(b.woff[g], b.woff[g + 1]):
            f = out["forces"][w]
            Gb += 2 * np.outer(G @ f - b.wrench[w], f)
        for i in range(b.m_max):
            nh = N0[g, i] / np.linalg.norm(N0[g, i])
            d = Gb[:3, 3 * i] + 20.0 * np.cross(Gb[3:, 3 * i], P0[g, i])
            bad[g, i] = (d - nh * (nh @ d)) / np.linalg.norm(N0[g, i])
    assert not all(_rel_ok(bad[g], fN[g]) for g in range(b.n_grasps))
    assert all(_rel_ok(gN[g], fN[g]) for g in range(b.n_grasps))
