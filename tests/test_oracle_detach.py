"""Pins of the fine-stage surrogate oracle (Sec. IV-C, Eq. 10-11) against
what the definitions fix, independently of the oracle's own formulas:

* forward values: Detach changes no value, so Q' and E^f_d are the plain
  squared distances of the fine nearest points c^f_{i,w} -- also for link
  matrices that are not rotations (the link-frame point uses R^{-1}, not R^T);
* the gradient equals reverse-mode autodiff (torch, FP64) of Eq. 11 written
  with an explicit detach, and central finite differences in (R_i, T_i) with
  the link-frame point held fixed (the meaning of Detach);
* padding contacts add nothing and get zero gradients.
"""
import numpy as np
import pytest

from oracle import detach as od
from paper_2412_16490_amd import workload as wl


def _inputs(seed=3, G=6, m_choices=(3, 4, 5)):
    f = wl.fine_contacts(seed, G, m_choices=m_choices)
    return (f.link_rot.astype(np.float64), f.link_trans.astype(np.float64), f.hand_fine.astype(np.float64),
            f.obj_fine.astype(np.float64), f.obj_coarse.astype(np.float64), f.counts,
            f.w_q.astype(np.float64), f.w_e.astype(np.float64))


def test_values_are_plain_distances_of_fine_points():
    R, T, cw, pf, pc, cnt, wq, we = _inputs()
    Qp, Ed, _, _ = od.detach_energy(R, T, cw, pf, pc, cnt, wq, we)
    for g in range(len(cnt)):
        m = cnt[g]
        assert Qp[g] == pytest.approx(np.sum((cw[g, :m] - pc[g, :m]) ** 2), rel=1e-12)
        assert Ed[g] == pytest.approx(np.sum((cw[g, :m] - pf[g, :m]) ** 2), rel=1e-12)


def test_values_with_general_link_matrices_use_the_inverse():
    R, T, cw, pf, pc, cnt, wq, we = _inputs(seed=5)
    rng = np.random.default_rng(7)
    A = R * rng.uniform(0.5, 2.0, size=R.shape[:-2] + (3, 1))  # rows scaled: not orthogonal
    Qp, Ed, _, _ = od.detach_energy(A, T, cw, pf, pc, cnt, wq, we)
    for g in range(len(cnt)):
        m = cnt[g]
        assert Qp[g] == pytest.approx(np.sum((cw[g, :m] - pc[g, :m]) ** 2), rel=1e-10)
        assert Ed[g] == pytest.approx(np.sum((cw[g, :m] - pf[g, :m]) ** 2), rel=1e-10)


def test_gradient_matches_autodiff_with_detach():
    torch = pytest.importorskip("torch")
    R, T, cw, pf, pc, cnt, wq, we = _inputs(seed=11)
    _, _, dR, dT = od.detach_energy(R, T, cw, pf, pc, cnt, wq, we)
    Rt = torch.tensor(R, dtype=torch.float64, requires_grad=True)
    Tt = torch.tensor(T, dtype=torch.float64, requires_grad=True)
    loss = 0.0
    for g in range(len(cnt)):
        for i in range(cnt[g]):
            cwt = torch.tensor(cw[g, i], dtype=torch.float64)
            # Eq. 11 as written: link-frame point through R^{-1}, then detached
            c_l = torch.linalg.inv(Rt[g, i]) @ (cwt - Tt[g, i])
            c_w = Rt[g, i] @ c_l.detach() + Tt[g, i]
            loss = loss + wq[g] * torch.sum((c_w - torch.tensor(pc[g, i])) ** 2)
            loss = loss + we[g] * torch.sum((c_w - torch.tensor(pf[g, i])) ** 2)
    loss.backward()
    np.testing.assert_allclose(dR, Rt.grad.numpy(), rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(dT, Tt.grad.numpy(), rtol=1e-10, atol=1e-14)


def _loss_fixed_link_point(R, T, c_l, pf, pc, wq, we):
    c_w = R @ c_l + T
    return wq * np.sum((c_w - pc) ** 2) + we * np.sum((c_w - pf) ** 2)


def test_gradient_matches_finite_differences_with_link_point_fixed():
    R, T, cw, pf, pc, cnt, wq, we = _inputs(seed=13, G=3)
    _, _, dR, dT = od.detach_energy(R, T, cw, pf, pc, cnt, wq, we)
    h = 1e-6
    for g in range(len(cnt)):
        for i in range(cnt[g]):
            c_l = np.linalg.solve(R[g, i], cw[g, i] - T[g, i])
            args = (pf[g, i], pc[g, i], wq[g], we[g])
            for a in range(3):
                for b in range(3):
                    E = np.zeros((3, 3))
                    E[a, b] = h
                    fd = (_loss_fixed_link_point(R[g, i] + E, T[g, i], c_l, *args)
                          - _loss_fixed_link_point(R[g, i] - E, T[g, i], c_l, *args)) / (2 * h)
                    assert dR[g, i, a, b] == pytest.approx(fd, rel=1e-6, abs=1e-12)
                e = np.zeros(3)
                e[a] = h
                fd = (_loss_fixed_link_point(R[g, i], T[g, i] + e, c_l, *args)
                      - _loss_fixed_link_point(R[g, i], T[g, i] - e, c_l, *args)) / (2 * h)
                assert dT[g, i, a] == pytest.approx(fd, rel=1e-6, abs=1e-12)


def test_transposed_gradient_would_fail_the_difference_check():
    # the check above is sensitive to the outer product's orientation
    R, T, cw, pf, pc, cnt, wq, we = _inputs(seed=13, G=1, m_choices=(5,))
    _, _, dR, _ = od.detach_energy(R, T, cw, pf, pc, cnt, wq, we)
    c_l = np.linalg.solve(R[0, 0], cw[0, 0] - T[0, 0])
    h = 1e-6
    fd = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            E = np.zeros((3, 3))
            E[a, b] = h
            fd[a, b] = (_loss_fixed_link_point(R[0, 0] + E, T[0, 0], c_l, pf[0, 0], pc[0, 0], wq[0], we[0])
                        - _loss_fixed_link_point(R[0, 0] - E, T[0, 0], c_l, pf[0, 0], pc[0, 0], wq[0], we[0])) / (2 * h)
    assert np.allclose(dR[0, 0], fd, rtol=1e-6, atol=1e-12)
    assert not np.allclose(dR[0, 0].T, fd, rtol=1e-3, atol=1e-9)


def test_padding_contacts_are_inert():
    R, T, cw, pf, pc, cnt, wq, we = _inputs(seed=17, G=8, m_choices=(2, 5))
    Qp, Ed, dR, dT = od.detach_energy(R, T, cw, pf, pc, cnt, wq, we)
    R2, T2, cw2 = R.copy(), T.copy(), cw.copy()
    for g in range(len(cnt)):
        R2[g, cnt[g]:] = 3.0
        T2[g, cnt[g]:] = 1.0
        cw2[g, cnt[g]:] = -1.0
        assert np.all(dR[g, cnt[g]:] == 0) and np.all(dT[g, cnt[g]:] == 0)
    Qp2, Ed2, _, _ = od.detach_energy(R2, T2, cw2, pf, pc, cnt, wq, we)
    np.testing.assert_array_equal(Qp, Qp2)
    np.testing.assert_array_equal(Ed, Ed2)


def test_zero_weights_give_zero_gradient():
    R, T, cw, pf, pc, cnt, _, _ = _inputs(seed=19)
    _, _, dR, dT = od.detach_energy(R, T, cw, pf, pc, cnt)
    assert not dR.any() and not dT.any()
