"""GPU parity of the fine-stage surrogate energies with Detach (Sec. IV-C,
Eq. 10-11) against the FP64 oracle, through the C ABI.

Tolerance (FP32 kernel vs FP64 oracle), derived from the arithmetic per
contact: with u = 2^-24 the kernel's link-frame point c_l carries an error of
at most d_l = 16 u |c^f_w - T| (adjugate, determinant, one division; link
matrices with condition number ~1) and its c' an error of at most
d = 16 u (|c^f_w - T| + |c^f_w|).  Then
  Q', E^f_d:  sum_i (2 |c'_i - p_i| d_i + d_i^2) + 8 u value
  dL/dT:      2 (|w_q| + |w_e|) d_i + 4 u |g_i|                   (each entry)
  dL/dR:      tol(dL/dT) |c_l| + |g_i| d_l + 2 u |g_i| |c_l|     (each entry)
"""
import ctypes

import numpy as np
import pytest

from oracle import detach as od
from paper_2412_16490_amd import api
from paper_2412_16490_amd import workload as wl

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


@pytest.fixture(scope="module")
def solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = api.Solver(api.default_params())
    yield s
    s.close()


def _run(solver, fc, grads=True, counts=True, accumulate_from=None):
    import torch
    dfc = api.DeviceFineContacts(fc)
    G, m = dfc.n_grasps, dfc.m
    out = {"q_surr": torch.empty(G, device="cuda"), "e_dist": torch.empty(G, device="cuda")}
    if grads:
        if accumulate_from is None:
            out["dL_dR"] = torch.full((G, m, 3, 3), float("nan"), device="cuda")
            out["dL_dT"] = torch.full((G, m, 3), float("nan"), device="cuda")
        else:
            out["dL_dR"] = torch.as_tensor(accumulate_from[0], device="cuda").contiguous()
            out["dL_dT"] = torch.as_tensor(accumulate_from[1], device="cuda").contiguous()
    api.bodex_qp_detach_energy(solver.h, dfc, out["q_surr"], out["e_dist"], dfc.w_q, dfc.w_e,
                               out.get("dL_dR"), out.get("dL_dT"), accumulate=accumulate_from is not None,
                               counts=counts)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}


def _reference(fc, grasps=None, counts=True):
    sel = slice(None) if grasps is None else grasps
    f64 = lambda a: a[sel].astype(np.float64)
    cnt = fc.counts[sel] if counts else None
    return od.detach_energy(f64(fc.link_rot), f64(fc.link_trans), f64(fc.hand_fine), f64(fc.obj_fine),
                            f64(fc.obj_coarse), cnt, f64(fc.w_q), f64(fc.w_e))


def _check(fc, gpu, ref, grasps=None, grads=True, counts=True):
    sel = slice(None) if grasps is None else grasps
    R, T, cw = (fc.link_rot[sel].astype(np.float64), fc.link_trans[sel].astype(np.float64),
                fc.hand_fine[sel].astype(np.float64))
    pf, pc = fc.obj_fine[sel].astype(np.float64), fc.obj_coarse[sel].astype(np.float64)
    wq, we = fc.w_q[sel].astype(np.float64), fc.w_e[sel].astype(np.float64)
    G, M = T.shape[:2]
    cnt = fc.counts[sel] if counts else np.full(G, M)
    live = np.arange(M)[None, :] < cnt[:, None]
    v = np.linalg.norm(cw - T, axis=-1)
    d = 16 * U * (v + np.linalg.norm(cw, axis=-1))
    d_l = 16 * U * v
    Qp, Ed, dR, dT = ref
    for val, p, key in ((Qp, pc, "q_surr"), (Ed, pf, "e_dist")):
        dist = np.linalg.norm(cw - p, axis=-1)
        tol = np.sum(np.where(live, 2 * dist * d + d * d, 0.0), axis=1) + 8 * U * val
        err = np.abs(gpu[key][sel] - val)
        assert np.all(err <= tol), "%s: worst err/tol %.3g at grasp %d" % (key, np.max(err / tol),
                                                                           np.argmax(err / tol))
    if not grads:
        return
    gnorm = np.linalg.norm(dT, axis=-1)
    c_l = np.linalg.norm(np.linalg.solve(R, (cw - T)[..., None])[..., 0], axis=-1)
    tol_t = 2 * (np.abs(wq) + np.abs(we))[:, None] * d + 4 * U * gnorm
    tol_r = tol_t * c_l + gnorm * d_l + 2 * U * gnorm * c_l
    errT = np.abs(gpu["dL_dT"][sel] - dT).max(axis=-1)
    errR = np.abs(gpu["dL_dR"][sel] - dR).max(axis=(-1, -2))
    assert np.all(errT <= np.where(live, tol_t, 0.0)), "dL/dT: worst err/tol %.3g" % np.max(errT / (tol_t + 1e-300))
    assert np.all(errR <= np.where(live, tol_r, 0.0)), "dL/dR: worst err/tol %.3g" % np.max(errR / (tol_r + 1e-300))


@pytest.mark.parametrize("m,choices,G", [(5, None, 1000), (4, None, 777), (None, (3, 4, 5), 1234),
                                         (1, None, 300), (8, None, 129), (None, (1, 8), 500)])
def test_detach_parity(solver, m, choices, G):
    fc = wl.fine_contacts(40 + G, G, m=m or 5, m_choices=choices)
    print("detach parity G=%d m=%s choices=%s" % (G, m, choices), flush=True)
    gpu = _run(solver, fc)
    _check(fc, gpu, _reference(fc), )


def test_detach_without_gradients_and_without_counts(solver):
    fc = wl.fine_contacts(5, 600, m_choices=(2, 5))
    gpu = _run(solver, fc, grads=False, counts=False)
    _check(fc, gpu, _reference(fc, counts=False), grads=False, counts=False)


def test_detach_accumulates(solver):
    fc = wl.fine_contacts(6, 400, m_choices=(3, 5))
    rng = np.random.default_rng(1)
    G, M = fc.n_grasps, fc.m_max
    r0 = rng.standard_normal((G, M, 3, 3)).astype(np.float32)
    t0 = rng.standard_normal((G, M, 3)).astype(np.float32)
    gpu = _run(solver, fc, accumulate_from=(r0, t0))
    Qp, Ed, dR, dT = _reference(fc)
    gpu["dL_dR"] -= r0
    gpu["dL_dT"] -= t0
    # the subtraction of O(1) start values costs a few ulps of them
    live = (np.arange(M)[None, :] < fc.counts[:, None])
    assert np.all(gpu["dL_dR"][~live] == 0) and np.all(gpu["dL_dT"][~live] == 0)
    np.testing.assert_allclose(gpu["dL_dR"], dR, rtol=0, atol=4 * U * 8 + np.abs(dR).max() * 1e-5)
    np.testing.assert_allclose(gpu["dL_dT"], dT, rtol=0, atol=4 * U * 8 + np.abs(dT).max() * 1e-5)


def test_detach_unaligned_arrays(solver):
    # arrays 4- but not 16-byte aligned take the scalar-word staging
    import torch
    fc = wl.fine_contacts(9, 333, m_choices=(4, 5))
    dfc = api.DeviceFineContacts(fc)

    def shift(t):
        buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=t.device)
        v = buf[1:].view(t.shape)
        v.copy_(t)
        assert v.data_ptr() % 16 != 0
        return v

    for name in ("link_rot", "hand_fine", "obj_coarse"):
        setattr(dfc, name, shift(getattr(dfc, name)))
    G, m = dfc.n_grasps, dfc.m
    q = torch.empty(G, device="cuda")
    e = torch.empty(G, device="cuda")
    dR = shift(torch.zeros((G, m, 3, 3), device="cuda"))
    dT = torch.zeros((G, m, 3), device="cuda")
    api.bodex_qp_detach_energy(solver.h, dfc, q, e, dfc.w_q, dfc.w_e, dR, dT)
    torch.cuda.synchronize()
    gpu = {"q_surr": q.cpu().numpy().astype(np.float64), "e_dist": e.cpu().numpy().astype(np.float64),
           "dL_dR": dR.cpu().numpy().astype(np.float64), "dL_dT": dT.cpu().numpy().astype(np.float64)}
    _check(fc, gpu, _reference(fc))


def test_detach_zero_weights_give_zero_gradient(solver):
    import torch
    fc = wl.fine_contacts(7, 300)
    dfc = api.DeviceFineContacts(fc)
    G, m = dfc.n_grasps, dfc.m
    q = torch.empty(G, device="cuda")
    e = torch.empty(G, device="cuda")
    dR = torch.full((G, m, 3, 3), 5.0, device="cuda")
    dT = torch.full((G, m, 3), 5.0, device="cuda")
    api.bodex_qp_detach_energy(solver.h, dfc, q, e, None, None, dR, dT)
    torch.cuda.synchronize()
    assert not dR.any().item() and not dT.any().item()


def test_detach_full_size_sampled(solver):
    # the benchmark's shape: 2^20 grasps x 5 fingertips, one launch
    G = 1 << 20
    fc = wl.fine_contacts(16496, G, m=5)
    gpu = _run(solver, fc)
    rng = np.random.default_rng(2)
    grasps = np.unique(np.concatenate([rng.integers(0, G, 400), [0, G - 1], np.arange(G - 60, G)]))
    _check(fc, {k: v for k, v in gpu.items()}, _reference(fc, grasps), grasps=grasps)
    assert np.all(np.isfinite(gpu["q_surr"])) and np.all(np.isfinite(gpu["dL_dR"]))


def test_detach_empty_and_argument_errors(solver):
    import torch
    fc = wl.fine_contacts(8, 4)
    dfc = api.DeviceFineContacts(fc)
    q = torch.empty(4, device="cuda")
    e = torch.empty(4, device="cuda")
    f = dfc.c_struct()
    f.n_grasps = 0
    L = api.lib()
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    assert L.bodex_qp_detach_energy(solver.h, ctypes.byref(f), None, None, None, None, None, None, 0) == 0
    for m in (0, 9):
        f = dfc.c_struct()
        f.m = m
        assert L.bodex_qp_detach_energy(solver.h, ctypes.byref(f), None, None, P(q), P(e), None, None,
                                        0) == api.EINVAL
    f = dfc.c_struct()
    dR = torch.zeros((4, 5, 3, 3), device="cuda")
    assert L.bodex_qp_detach_energy(solver.h, ctypes.byref(f), None, None, P(q), P(e), P(dR), None,
                                    0) == api.EINVAL
    assert L.bodex_qp_detach_energy(solver.h, ctypes.byref(f), None, None, None, P(e), None, None,
                                    0) == api.EINVAL
    assert b"NULL" in L.bodex_qp_last_error(solver.h)
