"""ctypes binding of the C ABI in include/bodex_qp.h (argument marshalling only).

Every step of the solve runs in the HIP library; this module converts torch
tensors to device pointers and host arrays to C arrays.  If the library has not
been built, importing works but every call raises -- there is no fallback.

Functions keep the C names (``bodex_qp_create``, ``bodex_qp_solve``,
``bodex_qp_backward``, ``bodex_qp_destroy``); ``Solver`` bundles them.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbodex_qp.so")

OK, EINVAL, EHIP, EBUDGET, EINFEAS, EUNSUP, ENODEV = 0, -1, -2, -3, -4, -5, -6
ST_CONVERGED, ST_MAX_ITER, ST_NONFINITE, ST_FP64_CHOL, ST_POLISH_REJ, ST_POLISHED = (
    0x01, 0x02, 0x04, 0x08, 0x10, 0x20)
F_WARM_START, F_POLISH, F_ADAPTIVE_RHO, F_BATCHED, F_GRAPH, F_TIMING = 0x01, 0x02, 0x04, 0x08, 0x10, 0x20
F_SIGNED_DIST = 0x40
CONE_PYRAMID8, CONE_CIRCULAR = 0, 1


class BodexError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("bodex_qp error %d: %s" % (code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("m_max", ctypes.c_int), ("s_max", ctypes.c_int),
        ("force_max", ctypes.c_float), ("gamma", ctypes.c_float),
        ("beta", ctypes.c_float), ("eps_reg", ctypes.c_float),
        ("torque_scale", ctypes.c_float), ("tol_rel", ctypes.c_float),
        ("max_iters", ctypes.c_int), ("rho0", ctypes.c_float),
        ("alpha", ctypes.c_float), ("check_every", ctypes.c_int),
        ("rho_min", ctypes.c_float), ("rho_max", ctypes.c_float),
        ("rho_hysteresis", ctypes.c_float), ("fp64_cond", ctypes.c_float),
        ("polish_steps", ctypes.c_int), ("polish_chunk", ctypes.c_int),
        ("flags", ctypes.c_uint), ("admm_waves", ctypes.c_int),
        ("admm_tol", ctypes.c_float), ("friction_cone", ctypes.c_int),
    ]


class Batch(ctypes.Structure):
    _fields_ = [
        ("n_grasps", ctypes.c_int), ("n_qps", ctypes.c_int),
        ("contact_count", ctypes.POINTER(ctypes.c_int)),
        ("wrench_offset", ctypes.POINTER(ctypes.c_int)),
        ("points", ctypes.c_void_p), ("normals", ctypes.c_void_p),
        ("mu", ctypes.c_void_p), ("wrench_dir", ctypes.c_void_p),
    ]


class FineContacts(ctypes.Structure):
    _fields_ = [
        ("n_grasps", ctypes.c_int), ("m", ctypes.c_int),
        ("contact_count", ctypes.c_void_p), ("link_rot", ctypes.c_void_p),
        ("link_trans", ctypes.c_void_p), ("hand_fine", ctypes.c_void_p),
        ("obj_fine", ctypes.c_void_p), ("obj_coarse", ctypes.c_void_p),
    ]


class Hand(ctypes.Structure):
    _fields_ = [
        ("n_grasps", ctypes.c_int), ("m", ctypes.c_int),
        ("contact_count", ctypes.c_void_p), ("tip_local", ctypes.c_void_p),
        ("semi_axes", ctypes.c_void_p), ("hand_rot", ctypes.c_void_p),
        ("hand_trans", ctypes.c_void_p),
    ]


class Descent(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int), ("w_qp", ctypes.c_float), ("w_dist", ctypes.c_float),
        ("radius", ctypes.c_float), ("offset", ctypes.c_float),
        ("step_rot", ctypes.c_float), ("step_trans", ctypes.c_float),
    ]


class State(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("rho", ctypes.c_void_p),
                ("r", ctypes.c_void_p), ("stride", ctypes.c_int), ("rho_len", ctypes.c_int),
                ("qp_offset", ctypes.POINTER(ctypes.c_int)), ("grasp_offset", ctypes.POINTER(ctypes.c_int))]


class Result(ctypes.Structure):
    _fields_ = [
        ("forces", ctypes.c_void_p), ("qp_obj", ctypes.c_void_p),
        ("energy", ctypes.c_void_p), ("kkt_rel", ctypes.c_void_p),
        ("iters", ctypes.c_void_p), ("status", ctypes.c_void_p),
        ("state", State), ("polish_flops", ctypes.c_void_p),
    ]


_lib = None
_lock = threading.Lock()


def lib():
    """The loaded library; raises when it is missing (no CPU fallback)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built; run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        L.bodex_qp_default_params.argtypes = [ctypes.POINTER(Params)]
        L.bodex_qp_default_params.restype = None
        L.bodex_qp_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]
        L.bodex_qp_create.restype = ctypes.c_int
        L.bodex_qp_set_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.bodex_qp_set_stream.restype = ctypes.c_int
        L.bodex_qp_solve.argtypes = [ctypes.c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(Result)]
        L.bodex_qp_solve.restype = ctypes.c_int
        L.bodex_qp_solve_static.argtypes = [ctypes.c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(Result)]
        L.bodex_qp_solve_static.restype = ctypes.c_int
        L.bodex_qp_backward.argtypes = [ctypes.c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(State),
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int]
        L.bodex_qp_backward.restype = ctypes.c_int
        L.bodex_qp_destroy.argtypes = [ctypes.c_void_p]
        L.bodex_qp_destroy.restype = ctypes.c_int
        L.bodex_qp_last_error.argtypes = [ctypes.c_void_p]
        L.bodex_qp_last_error.restype = ctypes.c_char_p
        L.bodex_qp_state_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.bodex_qp_state_bytes.restype = ctypes.c_size_t
        L.bodex_qp_last_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.bodex_qp_last_stats.restype = ctypes.c_int
        L.bodex_qp_effective_params.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(ctypes.c_float),
                                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_int)]
        L.bodex_qp_effective_params.restype = ctypes.c_int
        L.bodex_qp_kernel_times.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                            ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
        L.bodex_qp_kernel_times.restype = ctypes.c_int
        L.bodex_qp_detach_energy.argtypes = [ctypes.c_void_p, ctypes.POINTER(FineContacts)] + [ctypes.c_void_p] * 6 + [
            ctypes.c_int]
        L.bodex_qp_detach_energy.restype = ctypes.c_int
        L.bodex_qp_contact_query.argtypes = [ctypes.c_void_p, ctypes.POINTER(Hand)] + [ctypes.c_void_p] * 3
        L.bodex_qp_contact_query.restype = ctypes.c_int
        L.bodex_qp_pose_gradient.argtypes = [ctypes.c_void_p, ctypes.POINTER(Hand), ctypes.c_void_p,
                                             ctypes.c_void_p] + [ctypes.c_float] * 3 + [ctypes.c_void_p] * 3
        L.bodex_qp_pose_gradient.restype = ctypes.c_int
        L.bodex_qp_descend.argtypes = [ctypes.c_void_p, ctypes.POINTER(Hand), ctypes.POINTER(Batch),
                                       ctypes.POINTER(Descent), ctypes.POINTER(Result), ctypes.c_void_p]
        L.bodex_qp_descend.restype = ctypes.c_int
        _lib = L
        return L


EXPORTED = ("bodex_qp_default_params", "bodex_qp_create", "bodex_qp_set_stream",
            "bodex_qp_solve", "bodex_qp_solve_static", "bodex_qp_backward", "bodex_qp_destroy",
            "bodex_qp_last_error", "bodex_qp_state_bytes", "bodex_qp_last_stats",
            "bodex_qp_kernel_times", "bodex_qp_detach_energy", "bodex_qp_contact_query",
            "bodex_qp_pose_gradient", "bodex_qp_descend", "bodex_qp_effective_params")


def default_params(**overrides) -> Params:
    p = Params()
    lib().bodex_qp_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if k == "flags_set":
            p.flags |= int(v)
        elif k == "flags_clear":
            p.flags &= ~int(v)
        else:
            setattr(p, k, v)
    return p


def bodex_qp_effective_params(p: Params, n_qps: int) -> dict:
    """The values the library takes for the parameters whose rule it owns:
    ADMM's tolerance, iteration cap and check period, and the polish's
    factorisation budget, for a solve of n_qps QPs (no device needed)."""
    tol, mi, ce, pc = ctypes.c_float(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().bodex_qp_effective_params(ctypes.byref(p), int(n_qps), ctypes.byref(tol), ctypes.byref(mi),
                                           ctypes.byref(ce), ctypes.byref(pc)))
    return {"admm_tol": tol.value, "max_iters": mi.value, "check_every": ce.value, "polish_chunk": pc.value}


def admm_check_period(p: Params) -> int:
    """The residual-check period the library's ADMM uses for these parameters."""
    return bodex_qp_effective_params(p, 0)["check_every"]


def _check(rc, handle=None):
    if rc != 0:
        msg = lib().bodex_qp_last_error(handle)
        raise BodexError(rc, msg.decode() if msg else "")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def bodex_qp_create(params: Params, device: int = 0, stream=None, budget: int = 0):
    h = ctypes.c_void_p()
    s = ctypes.c_void_p(stream) if stream else None
    _check(lib().bodex_qp_create(ctypes.byref(params), int(device), s, ctypes.c_size_t(budget),
                                 ctypes.byref(h)))
    return h


def bodex_qp_destroy(h) -> None:
    if h:
        _check(lib().bodex_qp_destroy(h))


def bodex_qp_state_bytes(n_grasps: int, n_qps: int, m_max: int) -> int:
    return int(lib().bodex_qp_state_bytes(n_grasps, n_qps, m_max))


class DeviceBatch:
    """Device copies of a workload.Batch plus its host CSR arrays."""

    def __init__(self, batch, device="cuda"):
        import torch
        self.counts = np.ascontiguousarray(batch.counts, dtype=np.int32)
        self.woff = np.ascontiguousarray(batch.woff, dtype=np.int32)
        self.points = torch.as_tensor(np.ascontiguousarray(batch.points, np.float32), device=device)
        self.normals = torch.as_tensor(np.ascontiguousarray(batch.normals, np.float32), device=device)
        self.mu = torch.as_tensor(np.ascontiguousarray(batch.mu, np.float32), device=device)
        self.wrench = torch.as_tensor(np.ascontiguousarray(batch.wrench, np.float32), device=device)
        self.n_grasps = int(self.counts.shape[0])
        self.n_qps = int(self.woff[-1])
        self.m_max = int(self.points.shape[1])

    def c_batch(self) -> Batch:
        b = Batch()
        b.n_grasps = self.n_grasps
        b.n_qps = self.n_qps
        b.contact_count = self.counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        b.wrench_offset = self.woff.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        b.points = _ptr(self.points)
        b.normals = _ptr(self.normals)
        b.mu = _ptr(self.mu)
        b.wrench_dir = _ptr(self.wrench)
        return b


def new_state(n_grasps, n_qps, m_max, device="cuda", cone=False, residual=True):
    """Caller-held ADMM state; cone: the circular-cone layout (3 m_max + 1
    rows of z and y instead of 9 m_max + 1); residual: also the wrench
    residual the backward uses (state.r)."""
    import torch
    nr = (3 if cone else 9) * m_max + 1
    st = {
        "x": torch.zeros((3 * m_max, n_qps), dtype=torch.float32, device=device),
        "z": torch.zeros((nr, n_qps), dtype=torch.float32, device=device),
        "y": torch.zeros((nr, n_qps), dtype=torch.float32, device=device),
        "rho": torch.zeros((n_grasps,), dtype=torch.float32, device=device),
    }
    if residual:
        st["r"] = torch.zeros((6, n_qps), dtype=torch.float32, device=device)
    return st


def new_result(n_grasps, n_qps, m_max, device="cuda", polish_flops=False):
    import torch
    out = {
        "forces": torch.empty((n_qps, 3 * m_max), dtype=torch.float32, device=device),
        "qp_obj": torch.empty((n_qps,), dtype=torch.float32, device=device),
        "energy": torch.empty((n_grasps,), dtype=torch.float32, device=device),
        "kkt_rel": torch.empty((n_qps,), dtype=torch.float32, device=device),
        "iters": torch.empty((n_qps,), dtype=torch.int32, device=device),
        "status": torch.empty((n_qps,), dtype=torch.uint8, device=device),
    }
    if polish_flops:
        out["polish_flops"] = torch.zeros((n_qps,), dtype=torch.float32, device=device)
    return out


def _c_state(st) -> State:
    """A state dict (x, z, y, rho[, r]) or a pooled view of one (the same plus
    'qp_offset' and 'grasp_offset' host int32 arrays for the batch's grasps;
    the pool's column count and rho length are taken from the arrays)."""
    s = State()
    if st is not None:
        s.x, s.z, s.y, s.rho = _ptr(st["x"]), _ptr(st["z"]), _ptr(st["y"]), _ptr(st["rho"])
        s.r = _ptr(st["r"]) if st.get("r") is not None else None
        if st.get("qp_offset") is not None:
            qo = np.ascontiguousarray(st["qp_offset"], np.int32)
            go = np.ascontiguousarray(st["grasp_offset"], np.int32)
            st["_keep"] = (qo, go)  # alive for the call
            s.stride = int(st["x"].shape[1])
            s.rho_len = int(st["rho"].shape[0])
            s.qp_offset = qo.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
            s.grasp_offset = go.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    return s


def _c_result(result: dict, state: dict | None) -> Result:
    r = Result()
    r.forces = _ptr(result["forces"])
    r.qp_obj = _ptr(result["qp_obj"])
    r.energy = _ptr(result["energy"])
    r.kkt_rel = _ptr(result["kkt_rel"])
    r.iters = _ptr(result["iters"])
    r.status = _ptr(result["status"])
    r.state = _c_state(state)
    r.polish_flops = _ptr(result["polish_flops"]) if result.get("polish_flops") is not None else None
    return r


def _c_result(result: dict, state: dict | None):
    r = Result()
    r.forces = _ptr(result["forces"])
    r.qp_obj = _ptr(result["qp_obj"])
    r.energy = _ptr(result["energy"])
    r.kkt_rel = _ptr(result["kkt_rel"])
    r.iters = _ptr(result["iters"])
    r.status = _ptr(result["status"])
    r.state = _c_state(state)
    r.polish_flops = _ptr(result["polish_flops"]) if result.get("polish_flops") is not None else None
    return r


def bodex_qp_solve(h, batch: DeviceBatch, result: dict, state: dict | None = None) -> None:
    r = _c_result(result, state)
    b = batch.c_batch()
    _check(lib().bodex_qp_solve(h, ctypes.byref(b), ctypes.byref(r)), h)


def bodex_qp_solve_static(h, batch: DeviceBatch, result: dict, state: dict) -> None:
    """The allocation-free solve: descriptor in the library's static device
    scratch, state from the caller."""
    r = _c_result(result, state)
    b = batch.c_batch()
    _check(lib().bodex_qp_solve_static(h, ctypes.byref(b), ctypes.byref(r)), h)


def bodex_qp_backward(h, batch: DeviceBatch, state: dict, dL_dE=None, dL_dQ=None,
                      dL_dpoints=None, dL_dnormals=None, accumulate: bool = False) -> None:
    b = batch.c_batch()
    s = _c_state(state)
    _check(lib().bodex_qp_backward(h, ctypes.byref(b), ctypes.byref(s), _ptr(dL_dE), _ptr(dL_dQ),
                                   _ptr(dL_dpoints), _ptr(dL_dnormals), 1 if accumulate else 0), h)


def last_stats(h):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().bodex_qp_last_stats(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), h)
    return {"launches": a.value, "graph_replays": b.value, "tiles": c.value}


def bodex_qp_kernel_times(h):
    a, b, c = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
    _check(lib().bodex_qp_kernel_times(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), h)
    return {"admm_ms": a.value, "finalize_ms": b.value, "backward_ms": c.value}


class DeviceFineContacts:
    """Device copies of a workload.FineContacts (all arrays on the GPU)."""

    def __init__(self, fc, device="cuda"):
        import torch
        t = lambda a, dt=np.float32: torch.as_tensor(np.ascontiguousarray(a, dt), device=device)
        self.counts = t(fc.counts, np.int32)
        self.link_rot = t(fc.link_rot)
        self.link_trans = t(fc.link_trans)
        self.hand_fine = t(fc.hand_fine)
        self.obj_fine = t(fc.obj_fine)
        self.obj_coarse = t(fc.obj_coarse)
        self.w_q = t(fc.w_q)
        self.w_e = t(fc.w_e)
        self.n_grasps = int(self.link_trans.shape[0])
        self.m = int(self.link_trans.shape[1])

    def c_struct(self, counts=True) -> FineContacts:
        f = FineContacts()
        f.n_grasps = self.n_grasps
        f.m = self.m
        f.contact_count = _ptr(self.counts) if counts else None
        f.link_rot = _ptr(self.link_rot)
        f.link_trans = _ptr(self.link_trans)
        f.hand_fine = _ptr(self.hand_fine)
        f.obj_fine = _ptr(self.obj_fine)
        f.obj_coarse = _ptr(self.obj_coarse)
        return f


def bodex_qp_detach_energy(h, fc: DeviceFineContacts, q_surr, e_dist, w_q=None, w_e=None,
                           dL_dR=None, dL_dT=None, accumulate: bool = False, counts: bool = True) -> None:
    f = fc.c_struct(counts)
    _check(lib().bodex_qp_detach_energy(h, ctypes.byref(f), _ptr(w_q), _ptr(w_e), _ptr(q_surr), _ptr(e_dist),
                                        _ptr(dL_dR), _ptr(dL_dT), 1 if accumulate else 0), h)


class DeviceHand:
    """Device copies of a workload.HandBatch: the hand side (fingertips,
    object, pose; the pose tensors are updated in place by descend) and the
    QP side (host CSR arrays, friction, desired wrenches)."""

    def __init__(self, hb, device="cuda"):
        import torch
        t = lambda a, dt=np.float32: torch.as_tensor(np.ascontiguousarray(a, dt), device=device).clone()
        self.counts = np.ascontiguousarray(hb.counts, dtype=np.int32)
        self.woff = np.ascontiguousarray(hb.woff, dtype=np.int32)
        self.d_counts = t(hb.counts, np.int32)
        self.tip = t(hb.tip_local)
        self.axes = t(hb.semi_axes)
        self.rot = t(hb.rot)
        self.trans = t(hb.trans)
        self.mu = t(hb.mu)
        self.wrench = t(hb.wrench)
        self.n_grasps = int(self.counts.shape[0])
        self.n_qps = int(self.woff[-1])
        self.m = int(self.tip.shape[1])

    def c_struct(self, counts=True) -> Hand:
        h = Hand()
        h.n_grasps = self.n_grasps
        h.m = self.m
        h.contact_count = _ptr(self.d_counts) if counts else None
        h.tip_local = _ptr(self.tip)
        h.semi_axes = _ptr(self.axes)
        h.hand_rot = _ptr(self.rot)
        h.hand_trans = _ptr(self.trans)
        return h

    def c_qp(self) -> Batch:
        """The QP side for descend (points and normals NULL)."""
        b = Batch()
        b.n_grasps = self.n_grasps
        b.n_qps = self.n_qps
        b.contact_count = self.counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        b.wrench_offset = self.woff.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        b.points = None
        b.normals = None
        b.mu = _ptr(self.mu)
        b.wrench_dir = _ptr(self.wrench)
        return b


def bodex_qp_contact_query(h, hand: DeviceHand, points, normals, dist=None, counts: bool = True) -> None:
    c = hand.c_struct(counts)
    _check(lib().bodex_qp_contact_query(h, ctypes.byref(c), _ptr(points), _ptr(normals), _ptr(dist)), h)


def bodex_qp_pose_gradient(h, hand: DeviceHand, dL_dpoints=None, dL_dnormals=None, w_dist=0.0, radius=0.0,
                           offset=0.0, e_dist=None, dL_drot=None, dL_dtrans=None, counts: bool = True) -> None:
    c = hand.c_struct(counts)
    _check(lib().bodex_qp_pose_gradient(h, ctypes.byref(c), _ptr(dL_dpoints), _ptr(dL_dnormals), float(w_dist),
                                        float(radius), float(offset), _ptr(e_dist), _ptr(dL_drot),
                                        _ptr(dL_dtrans)), h)


def descent(iters=20, w_qp=1.0, w_dist=1000.0, radius=0.01, offset=0.0, step_rot=2e-3,
            step_trans=1e-5) -> Descent:
    """Descent parameters (defaults: the synthetic coarse-stage setting)."""
    d = Descent()
    d.iters, d.w_qp, d.w_dist, d.radius, d.offset = int(iters), w_qp, w_dist, radius, offset
    d.step_rot, d.step_trans = step_rot, step_trans
    return d


def bodex_qp_descend(h, hand: DeviceHand, d: Descent, result: dict, state: dict | None = None,
                     loss_trace=None) -> None:
    c = hand.c_struct(counts=False)
    b = hand.c_qp()
    r = _c_result(result, state)
    _check(lib().bodex_qp_descend(h, ctypes.byref(c), ctypes.byref(b), ctypes.byref(d), ctypes.byref(r),
                                  _ptr(loss_trace)), h)


class Solver:
    """A handle on one device and stream (torch's current stream by default)."""

    def __init__(self, params: Params | None = None, device: int = 0, stream=None,
                 budget: int = 0, **overrides):
        import torch
        self.params = params if params is not None else default_params(**overrides)
        if params is not None:
            for k, v in overrides.items():
                setattr(self.params, k, v)
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.stream = stream
        self.h = bodex_qp_create(self.params, device, stream, budget)

    def solve(self, batch: DeviceBatch, state: dict | None = None, result: dict | None = None):
        if result is None:
            result = new_result(batch.n_grasps, batch.n_qps, self.params.m_max)
        bodex_qp_solve(self.h, batch, result, state)
        return result

    def backward(self, batch: DeviceBatch, state: dict, dL_dE=None, dL_dQ=None, out=None,
                 accumulate=False):
        import torch
        if out is None:
            out = (torch.zeros_like(batch.points), torch.zeros_like(batch.normals))
        bodex_qp_backward(self.h, batch, state, dL_dE, dL_dQ, out[0], out[1], accumulate)
        return out

    def detach_energy(self, fc: DeviceFineContacts, grads=True, out=None, accumulate=False):
        """Q', E^f_d [G] and, with grads, dL/dR [G][m][3][3], dL/dT [G][m][3]
        for the weights fc.w_q, fc.w_e."""
        import torch
        G, m = fc.n_grasps, fc.m
        dev = fc.link_trans.device
        if out is None:
            out = {"q_surr": torch.empty(G, dtype=torch.float32, device=dev),
                   "e_dist": torch.empty(G, dtype=torch.float32, device=dev)}
            if grads:
                out["dL_dR"] = torch.zeros((G, m, 3, 3), dtype=torch.float32, device=dev)
                out["dL_dT"] = torch.zeros((G, m, 3), dtype=torch.float32, device=dev)
        bodex_qp_detach_energy(self.h, fc, out["q_surr"], out["e_dist"], fc.w_q, fc.w_e,
                               out.get("dL_dR"), out.get("dL_dT"), accumulate)
        return out

    def contact_query(self, hand: DeviceHand, out=None):
        """points, normals [G][m][3] and signed distances [G][m] of the pose."""
        import torch
        G, m = hand.n_grasps, hand.m
        dev = hand.tip.device
        if out is None:
            out = {"points": torch.empty((G, m, 3), dtype=torch.float32, device=dev),
                   "normals": torch.empty((G, m, 3), dtype=torch.float32, device=dev),
                   "dist": torch.empty((G, m), dtype=torch.float32, device=dev)}
        bodex_qp_contact_query(self.h, hand, out["points"], out["normals"], out.get("dist"))
        return out

    def pose_gradient(self, hand: DeviceHand, dL_dpoints=None, dL_dnormals=None, w_dist=0.0, radius=0.0,
                      offset=0.0):
        """E^c_d [G], dL/domega [G][3], dL/dT [G][3]."""
        import torch
        G = hand.n_grasps
        dev = hand.tip.device
        out = {"e_dist": torch.empty(G, dtype=torch.float32, device=dev),
               "dL_drot": torch.empty((G, 3), dtype=torch.float32, device=dev),
               "dL_dtrans": torch.empty((G, 3), dtype=torch.float32, device=dev)}
        bodex_qp_pose_gradient(self.h, hand, dL_dpoints, dL_dnormals, w_dist, radius, offset,
                               out["e_dist"], out["dL_drot"], out["dL_dtrans"])
        return out

    def descend(self, hand: DeviceHand, d: Descent | None = None, state: dict | None = None,
                result: dict | None = None, trace: bool = True):
        """Run d.iters descent steps (hand.rot / hand.trans updated in place);
        returns the last step's QP result and the loss trace [iters][G]."""
        import torch
        d = d if d is not None else descent()
        if result is None:
            result = new_result(hand.n_grasps, hand.n_qps, self.params.m_max)
        tr = torch.empty((d.iters, hand.n_grasps), dtype=torch.float32, device=hand.tip.device) \
            if trace and d.iters > 0 else None
        bodex_qp_descend(self.h, hand, d, result, state, tr)
        return result, tr

    def stats(self):
        return last_stats(self.h)

    def kernel_times(self):
        return bodex_qp_kernel_times(self.h)

    def close(self):
        if getattr(self, "h", None):
            bodex_qp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
