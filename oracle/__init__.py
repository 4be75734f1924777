"""FP64 CPU oracle for the BODex lower-level contact-force QP (arXiv 2412.16490).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product path (the HIP
library and its Python binding) never touches it, and the two share no code.

The arithmetic lives in ``oracle.c`` (plain C11, FP64); this module compiles it
with gcc on first use and exposes numpy wrappers:

* ``frame``/``grasp_matrix``  -- Sec. III Eq. 2 with the torque rows scaled by
  kappa and the tangent basis of Duff et al. 2017 (n = d x e).
* ``constraints``              -- the 8-facet inscribed pyramid of Sec. IV-A,
  0 <= f_1 <= fmax (Eq. 1) and sum f_1 >= gamma (Eq. 9), one-sided form.
* ``qp_solve``/``solve_batch`` -- Eq. 7-9 with the pyramid, solved exactly by
  the Goldfarb-Idnani dual active-set method.
* ``grad_batch``               -- Danskin gradient of the energy sum_j Q_j
  (Sec. IV-A, Eq. 3) chained to contact points and normals.
* ``admm_rel_kkt``             -- relative KKT residual of an ADMM-form state.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_LIB names another library path and ORACLE_CFLAGS adds compiler
# flags (a sanitizer build of the same source, kept apart from the default)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_EXTRA = os.environ.get("ORACLE_CFLAGS", "").split()
_lock = threading.Lock()
_lib = None

MAX_CONTACTS = 8


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, -O2, FP64)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-D_GNU_SOURCE",
           "-ffp-contract=off", "-Wall", "-Wextra", "-Wno-unused-parameter",
           *_EXTRA, _SRC, "-o", tmp, "-lm", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("beta", ctypes.c_double),
                ("eps", ctypes.c_double), ("fmax", ctypes.c_double),
                ("gamma", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("steps", ctypes.c_int),
                ("n_active", ctypes.c_int), ("stat", ctypes.c_double),
                ("primal", ctypes.c_double), ("dual", ctypes.c_double),
                ("comp", ctypes.c_double)]


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_frame.argtypes = [_D, _D, _D, _D]
        lib.orc_grasp_matrix.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double, _D]
        lib.orc_constraints.argtypes = [ctypes.c_int, _D, ctypes.c_double,
                                        ctypes.c_double, _D, _D]
        lib.orc_constraints.restype = ctypes.c_int
        lib.orc_qp_solve.argtypes = [ctypes.c_int, _D, _D, _D,
                                     ctypes.POINTER(Params), _D, _D, _D,
                                     ctypes.POINTER(Info)]
        lib.orc_qp_solve.restype = ctypes.c_int
        lib.orc_grasp_grad.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D,
                                       _D, _D, ctypes.POINTER(Params), _D, _D]
        lib.orc_solve_batch.argtypes = [ctypes.c_int, ctypes.c_int, _I, _I, _D,
                                        _D, _D, _D, ctypes.POINTER(Params),
                                        ctypes.c_int, _D, _D, _D, _I, _D]
        lib.orc_solve_batch.restype = ctypes.c_int
        lib.orc_grad_batch.argtypes = [ctypes.c_int, ctypes.c_int, _I, _I, _D,
                                       _D, _D, _D, _D, _D,
                                       ctypes.POINTER(Params), ctypes.c_int,
                                       _D, _D]
        lib.orc_grad_batch.restype = ctypes.c_int
        lib.orc_admm_rel_kkt.argtypes = [ctypes.c_int, _D, _D, _D,
                                         ctypes.POINTER(Params), _D, _D, _D, _D]
        lib.orc_inv_reduced_curvature.argtypes = [ctypes.c_int, _D, _D,
                                                  ctypes.POINTER(Params), _D]
        lib.orc_inv_reduced_curvature.restype = ctypes.c_double
        _lib = lib
        return lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I)


def params(kappa=20.0, beta=1.0, eps=1e-6, fmax=1.0, gamma=0.0) -> Params:
    return Params(float(kappa), float(beta), float(eps), float(fmax), float(gamma))


def frame(n):
    lib = _load()
    n, pn = _d(n)
    out = [np.zeros(3) for _ in range(3)]
    lib.orc_frame(pn, *[o.ctypes.data_as(_D) for o in out])
    return tuple(out)


def grasp_matrix(p, n, kappa=20.0):
    lib = _load()
    p, pp = _d(np.reshape(p, (-1, 3)))
    n, pn = _d(np.reshape(n, (-1, 3)))
    m = p.shape[0]
    G = np.zeros((6, 3 * m))
    lib.orc_grasp_matrix(m, pp, pn, float(kappa), G.ctypes.data_as(_D))
    return G


def constraints(mu, fmax=1.0, gamma=0.0):
    lib = _load()
    mu, pmu = _d(np.atleast_1d(mu))
    m = mu.shape[0]
    C = np.zeros((9 * m + 1, 3 * m))
    b = np.zeros(9 * m + 1)
    nc = lib.orc_constraints(m, pmu, float(fmax), float(gamma),
                             C.ctypes.data_as(_D), b.ctypes.data_as(_D))
    return C[:nc].copy(), b[:nc].copy()


def qp_solve(G, mu, t, prm: Params | None = None):
    """Solve one QP; returns (f, lam, Q, info-dict)."""
    lib = _load()
    prm = prm or params()
    G, pG = _d(G)
    mu, pmu = _d(np.atleast_1d(mu))
    t, pt = _d(t)
    m = mu.shape[0]
    f = np.zeros(3 * m)
    lam = np.zeros(9 * m + 1)
    Q = ctypes.c_double(0.0)
    info = Info()
    lib.orc_qp_solve(m, pG, pmu, pt, ctypes.byref(prm), f.ctypes.data_as(_D),
                     lam.ctypes.data_as(_D), ctypes.byref(Q), ctypes.byref(info))
    nc = 9 * m + (1 if prm.gamma > 0 else 0)
    d = {k: getattr(info, k) for k, _ in Info._fields_}
    return f, lam[:nc].copy(), Q.value, d


def solve_batch(counts, woff, p, n, mu, t, prm: Params | None = None,
                nthreads: int = 0, want_kkt: bool = False):
    """Batched oracle solve.  Shapes: counts [G], woff [G+1], p/n [G,M,3],
    mu [G,M], t [W,6] (any float dtype; converted exactly to FP64)."""
    lib = _load()
    prm = prm or params()
    counts, pc = _i(counts)
    woff, pw = _i(woff)
    p, pp = _d(p)
    n, pn = _d(n)
    mu, pmu = _d(mu)
    t, pt = _d(t)
    G_, M = p.shape[0], p.shape[1]
    W = int(woff[-1])
    forces = np.zeros((W, 3 * M))
    qobj = np.zeros(W)
    energy = np.zeros(G_)
    status = np.zeros(W, dtype=np.int32)
    kkt = np.zeros((W, 4)) if want_kkt else None
    rc = lib.orc_solve_batch(G_, M, pc, pw, pp, pn, pmu, pt, ctypes.byref(prm),
                             int(nthreads), forces.ctypes.data_as(_D),
                             qobj.ctypes.data_as(_D), energy.ctypes.data_as(_D),
                             status.ctypes.data_as(_I),
                             kkt.ctypes.data_as(_D) if want_kkt else None)
    if rc != 0:
        raise ValueError("oracle: invalid batch")
    out = {"forces": forces, "qobj": qobj, "energy": energy, "status": status}
    if want_kkt:
        out["kkt"] = kkt
    return out


def grad_batch(counts, woff, p, n, t, forces, wq=None, we=None,
               prm: Params | None = None, nthreads: int = 0):
    """dL/dp, dL/dn [G,M,3] for L = sum_w wq[w] Q_w + sum_g we[g] E_g."""
    lib = _load()
    prm = prm or params()
    counts, pc = _i(counts)
    woff, pw = _i(woff)
    p, pp = _d(p)
    n, pn = _d(n)
    t, pt = _d(t)
    forces, pf = _d(forces)
    G_, M = p.shape[0], p.shape[1]
    if wq is not None:
        wq, pwq = _d(wq)
    else:
        pwq = None
    if we is not None:
        we, pwe = _d(we)
    else:
        pwe = None
    dp = np.zeros((G_, M, 3))
    dn = np.zeros((G_, M, 3))
    rc = lib.orc_grad_batch(G_, M, pc, pw, pp, pn, pt, pf, pwq, pwe,
                            ctypes.byref(prm), int(nthreads),
                            dp.ctypes.data_as(_D), dn.ctypes.data_as(_D))
    if rc != 0:
        raise ValueError("oracle: invalid batch")
    return dp, dn


def grasp_grad(p, n, f, t, w, prm: Params | None = None):
    lib = _load()
    prm = prm or params()
    p, pp = _d(np.reshape(p, (-1, 3)))
    n, pn = _d(np.reshape(n, (-1, 3)))
    m = p.shape[0]
    f, pf = _d(np.reshape(f, (-1, 3 * m)))
    s = f.shape[0]
    t, pt = _d(np.reshape(t, (s, 6)))
    w, pwt = _d(np.broadcast_to(np.asarray(w, dtype=np.float64), (s,)))
    dp = np.zeros((m, 3))
    dn = np.zeros((m, 3))
    lib.orc_grasp_grad(m, s, pp, pn, pf, pt, pwt, ctypes.byref(prm),
                       dp.ctypes.data_as(_D), dn.ctypes.data_as(_D))
    return dp, dn


def admm_rel_kkt(G, mu, t, x, z, y, prm: Params | None = None):
    """(rel, primal part, dual part, bound/sign violation) of an ADMM state."""
    lib = _load()
    prm = prm or params()
    G, pG = _d(G)
    mu, pmu = _d(np.atleast_1d(mu))
    t, pt = _d(t)
    x, px = _d(x)
    z, pz = _d(z)
    y, py = _d(y)
    out = np.zeros(4)
    lib.orc_admm_rel_kkt(mu.shape[0], pG, pmu, pt, ctypes.byref(prm), px, pz,
                         py, out.ctypes.data_as(_D))
    return out


def inv_reduced_curvature(G, mu, lam, prm: Params | None = None) -> float:
    lib = _load()
    prm = prm or params()
    G, pG = _d(G)
    mu, pmu = _d(np.atleast_1d(mu))
    lam_full = np.zeros(9 * mu.shape[0] + 1)
    lam_full[:len(lam)] = lam
    lam_full, pl = _d(lam_full)
    return lib.orc_inv_reduced_curvature(mu.shape[0], pG, pmu, ctypes.byref(prm), pl)
