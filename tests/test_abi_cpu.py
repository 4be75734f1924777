"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad parameters before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2412_16490_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bodex_qp.h")).read()
    return sorted(set(re.findall(r"\b(bodex_qp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(api.LIB_PATH):
        pytest.skip("library not built")
    return api.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert set(names) == set(api.EXPORTED)
    for n in names:
        assert hasattr(L, n), n


def test_default_params_are_valid(L):
    p = api.default_params()
    assert p.m_max == 5 and p.max_iters == 500 and abs(p.eps_reg - 1e-6) < 1e-12
    assert p.flags & api.F_POLISH and p.flags & api.F_ADAPTIVE_RHO


@pytest.mark.parametrize("field,value", [("m_max", 0), ("m_max", 9), ("s_max", 0), ("s_max", 65),
                                         ("eps_reg", 0.0), ("alpha", 2.0), ("max_iters", 0),
                                         ("force_max", -1.0), ("rho_min", 0.0), ("tol_rel", 0.0)])
def test_create_rejects_bad_params(L, field, value):
    p = api.default_params()
    setattr(p, field, value)
    h = ctypes.c_void_p()
    rc = L.bodex_qp_create(ctypes.byref(p), 0, None, 0, ctypes.byref(h))
    assert rc == api.EINVAL
    assert not h.value
    assert L.bodex_qp_last_error(None)


def test_create_without_device_reports_enodev(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = api.default_params()
    h = ctypes.c_void_p()
    assert L.bodex_qp_create(ctypes.byref(p), 0, None, 0, ctypes.byref(h)) == api.ENODEV


def test_state_bytes(L):
    # x (15), z and y (46 each) and the residual (6) per QP, rho per grasp
    assert api.bodex_qp_state_bytes(10, 100, 5) == (100 * (15 + 2 * 46 + 6) + 10) * 4
    assert api.bodex_qp_state_bytes(-1, 1, 5) == 0


def test_destroy_null_is_noop(L):
    assert L.bodex_qp_destroy(None) == 0


def test_effective_params_follow_the_header_rules(L):
    # bodex_qp.h: with the polish on and admm_tol 0 the pyramid's warm-start
    # ADMM stops at 1e-1 and checks every max(check_every, 20) iterations;
    # the cone's stops at 1e-4 or min(max_iters, 200) iterations; without the
    # polish ADMM runs to tol_rel; the polish budget follows polish_chunk
    # (-1: 1 up to 40,960 QPs, else 16) for the pyramid with
    # gamma = 0, and is 0 otherwise
    p = api.default_params()
    assert p.check_every == 10 and p.admm_tol == 0.0 and p.friction_cone == api.CONE_PYRAMID8
    e = api.bodex_qp_effective_params(p, 131072)
    assert e["check_every"] == 20 and e["max_iters"] == 500 and abs(e["admm_tol"] - 0.1) < 1e-7
    assert e["polish_chunk"] == 16
    assert [api.bodex_qp_effective_params(p, n)["polish_chunk"] for n in (1, 40960, 40961, 98304, 98305)] == \
        [1, 1, 16, 16, 16]
    p.check_every = 30
    assert api.admm_check_period(p) == 30
    q = api.default_params(admm_tol=1e-3, polish_chunk=7)
    e = api.bodex_qp_effective_params(q, 1000)
    assert e["check_every"] == 10 and abs(e["admm_tol"] - 1e-3) < 1e-9 and e["polish_chunk"] == 7
    c = api.default_params(friction_cone=api.CONE_CIRCULAR)
    e = api.bodex_qp_effective_params(c, 1000)
    assert e["check_every"] == 10 and e["max_iters"] == 200 and abs(e["admm_tol"] - 1e-4) < 1e-9
    assert e["polish_chunk"] == 0
    n = api.default_params(flags_clear=api.F_POLISH)
    e = api.bodex_qp_effective_params(n, 1000)
    assert abs(e["admm_tol"] - n.tol_rel) < 1e-12 and e["check_every"] == 10 and e["polish_chunk"] == 0
    assert api.bodex_qp_effective_params(api.default_params(gamma=0.5), 1000)["polish_chunk"] == 0
    bad = api.default_params(m_max=0)
    with pytest.raises(api.BodexError):
        api.bodex_qp_effective_params(bad, 10)
