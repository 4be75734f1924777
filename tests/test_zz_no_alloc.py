"""The allocation-free solve (bodex_qp_solve_static) against bodex_qp_solve,
through the C ABI: two calls in a row on one handle, the second with a
smaller batch, each compared element by element with the allocating entry
point on the same inputs.  The static solve runs the one-lane polish to the
end (the contact-parallel polish needs workspace), so against bodex_qp_solve
with polish_chunk = 0 (same kernels and tiles) the results are identical,
and against the default chunked polish they agree to the parity bar (both
reach the minimiser); also a cone handle, the size limit and the rejected
flags."""
import numpy as np
import pytest

from paper_2412_16490_amd import api
from paper_2412_16490_amd import workload as wl

pytestmark = pytest.mark.gpu

KEYS = ("forces", "qp_obj", "energy", "kkt_rel", "iters", "status")


def _both(s, b, cone=False):
    import torch
    db = api.DeviceBatch(b)
    st_a = api.new_state(db.n_grasps, db.n_qps, db.m_max, cone=cone)
    st_b = api.new_state(db.n_grasps, db.n_qps, db.m_max, cone=cone)
    r_a = api.new_result(db.n_grasps, db.n_qps, db.m_max)
    r_b = api.new_result(db.n_grasps, db.n_qps, db.m_max)
    api.bodex_qp_solve(s.h, db, r_a, st_a)
    api.bodex_qp_solve_static(s.h, db, r_b, st_b)
    torch.cuda.synchronize()
    return ({k: v.cpu().numpy() for k, v in r_a.items()}, {k: v.cpu().numpy() for k, v in r_b.items()},
            {k: v.cpu().numpy() for k, v in st_a.items()}, {k: v.cpu().numpy() for k, v in st_b.items()})


def _same(a, b, sa, sb):
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    for k in ("x", "z", "y", "rho", "r"):
        np.testing.assert_array_equal(sa[k], sb[k], err_msg="state " + k)


def _close(a, b, batch):
    # the parity bar: objective 1e-5 relative (floor 1e-2 |t|^2), forces 1e-4
    # fmax, energy 1e-5 relative (floor 1e-2 s)
    tn = np.sum(batch.wrench.astype(np.float64) ** 2, axis=1)
    q = np.abs(a["qp_obj"] - b["qp_obj"]) / np.maximum(np.abs(a["qp_obj"]), 1e-2 * tn)
    assert q.max() <= 1e-5
    assert np.abs(a["forces"] - b["forces"]).max() <= 1e-4
    s = np.diff(batch.woff)
    e = np.abs(a["energy"] - b["energy"]) / np.maximum(np.abs(a["energy"]), 1e-2 * s)
    assert e.max() <= 1e-5
    np.testing.assert_array_equal(a["status"] & api.ST_CONVERGED, b["status"] & api.ST_CONVERGED)


def test_static_solve_matches_the_allocating_solve_twice():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s0 = api.Solver(api.default_params(m_max=5, s_max=32, polish_chunk=0))
    s = api.Solver(api.default_params(m_max=5, s_max=32))
    print("static solve: 2000 grasps uneven, then 150 grasps", flush=True)
    big = wl.config(3, 2000)
    small = wl.config(1, 150)
    for b in (big, small):
        a, c, sa, sc = _both(s0, b)
        _same(a, c, sa, sc)
        assert np.all(c["status"] & api.ST_CONVERGED)
        a2, c2, _, _ = _both(s, b)
        _close(a2, c2, b)
    s0.close()
    s.close()


def test_static_solve_circular_cone():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = api.default_params(m_max=5, s_max=16, polish_chunk=0)
    p.friction_cone = api.CONE_CIRCULAR
    s = api.Solver(p)
    print("static solve: circular cone, 64 grasps", flush=True)
    a, c, sa, sc = _both(s, wl.config(1, 64), cone=True)
    _same(a, c, sa, sc)
    s.close()


def test_static_solve_limits_and_flags():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    b = wl.config(1, 8)
    db = api.DeviceBatch(b)
    r = api.new_result(db.n_grasps, db.n_qps, 5)
    st = api.new_state(db.n_grasps, db.n_qps, 5)
    for flag in (api.F_BATCHED, api.F_GRAPH):
        s = api.Solver(api.default_params(m_max=5, s_max=16, flags_set=flag))
        with pytest.raises(api.BodexError) as e:
            api.bodex_qp_solve_static(s.h, db, r, st)
        assert e.value.code == api.EUNSUP
        s.close()
    s = api.Solver(api.default_params(m_max=5, s_max=16))
    with pytest.raises(api.BodexError) as e:
        api.bodex_qp_solve_static(s.h, db, r, None)  # no state: the static path has no workspace for it
    assert e.value.code == api.EINVAL
    # beyond the scratch: 3 G + tiles + 6 > 2^20 ints (checked before any device work)
    G = 360000
    huge = wl.Batch(np.zeros((G, 5, 3), np.float32), np.tile(np.float32([0, 0, 1]), (G, 5, 1)),
                    np.full((G, 5), 0.5, np.float32), np.tile(np.float32([1, 0, 0, 0, 0, 0]), (G, 1)),
                    np.full(G, 5, np.int32), np.arange(G + 1, dtype=np.int32), "huge")
    dh = api.DeviceBatch(huge)
    rh = api.new_result(G, G, 5)
    sh = api.new_state(G, G, 5)
    with pytest.raises(api.BodexError) as e:
        api.bodex_qp_solve_static(s.h, dh, rh, sh)
    assert e.value.code == api.EUNSUP and "scratch" in str(e.value)
    s.close()
