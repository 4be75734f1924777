"""QPs of the 60-s served stream (Poisson 200 requests/s, 50 warm-started
forward+backward steps on a random walk) whose polish once failed, replayed
alone through the C ABI as the server runs them: each must now end converged
and polished at the oracle's minimiser.  The requests are rebuilt from the
seeded stream; the (request, step, QP) triples name where the polish had
failed:

* request 3238, step 0 (a cold solve): the warm set's first step found the
  violated row dependent on the active rows with no multiplier to drop, and
  no one-row change had been used, so nothing was retried (now: the restart
  from the empty active set);
* request 5716, step 38: the exact re-solve after the last step moved the
  point across an inactive row by 1.4e-5 and the acceptance check rejected it
  (now: more steps);
* request 479, step 40: as the first, after warm-started steps."""
import numpy as np
import pytest

import oracle
from gpu_common import oracle_params
from paper_2412_16490_amd import api
from paper_2412_16490_amd import serve as sv
from paper_2412_16490_amd import workload as wl

pytestmark = pytest.mark.gpu

CASES = [(3238, 0, 6318), (5716, 38, 42066), (479, 40, 28954)]


@pytest.mark.parametrize("rid,step,qp", CASES)
def test_served_qp_converges_at_the_oracle_minimiser(rid, step, qp):
    import torch
    req = next(wl.request_stream(rate=200.0, duration=60.0, start=rid))
    assert req.rid == rid
    b = req.batch
    print("served request %d (%d grasps, %d QPs), step %d, QP %d" % (rid, b.n_grasps, b.n_qps, step, qp), flush=True)
    p = api.default_params(m_max=5, s_max=32)
    p.flags |= api.F_WARM_START
    s = api.Solver(p)
    pts = torch.as_tensor(b.points, device="cuda").clone()
    nrm = torch.as_tensor(b.normals, device="cuda")
    mu = torch.as_tensor(b.mu, device="cuda")
    wr = torch.as_tensor(b.wrench, device="cuda")
    counts = np.ascontiguousarray(b.counts, np.int32)
    woff = np.ascontiguousarray(b.woff, np.int32)
    st = api.new_state(b.n_grasps, b.n_qps, 5)
    walk = torch.as_tensor(req.walk, device="cuda")
    ones = torch.ones(b.n_grasps, device="cuda")
    for k in range(step + 1):
        tb = sv._Batch(pts, nrm, mu, wr, counts, woff)
        res = api.new_result(b.n_grasps, b.n_qps, 5)
        s.solve(tb, state=st, result=res)
        if k == step:
            torch.cuda.synchronize()
            status = int(res["status"][qp])
            forces = res["forces"][qp].cpu().numpy().astype(np.float64)
            qobj = float(res["qp_obj"][qp])
            g = int(np.searchsorted(woff, qp, side="right") - 1)
            points = pts[g].cpu().numpy().astype(np.float64)
            break
        s.backward(tb, st, dL_dE=ones)
        pts += walk[k]
    s.close()
    assert status & api.ST_CONVERGED and status & api.ST_POLISHED, "status 0x%02x" % status
    m = int(counts[g])
    G = oracle.grasp_matrix(points[:m], b.normals[g, :m].astype(np.float64), 20.0)
    t = b.wrench[qp].astype(np.float64)
    fs, lam, Qs, info = oracle.qp_solve(G, b.mu[g, :m].astype(np.float64), t, oracle_params())
    assert info["status"] == 0
    qerr = abs(qobj - Qs) / max(Qs, 1e-2 * (t @ t))
    ferr = np.abs(forces[:3 * m] - fs).max()
    print("objective error %.2e, force error %.2e" % (qerr, ferr), flush=True)
    assert qerr <= 1e-5 and ferr <= 1e-4
