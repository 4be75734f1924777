"""torch.autograd.Function over the HIP solve/backward.

``BodexQPEnergy.apply(points, normals, mu, wrench_dir, offsets, counts, params)``
returns ``(energy[G], qp_obj[W], forces[W, 3 m_max])``.  Its backward runs the
hand-written backward kernel, which recomputes the optimal forces from the
solve's final state (no ADMM iterates are stored) and applies Danskin's
theorem (Sec. IV-A: Q_j is differentiable through G_i); gradients flow to
points and normals only (friction and desired wrenches are data).
"""
from __future__ import annotations

import numpy as np
import torch

from . import api

_solvers: dict = {}


def _solver(params: api.Params, device: int, stream) -> api.Solver:
    key = (bytes(params), device, stream)
    s = _solvers.get(key)
    if s is None:
        p = api.Params.from_buffer_copy(bytes(params))
        s = api.Solver(p, device=device, stream=stream)
        _solvers[key] = s
    return s


class _TensorBatch(api.DeviceBatch):
    """A DeviceBatch view over caller tensors (no copies)."""

    def __init__(self, points, normals, mu, wrench, counts, woff):  # noqa: D401
        self.counts = np.ascontiguousarray(counts, dtype=np.int32)
        self.woff = np.ascontiguousarray(woff, dtype=np.int32)
        self.points = points.contiguous()
        self.normals = normals.contiguous()
        self.mu = mu.contiguous()
        self.wrench = wrench.contiguous()
        self.n_grasps = int(self.counts.shape[0])
        self.n_qps = int(self.woff[-1])
        self.m_max = int(points.shape[1])


class BodexQPEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, points, normals, mu, wrench_dir, offsets, counts, params=None):
        counts = np.asarray(counts.cpu() if torch.is_tensor(counts) else counts, dtype=np.int32)
        offsets = np.asarray(offsets.cpu() if torch.is_tensor(offsets) else offsets, dtype=np.int32)
        m_max = int(points.shape[1])
        if params is None:
            s_max = int(np.max(np.diff(offsets))) if len(offsets) > 1 else 1
            params = api.default_params(m_max=m_max, s_max=max(1, s_max))
        dev = points.device.index or 0
        stream = torch.cuda.current_stream(points.device).cuda_stream
        solver = _solver(params, dev, stream)
        tb = _TensorBatch(points.detach().float(), normals.detach().float(), mu.detach().float(),
                          wrench_dir.detach().float(), counts, offsets)
        state = api.new_state(tb.n_grasps, tb.n_qps, m_max, device=points.device)
        res = solver.solve(tb, state=state)
        ctx.solver = solver
        ctx.tb = tb
        ctx.state = state
        ctx.mark_non_differentiable(res["forces"])
        return res["energy"], res["qp_obj"], res["forces"]

    @staticmethod
    def backward(ctx, dE, dQ, dF):
        tb = ctx.tb
        dE = dE.contiguous().float() if dE is not None else None
        dQ = dQ.contiguous().float() if dQ is not None else None
        gp = torch.zeros_like(tb.points)
        gn = torch.zeros_like(tb.normals)
        ctx.solver.backward(tb, ctx.state, dL_dE=dE, dL_dQ=dQ, out=(gp, gn))
        return gp, gn, None, None, None, None, None


def grasp_energy(points, normals, mu, wrench_dir, offsets, counts, params=None):
    """Energy per grasp (differentiable in points and normals)."""
    return BodexQPEnergy.apply(points, normals, mu, wrench_dir, offsets, counts, params)[0]
