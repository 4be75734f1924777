"""Serving loop: continuous batching of grasp-synthesis requests on one GPU.

A request is a batch of grasps that runs `steps` upper-level steps; each step
is a warm-started forward solve plus the backward pass (the gradient an upper
level descends on), after which the request's contact points move (here: the
seeded random walk of the synthetic stream).  The server

* admits waiting requests in arrival order while the device bytes they hold
  (inputs, warm-start state, outputs) fit the HBM budget -- a request that does
  not fit waits for memory to free up, it never overcommits;
* every tick gathers the next step of *all* active requests into one batch and
  launches one solve and one backward for it, so requests that arrived while
  others were on the GPU share the device with them;
* keeps each request's ADMM state (x, z, y, rho) on the device between steps
  and warm-starts the next step from it;
* enqueues tick t+1 while tick t runs (stream order carries the dependency) and
  records each request's latency from arrival to the completion of its last
  step.

The solve of a grasp depends only on that grasp's inputs and state, so a
request's results are the same alone and in a mix (tested).
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque

import numpy as np
import torch

from . import api


@dataclasses.dataclass
class _Active:
    rid: int
    arrival: float
    steps: int
    done_steps: int
    counts: np.ndarray
    woff: np.ndarray
    points: torch.Tensor
    normals: torch.Tensor
    mu: torch.Tensor
    wrench: torch.Tensor
    state: dict
    walk: torch.Tensor | None
    nbytes: int
    energy: torch.Tensor | None = None
    qobj: torch.Tensor | None = None
    forces: torch.Tensor | None = None
    grad_p: torch.Tensor | None = None
    finish_event: torch.cuda.Event | None = None


def request_bytes(n_grasps: int, n_qps: int, m_max: int) -> int:
    """Device bytes a request holds while active (inputs, state, outputs,
    and its share of the gathered tick batch)."""
    inputs = n_grasps * m_max * 7 * 4 + n_qps * 6 * 4
    state = api.bodex_qp_state_bytes(n_grasps, n_qps, m_max)
    outputs = n_qps * (3 * m_max + 4) * 4 + n_grasps * 4 + 2 * n_grasps * m_max * 3 * 4
    return 2 * (inputs + state + outputs)


class Server:
    def __init__(self, m_max=5, s_max=32, budget_bytes=4 << 30, max_inflight_ticks=2,
                 params: api.Params | None = None, device=0):
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(device=self.device)
        p = params if params is not None else api.default_params(m_max=m_max, s_max=s_max)
        p.flags |= api.F_WARM_START
        self.m_max = p.m_max
        self.solver = api.Solver(p, device=device, stream=self.stream.cuda_stream)
        self.budget = int(budget_bytes)
        self.in_use = 0
        self.max_inflight = max_inflight_ticks
        self.waiting: deque = deque()
        self.active: list[_Active] = []
        self.inflight: deque = deque()       # (event, [requests finishing at this tick])
        self.latency: dict[int, float] = {}
        self.results: dict[int, dict] = {}
        self.qp_solves = 0
        self.ticks = 0
        self.peak_in_use = 0
        self.keep_results = False

    # -- admission -----------------------------------------------------------
    def submit(self, req, now: float | None = None, keep_walk=True):
        """Queue a workload.Request (arrival time taken from it)."""
        self.waiting.append((req, keep_walk))

    def _admit(self):
        while self.waiting:
            req, keep_walk = self.waiting[0]
            b = req.batch
            nb = request_bytes(b.n_grasps, b.n_qps, self.m_max)
            if nb > self.budget:
                raise ValueError("request %d needs %d bytes, budget is %d" % (req.rid, nb, self.budget))
            if self.in_use + nb > self.budget:
                return
            self.waiting.popleft()
            with torch.cuda.stream(self.stream):
                dev = self.device
                a = _Active(
                    rid=req.rid, arrival=req.arrival, steps=req.steps, done_steps=0,
                    counts=np.ascontiguousarray(b.counts, np.int32),
                    woff=np.ascontiguousarray(b.woff, np.int32),
                    points=torch.as_tensor(b.points, device=dev),
                    normals=torch.as_tensor(b.normals, device=dev),
                    mu=torch.as_tensor(b.mu, device=dev),
                    wrench=torch.as_tensor(b.wrench, device=dev),
                    state=api.new_state(b.n_grasps, b.n_qps, self.m_max, device=dev),
                    walk=torch.as_tensor(req.walk, device=dev) if keep_walk and req.walk is not None else None,
                    nbytes=nb)
            self.in_use += nb
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.active.append(a)

    # -- one tick ------------------------------------------------------------
    def _tick(self):
        acts = self.active
        if not acts:
            return
        with torch.cuda.stream(self.stream):
            counts = np.concatenate([a.counts for a in acts])
            woffs = [0]
            for a in acts:
                woffs.extend((a.woff[1:] + woffs[-1]).tolist())
            woff = np.asarray(woffs, np.int32)
            pts = torch.cat([a.points for a in acts])
            nrm = torch.cat([a.normals for a in acts])
            mu = torch.cat([a.mu for a in acts])
            wr = torch.cat([a.wrench for a in acts])
            st = {k: torch.cat([a.state[k] for a in acts], dim=(0 if k == "rho" else 1)).contiguous()
                  for k in ("x", "z", "y", "rho")}
            tb = _Batch(pts, nrm, mu, wr, counts, woff)
            res = api.new_result(tb.n_grasps, tb.n_qps, self.m_max, device=self.device)
            self.solver.solve(tb, state=st, result=res)
            gp = torch.zeros_like(pts)
            gn = torch.zeros_like(nrm)
            ones = torch.ones(tb.n_grasps, device=self.device)
            self.solver.backward(tb, st, dL_dE=ones, out=(gp, gn))
            # scatter state and advance every request by one step
            g0 = 0
            w0 = 0
            finishing = []
            for a in acts:
                G, W = a.counts.shape[0], int(a.woff[-1])
                for k in ("x", "z", "y"):
                    a.state[k].copy_(st[k][:, w0:w0 + W])
                a.state["rho"].copy_(st["rho"][g0:g0 + G])
                if a.walk is not None and a.done_steps < a.walk.shape[0]:
                    a.points.add_(a.walk[a.done_steps])
                a.done_steps += 1
                if a.done_steps == a.steps:
                    if self.keep_results:
                        a.energy = res["energy"][g0:g0 + G].clone()
                        a.qobj = res["qp_obj"][w0:w0 + W].clone()
                        a.forces = res["forces"][w0:w0 + W].clone()
                        a.grad_p = gp[g0:g0 + G].clone()
                    finishing.append(a)
                g0 += G
                w0 += W
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self.qp_solves += tb.n_qps
        self.ticks += 1
        self.inflight.append((ev, finishing))
        for a in finishing:
            self.active.remove(a)

    def _reap(self, block=False):
        while self.inflight:
            ev, finishing = self.inflight[0]
            if not block and not ev.query():
                return
            ev.synchronize()
            t = time.perf_counter() - self._t0
            self.inflight.popleft()
            for a in finishing:
                self.latency[a.rid] = t - a.arrival
                self.in_use -= a.nbytes
                if self.keep_results:
                    self.results[a.rid] = {"energy": a.energy.cpu().numpy(), "qp_obj": a.qobj.cpu().numpy(),
                                           "forces": a.forces.cpu().numpy(),
                                           "grad_points": a.grad_p.cpu().numpy()}

    # -- main loop -----------------------------------------------------------
    def run(self, requests, realtime=True):
        """Serve an iterable of requests sorted by arrival.  With realtime the
        arrivals follow the wall clock from the start of the run."""
        reqs = deque(requests)
        self._t0 = time.perf_counter()
        while reqs or self.waiting or self.active or self.inflight:
            now = time.perf_counter() - self._t0
            while reqs and (not realtime or reqs[0].arrival <= now):
                self.submit(reqs.popleft())
            self._reap(block=False)
            self._admit()
            if self.active and len(self.inflight) < self.max_inflight:
                self._tick()
            elif self.inflight:
                self._reap(block=True)
            elif reqs and realtime:
                time.sleep(max(0.0, min(0.001, reqs[0].arrival - now)))
        wall = time.perf_counter() - self._t0
        lat = np.array([self.latency[k] for k in sorted(self.latency)])
        return {"requests": len(lat), "wall_s": wall, "qp_solves": self.qp_solves, "ticks": self.ticks,
                "qps_per_s": self.qp_solves / wall,
                "latency_p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
                "latency_p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
                "peak_device_bytes": self.peak_in_use}

    def close(self):
        self.solver.close()


class _Batch(api.DeviceBatch):
    def __init__(self, points, normals, mu, wrench, counts, woff):  # noqa: D401
        self.counts = counts
        self.woff = woff
        self.points = points
        self.normals = normals
        self.mu = mu
        self.wrench = wrench
        self.n_grasps = int(counts.shape[0])
        self.n_qps = int(woff[-1])
        self.m_max = int(points.shape[1])


def serve_fifo_plain(requests, m_max=5, s_max=32, realtime=True):
    """Baseline: one request-step per plain launch, requests in arrival order,
    no mixing (a queue only)."""
    stream = torch.cuda.Stream()
    p = api.default_params(m_max=m_max, s_max=s_max)
    p.flags |= api.F_WARM_START
    solver = api.Solver(p, stream=stream.cuda_stream)
    reqs = deque(requests)
    t0 = time.perf_counter()
    lat = []
    solves = 0
    while reqs:
        r = reqs.popleft()
        now = time.perf_counter() - t0
        if realtime and r.arrival > now:
            time.sleep(r.arrival - now)
        b = r.batch
        with torch.cuda.stream(stream):
            db = api.DeviceBatch(b)
            st = api.new_state(db.n_grasps, db.n_qps, m_max)
            walk = torch.as_tensor(r.walk, device="cuda") if r.walk is not None else None
            ones = torch.ones(db.n_grasps, device="cuda")
            gp = torch.zeros_like(db.points)
            gn = torch.zeros_like(db.normals)
            for k in range(r.steps):
                res = solver.solve(db, state=st)
                solver.backward(db, st, dL_dE=ones, out=(gp, gn))
                if walk is not None:
                    db.points.add_(walk[k])
                solves += db.n_qps
        stream.synchronize()
        lat.append(time.perf_counter() - t0 - r.arrival)
    wall = time.perf_counter() - t0
    solver.close()
    lat = np.asarray(lat)
    return {"requests": len(lat), "wall_s": wall, "qp_solves": solves, "qps_per_s": solves / wall,
            "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99))}
