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
* keeps each request's ADMM state (x, z, y, rho, and the wrench residual the
  backward reads) on the device between steps, in a pool of columns the
  request holds from admission to completion, and warm-starts the next step
  from it: the tick passes the pool with per-grasp column offsets to the
  solve and the backward, which read and write the state in place;
* enqueues tick t+1 while tick t runs (stream order carries the dependency) and
  records each request's latency from arrival to the completion of its last
  step.

Throughput counts only QP solves that end converged (relative KKT residual
<= tol_rel).  The run also reports the offered load, the queue over time and
the device time of each tick spent around its solve and backward (gathering
the requests' inputs, moving their contact points).

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


class _Ranges:
    """First-fit allocator of contiguous index ranges in [0, n)."""

    def __init__(self, n: int):
        self.free = [(0, n)]

    def take(self, k: int):
        for i, (a, ln) in enumerate(self.free):
            if ln >= k:
                if ln == k:
                    self.free.pop(i)
                else:
                    self.free[i] = (a + k, ln - k)
                return a
        return None

    def give(self, a: int, k: int):
        self.free.append((a, k))
        self.free.sort()
        merged = []
        for b, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == b:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((b, ln))
        self.free = merged


class _StatePool:
    """The state of every active request in one set of device arrays: x [3 m][cap],
    z, y [9 m + 1][cap], r [6][cap] (columns = QPs) and rho [cap_g]."""

    def __init__(self, cap_q: int, cap_g: int, m_max: int, device):
        nr = 9 * m_max + 1
        f = dict(dtype=torch.float32, device=device)
        self.x = torch.zeros((3 * m_max, cap_q), **f)
        self.z = torch.zeros((nr, cap_q), **f)
        self.y = torch.zeros((nr, cap_q), **f)
        self.r = torch.zeros((6, cap_q), **f)
        self.rho = torch.zeros((cap_g,), **f)
        self.cols = _Ranges(cap_q)
        self.slots = _Ranges(cap_g)

    @staticmethod
    def bytes_per(m_max: int):
        """(bytes per QP column, bytes per grasp slot)."""
        return (3 * m_max + 2 * (9 * m_max + 1) + 6) * 4, 4

    def take(self, nq: int, ng: int):
        q0 = self.cols.take(nq)
        if q0 is None:
            return None
        g0 = self.slots.take(ng)
        if g0 is None:
            self.cols.give(q0, nq)
            return None
        for t in (self.x, self.z, self.y, self.r):
            t[:, q0:q0 + nq].zero_()
        self.rho[g0:g0 + ng].zero_()  # rho 0: the first step starts from rho0
        return q0, g0

    def give(self, q0: int, nq: int, g0: int, ng: int):
        self.cols.give(q0, nq)
        self.slots.give(g0, ng)


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
    q0: int        # first state column in the pool
    g0: int        # first rho slot in the pool
    walk: torch.Tensor | None
    nbytes: int
    energy: torch.Tensor | None = None
    qobj: torch.Tensor | None = None
    forces: torch.Tensor | None = None
    grad_p: torch.Tensor | None = None
    finish_event: torch.cuda.Event | None = None


def request_bytes(n_grasps: int, n_qps: int, m_max: int) -> int:
    """Device bytes a request holds while active outside the state pool
    (inputs and its share of the gathered tick batch: inputs, outputs,
    gradients); its state columns come from the pool."""
    inputs = n_grasps * m_max * 7 * 4 + n_qps * 6 * 4
    outputs = n_qps * (3 * m_max + 4) * 4 + n_grasps * 4 + 2 * n_grasps * m_max * 3 * 4
    return 2 * inputs + outputs


# share of the HBM budget given to the state pool (a QP's state columns take
# about three times the bytes of its inputs, outputs and tick buffers)
POOL_SHARE = 0.75


class Server:
    def __init__(self, m_max=5, s_max=32, budget_bytes=4 << 30, max_inflight_ticks=2,
                 params: api.Params | None = None, device=0):
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(device=self.device)
        p = params if params is not None else api.default_params(m_max=m_max, s_max=s_max)
        p.flags |= api.F_WARM_START
        self.m_max = p.m_max
        self.solver = api.Solver(p, device=device, stream=self.stream.cuda_stream)
        bq, bg = _StatePool.bytes_per(self.m_max)
        pool_bytes = int(POOL_SHARE * budget_bytes)
        cap_q = max(64, pool_bytes // (bq + bg // 4))
        self.pool = _StatePool(cap_q, max(16, cap_q // 4), self.m_max, self.device)
        self.budget = int(budget_bytes) - pool_bytes
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
        self._conv = []         # per tick: converged QPs (device scalars)
        self._copy_ev = []      # per tick: events before/after the gather, after the backward, at the end
        self.queue_trace = []   # (time, waiting, active, bytes in use) per tick
        self.progress_every = 0.0
        self._ones = torch.ones(1, device=self.device)

    # -- admission -----------------------------------------------------------
    def submit(self, req, now: float | None = None, keep_walk=True):
        """Queue a workload.Request (arrival time taken from it)."""
        self.waiting.append((req, keep_walk))

    def _admit(self):
        while self.waiting:
            req, keep_walk = self.waiting[0]
            b = req.batch
            nb = request_bytes(b.n_grasps, b.n_qps, self.m_max)
            if nb > self.budget or b.n_qps > self.pool.x.shape[1] or b.n_grasps > self.pool.rho.shape[0]:
                raise ValueError("request %d needs %d bytes and %d state columns; budget %d bytes, pool %d columns"
                                 % (req.rid, nb, b.n_qps, self.budget, self.pool.x.shape[1]))
            if self.in_use + nb > self.budget:
                return
            with torch.cuda.stream(self.stream):
                got = self.pool.take(b.n_qps, b.n_grasps)
            if got is None:
                return  # waits for state columns to free up
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
                    q0=got[0], g0=got[1],
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
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            evs[0].record(self.stream)
            counts = np.concatenate([a.counts for a in acts])
            woffs = [0]
            for a in acts:
                woffs.extend((a.woff[1:] + woffs[-1]).tolist())
            woff = np.asarray(woffs, np.int32)
            pts = torch.cat([a.points for a in acts])
            nrm = torch.cat([a.normals for a in acts])
            mu = torch.cat([a.mu for a in acts])
            wr = torch.cat([a.wrench for a in acts])
            # the pool with each grasp's state columns (its requests' ranges)
            qoff = np.concatenate([a.q0 + a.woff[:-1] for a in acts]).astype(np.int32)
            goff = np.concatenate([a.g0 + np.arange(a.counts.shape[0]) for a in acts]).astype(np.int32)
            P = self.pool
            st = {"x": P.x, "z": P.z, "y": P.y, "rho": P.rho, "r": P.r, "qp_offset": qoff, "grasp_offset": goff}
            tb = _Batch(pts, nrm, mu, wr, counts, woff)
            res = api.new_result(tb.n_grasps, tb.n_qps, self.m_max, device=self.device)
            evs[1].record(self.stream)
            self.solver.solve(tb, state=st, result=res)
            # the backward overwrites every entry of its outputs
            gp = torch.empty_like(pts)
            gn = torch.empty_like(nrm)
            if self._ones.shape[0] < tb.n_grasps:
                self._ones = torch.ones(2 * tb.n_grasps, device=self.device)
            self.solver.backward(tb, st, dL_dE=self._ones[:tb.n_grasps], out=(gp, gn))
            self._conv.append(((res["status"] & api.ST_CONVERGED) != 0).sum())
            evs[2].record(self.stream)
            # advance every request by one step: the random walk of its
            # contact points (one multi-tensor add for all of them)
            walkers = [a for a in acts if a.walk is not None and a.done_steps < a.walk.shape[0]]
            if walkers:
                torch._foreach_add_([a.points for a in walkers], [a.walk[a.done_steps] for a in walkers])
            g0 = 0
            w0 = 0
            finishing = []
            for a in acts:
                G, W = a.counts.shape[0], int(a.woff[-1])
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
            evs[3].record(self.stream)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self._copy_ev.append(evs)
        self.qp_solves += tb.n_qps
        self.ticks += 1
        self.queue_trace.append((time.perf_counter() - self._t0, len(self.waiting), len(self.active), self.in_use))
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
                self.pool.give(a.q0, int(a.woff[-1]), a.g0, int(a.counts.shape[0]))
                if self.keep_results:
                    self.results[a.rid] = {"energy": a.energy.cpu().numpy(), "qp_obj": a.qobj.cpu().numpy(),
                                           "forces": a.forces.cpu().numpy(),
                                           "grad_points": a.grad_p.cpu().numpy()}

    # -- main loop -----------------------------------------------------------
    def run(self, requests, realtime=True):
        """Serve an iterable of requests sorted by arrival.  With realtime the
        arrivals follow the wall clock from the start of the run."""
        reqs = deque(requests)
        offered = sum(r.batch.n_qps * r.steps for r in reqs)
        span = reqs[-1].arrival if reqs else 0.0
        self._t0 = time.perf_counter()
        next_note = self.progress_every
        while reqs or self.waiting or self.active or self.inflight:
            now = time.perf_counter() - self._t0
            if self.progress_every and now >= next_note:
                print("serve: t=%.0f s, %d finished, %d waiting, %d active, %d ticks" % (
                    now, len(self.latency), len(self.waiting), len(self.active), self.ticks), flush=True)
                next_note += self.progress_every
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
        torch.cuda.synchronize(self.device)
        conv = int(sum(int(c.item()) for c in self._conv))
        copy_ms = sum(e[0].elapsed_time(e[1]) + e[2].elapsed_time(e[3]) for e in self._copy_ev)
        tick_ms = sum(e[0].elapsed_time(e[3]) for e in self._copy_ev)
        lat = np.array([self.latency[k] for k in sorted(self.latency)])
        qt = np.array(self.queue_trace) if self.queue_trace else np.zeros((0, 4))
        return {"requests": len(lat), "wall_s": wall, "arrival_span_s": span, "qp_solves": self.qp_solves,
                "qp_solves_converged": conv, "ticks": self.ticks,
                "qps_per_s": conv / wall, "offered_qp_solves_per_s": offered / max(span, 1e-9),
                "keeps_up": bool(conv / wall >= 0.95 * offered / max(span, 1e-9)),
                "latency_p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
                "latency_p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
                "around_solve_ms": copy_ms, "tick_device_ms": tick_ms,
                "around_solve_fraction": copy_ms / max(tick_ms, 1e-9),
                "queue_waiting_max": int(qt[:, 1].max()) if len(qt) else 0,
                "queue_waiting_at": _queue_samples(qt),
                "peak_device_bytes": self.peak_in_use}

    def close(self):
        self.solver.close()


def _queue_samples(qt, n=8):
    """Waiting requests at n evenly spaced times of the run."""
    if len(qt) == 0:
        return []
    times = np.linspace(qt[0, 0], qt[-1, 0], n)
    idx = np.searchsorted(qt[:, 0], times, side="right") - 1
    return [[round(float(t), 2), int(qt[max(i, 0), 1])] for t, i in zip(times, idx)]


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
    conv = []
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
                conv.append(((res["status"] & api.ST_CONVERGED) != 0).sum())
                if walk is not None:
                    db.points.add_(walk[k])
                solves += db.n_qps
        stream.synchronize()
        lat.append(time.perf_counter() - t0 - r.arrival)
    wall = time.perf_counter() - t0
    solver.close()
    lat = np.asarray(lat)
    nconv = int(sum(int(c.item()) for c in conv))
    return {"requests": len(lat), "wall_s": wall, "qp_solves": solves, "qp_solves_converged": nconv,
            "qps_per_s": nconv / wall,
            "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99))}
