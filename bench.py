"""Benchmark: contact-force QPs/s at relative KKT residual <= 1e-5.

Workload (one step): the plain solve of 8192 grasps x 5 contacts x 16 desired
wrenches = 131,072 QPs (ellipsoid contacts, mu ~ U[0.3, 0.8], seed 16491), inputs
resident in HBM.  A step is one call of the library's solve: grasp matrices,
per-grasp factorisation, fused ADMM with residual checks and rho adaptation,
FP64 polish, objectives, energies and state.

Prints one JSON line.  Besides the contract fields it carries:
  roofline      the kernel with the larger share of the step (ADMM: FP32 vector
                ALU peak; finalize/polish: FP64 vector ALU peak), with the
                other kernel in roofline_other_kernel
  cpu_baseline  the FP64 oracle on the host cores over the same QPs
  forms         the uneven batch (50,000 grasps) in one persistent graph launch
                vs per-(m, s) plain launches, and forward+backward on the
                differentiation workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 VALU lane-ops/s;
# an FMA counts 2 flops -> 78.6 TFLOP/s for FP32 without packed FMA (which this
# build does not use; the 157.3 TFLOP/s vendor figure assumes packed FMA) and
# 78.6 TFLOP/s for FP64 (full-rate FMA).
PEAK_FP32_TFLOPS = 78.6
PEAK_FP64_TFLOPS = 78.6
PROFILES = os.path.join(ROOT, "profiles")


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic_<kernel>.txt: 'source_hash', 'bytes_per_launch'), or
    None when it is missing or was taken on other sources."""
    path = os.path.join(PROFILES, "traffic_%s.txt" % kernel)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    from paper_2412_16490_amd.profile_summary import kernel_source_hash
    if vals.get("source_hash") != kernel_source_hash(kernel):
        return None
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def admm_flops(m: int, iters: np.ndarray, check_every: int) -> float:
    """Algorithmic flops of the ADMM kernel, counted from the arithmetic each
    lane performs (FMA = 2 flops, every other add/mul/min/max/select = 1):
      per iteration   18 m^2 + 92 m + 7   (917 at m = 5)
        right-hand side 28m + 2 ops (7m + 1 FMA), K^{-1} product n^2 ops
        (n(n-1) FMA, n = 3m), row update 47m + 3 ops (13m + 1 FMA)
      per residual check  246 m + 19      (1249 at m = 5)
    Factorisations (about n^3/3 per grasp and rho change) are left out."""
    it = iters.astype(np.float64)
    checks = np.floor(it / check_every)
    per_iter = 18 * m * m + 92 * m + 7
    per_check = 246 * m + 19
    return float(np.sum(it * per_iter + checks * per_check))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the extra forms")
    ap.add_argument("--serve-seconds", type=float, default=2.0,
                    help="length of the Poisson arrival window of the served form")
    ap.add_argument("--fifo-seconds", type=float, default=1.0,
                    help="window of the stream that both the served form and the FIFO baseline run")
    ap.add_argument("--served-only", action="store_true",
                    help="only run the served form and its FIFO baseline and print their JSON")
    ap.add_argument("--admm-waves", type=int, default=0, help="ADMM register budget (0 = default)")
    ap.add_argument("--cone-only", action="store_true",
                    help="only run the circular-cone form and print its JSON")
    ap.add_argument("--detach-only", action="store_true",
                    help="only run the fine-stage surrogate (Detach) form at 2^20 grasps and print its JSON")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only run the batch-size sweep of the headline shape")
    ap.add_argument("--descent-only", action="store_true",
                    help="only run the coarse-stage descent form (floating hands on ellipsoids)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run device copies of MIB MiB (to scale HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: measures one GPU only (got --gpus %d, WORLD_SIZE %d); the path shards by "
              "contiguous grasp ranges with no exchange between GPUs" % (args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4,
                          "launches": 3}), flush=True)
        return

    from paper_2412_16490_amd import api, build as hip_build
    from paper_2412_16490_amd import workload as wl

    if not os.path.exists(hip_build.LIB):
        hip_build.build()
    assert torch.cuda.is_available(), "no GPU"
    if args.cone_only:
        print(json.dumps({"circular_cone": cone_form(torch, api, wl)}), flush=True)
        return
    if args.detach_only:
        print(json.dumps({"detach_surrogate": detach_form(torch, api, wl, large_only=True)}), flush=True)
        return
    if args.sweep_only:
        print(json.dumps({"size_sweep": size_sweep(torch, api, wl)}), flush=True)
        return
    if args.descent_only:
        print(json.dumps({"coarse_descent": descent_form(torch, api, wl)}), flush=True)
        return
    if args.served_only:
        print(json.dumps(served(torch, wl, args.serve_seconds, args.fifo_seconds)), flush=True)
        return

    batch = wl.config(1)
    db = api.DeviceBatch(batch)
    p = api.default_params(m_max=5, s_max=16)
    p.flags |= api.F_TIMING
    p.admm_waves = args.admm_waves
    stream = torch.cuda.current_stream()
    solver = api.Solver(p, stream=stream.cuda_stream)
    st = api.new_state(db.n_grasps, db.n_qps, db.m_max)
    res = api.new_result(db.n_grasps, db.n_qps, db.m_max, polish_flops=True)

    for _ in range(args.warmup):
        solver.solve(db, state=st, result=res)
    torch.cuda.synchronize()

    # the timed steps run back to back (the host enqueues the next solve
    # while the device runs this one)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.solve(db, state=st, result=res)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps

    status = res["status"].cpu().numpy()
    iters = res["iters"].cpu().numpy()
    kkt = res["kkt_rel"].cpu().numpy()
    converged = int(np.sum((status & api.ST_CONVERGED) != 0))
    value = converged / (ms_step / 1e3)

    # per-launch kernel durations (HIP events on the solver's stream) from as
    # many steps again, each read after its step: waiting for the events
    # serialises the steps, so these are kept out of the timed region
    admm_ms, fin_ms = [], []
    for _ in range(args.steps):
        solver.solve(db, state=st, result=res)
        kt = solver.kernel_times()       # waits for this step's events
        admm_ms.append(kt["admm_ms"])
        fin_ms.append(kt["finalize_ms"])

    admm_avg = float(np.mean(admm_ms))
    fin_avg = float(np.mean(fin_ms))
    dev_ms = np.asarray(admm_ms) + np.asarray(fin_ms)  # device time of each step's launches
    flops_a = admm_flops(5, iters, api.admm_check_period(p))
    flops_f = float(np.sum(res["polish_flops"].double().cpu().numpy()))
    kernels = {
        "admm": {"bound": "alu", "kernel": "admm_kernel<5>", "dtype": "f32", "peak": PEAK_FP32_TFLOPS,
                 "ms": admm_avg, "flops": flops_a},
        "finalize": {"bound": "alu", "kernel": "FP64 polish: finalize_kernel<5> passes + gpolish_kernel<5,8>",
                     "dtype": "f64", "peak": PEAK_FP64_TFLOPS, "ms": fin_avg, "flops": flops_f},
    }

    def roof(name):
        k = kernels[name]
        achieved = k["flops"] / (k["ms"] / 1e3) / 1e12
        tr = measured_traffic(name)
        return {"bound": k["bound"], "achieved": round(achieved, 3), "peak": k["peak"], "unit": "TFLOP/s",
                "frac": round(achieved / k["peak"], 4), "traffic": tr, "kernel": k["kernel"],
                "kernel_dtype": k["dtype"], "kernel_ms": round(k["ms"], 4), "algorithmic_flops": k["flops"]}

    dominant = max(kernels, key=lambda n: kernels[n]["ms"])
    roofline = roof(dominant)
    other = roof("finalize" if dominant == "admm" else "admm")

    out = {
        "metric": "contact-force QPs/sec at rel. KKT resid <=1e-5 (plain vs batched/served); p50/p99",
        "value": round(value, 1),
        "unit": "QPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",  # FP32 ADMM iterations, FP64 polish and outputs' checks
        "data": "synthetic",
        "config": {"workload": "ellipsoid-m5-s16 (8192 grasps x 5 contacts x 16 wrenches, seed 16491)",
                   "qps": int(db.n_qps), "tol_rel": float(p.tol_rel), "form": "plain",
                   "polish": "fp64", "converged": converged,
                   "kkt_rel_max": float(np.max(kkt)),
                   "iters_mean": float(np.mean(iters)), "iters_p99": float(np.percentile(iters, 99)),
                   "finalize_ms": round(float(np.mean(fin_ms)), 4),
                   "polish_chunk": "auto (%d for %d QPs)" % (
                       api.bodex_qp_effective_params(p, db.n_qps)["polish_chunk"], db.n_qps),
                   "step_device_ms_median": round(float(np.median(dev_ms)), 4),
                   "step_device_ms_p99": round(float(np.percentile(dev_ms, 99)), 4)},
        "roofline": roofline,
        "roofline_other_kernel": other,
    }
    solver.close()

    if not args.no_forms:
        out["forms"] = forms(torch, api, wl)
        out["forms"]["tuning"] = tuning(torch, api, db)
        out["forms"]["sphere_m4_s6"] = small_form(torch, api, wl)
        out["forms"].update(served(torch, wl, args.serve_seconds, args.fifo_seconds))

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(batch)

    print(json.dumps(out), flush=True)


def forms(torch, api, wl):
    """Uneven batch: persistent graph launch vs per-(m, s) plain launches; and
    forward + backward on the differentiation workload."""
    from paper_2412_16490_amd import autotune
    res = {}
    b3 = wl.config(3)
    db3 = api.DeviceBatch(b3)
    s_max = int(np.max(np.diff(b3.woff)))
    side = torch.cuda.Stream()
    # the autotuner's choice for this shape: polish chunk (one-lane budget
    # before the contact-parallel polish), ADMM register budget, persistent
    # cost-sorted launch or not; cached per shape class
    base = api.default_params(m_max=5, s_max=s_max)
    t0 = time.perf_counter()
    knobs, table = autotune.tune(db3, base=base, reps=2)
    tune_s = time.perf_counter() - t0
    with torch.cuda.stream(side):
        pb = autotune.apply(base, knobs)
        pb.flags |= api.F_GRAPH
        sb = api.Solver(pb, stream=side.cuda_stream)
        st3 = api.new_state(db3.n_grasps, db3.n_qps, 5)
        r3 = api.new_result(db3.n_grasps, db3.n_qps, 5)
        for _ in range(2):
            sb.solve(db3, state=st3, result=r3)
        side.synchronize()
        t0 = time.perf_counter()
        n = 5
        for _ in range(n):
            sb.solve(db3, state=st3, result=r3)
        side.synchronize()
        tb = (time.perf_counter() - t0) / n
        conv = int(np.sum((r3["status"].cpu().numpy() & api.ST_CONVERGED) != 0))
        dflt = [t for t in table if t["knobs"] == {"polish_chunk": 20, "admm_waves": 2, "batched": 1}]
        res["batched"] = {"workload": "ellipsoid-m45-s6to32 (50,000 grasps, %d QPs)" % db3.n_qps,
                          "ms": round(tb * 1e3, 3), "qps_per_s": round(conv / tb, 1),
                          "converged": conv, "graph_replays": sb.stats()["graph_replays"],
                          "knobs": knobs, "knobs_from": "autotune cache (%d configurations, %.1f s)" % (
                              len(table), tune_s),
                          "tuning_best_ms": min(t["ms"] for t in table),
                          "tuning_chunk20_batched_ms": dflt[0]["ms"] if dflt else None}
        sb.close()
        # per-(m, s) plain launches of the same grasps
        groups = {}
        s_of = np.diff(b3.woff)
        for g in range(b3.n_grasps):
            groups.setdefault((int(b3.counts[g]), int(s_of[g])), []).append(g)
        subs = []
        for (m, s), gl in sorted(groups.items()):
            sub = b3.subset(gl)
            pp = api.default_params(m_max=5, s_max=s)
            subs.append((api.Solver(pp, stream=side.cuda_stream), api.DeviceBatch(sub)))
        outs = [(sv, d, api.new_state(d.n_grasps, d.n_qps, 5), api.new_result(d.n_grasps, d.n_qps, 5))
                for sv, d in subs]
        for sv, d, st, rr in outs:
            sv.solve(d, state=st, result=rr)
        side.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            for sv, d, st, rr in outs:
                sv.solve(d, state=st, result=rr)
        side.synchronize()
        tp = (time.perf_counter() - t0) / n
        convp = sum(int(np.sum((rr["status"].cpu().numpy() & api.ST_CONVERGED) != 0)) for _, _, _, rr in outs)
        res["per_size_plain"] = {"launches": len(outs), "ms": round(tp * 1e3, 3),
                                 "qps_per_s": round(convp / tp, 1), "converged": convp}
        for sv, _, _, _ in outs:
            sv.close()
    # the paper's force-closure energy on the headline grasps: six force-axis
    # wrenches per grasp with the normal-sum row (gamma = 0.5), and the beta = 0
    # QP baseline (gamma = 1)
    bfa = wl.force_axis_batch(wl.config(1))
    dfa = api.DeviceBatch(bfa)
    for name, gamma, beta in (("force_axis_gamma0.5", 0.5, 1.0), ("qp_baseline_beta0_gamma1", 1.0, 0.0)):
        pf = api.default_params(m_max=5, s_max=6)
        pf.gamma = gamma
        pf.beta = beta
        sf = api.Solver(pf)
        stf = api.new_state(dfa.n_grasps, dfa.n_qps, 5)
        rf = api.new_result(dfa.n_grasps, dfa.n_qps, 5)
        sf.solve(dfa, state=stf, result=rf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            sf.solve(dfa, state=stf, result=rf)
        torch.cuda.synchronize()
        tf = (time.perf_counter() - t0) / 5
        convf = int(np.sum((rf["status"].cpu().numpy() & api.ST_CONVERGED) != 0))
        res[name] = {"workload": "ellipsoid-m5, 8192 grasps x 6 force-axis wrenches (%d QPs)" % dfa.n_qps,
                     "ms": round(tf * 1e3, 3), "qps_per_s": round(convf / tf, 1), "converged": convf}
        sf.close()
    res["detach_surrogate"] = detach_form(torch, api, wl)
    res["circular_cone"] = cone_form(torch, api, wl)
    res["coarse_descent"] = descent_form(torch, api, wl)
    res["size_sweep"] = size_sweep(torch, api, wl)
    # forward + backward (differentiation workload, same shape as the headline)
    b2 = wl.config(2)
    db2 = api.DeviceBatch(b2)
    p2 = api.default_params(m_max=5, s_max=16)
    p2.flags |= api.F_TIMING
    s2 = api.Solver(p2)
    st2 = api.new_state(db2.n_grasps, db2.n_qps, 5)
    r2 = api.new_result(db2.n_grasps, db2.n_qps, 5)
    ones = torch.ones(db2.n_grasps, device="cuda")
    gp = torch.zeros_like(db2.points)
    gn = torch.zeros_like(db2.normals)
    for _ in range(2):
        s2.solve(db2, state=st2, result=r2)
        s2.backward(db2, st2, dL_dE=ones, out=(gp, gn))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bw = []
    for _ in range(5):
        s2.solve(db2, state=st2, result=r2)
        s2.backward(db2, st2, dL_dE=ones, out=(gp, gn))
        bw.append(s2.kernel_times()["backward_ms"])
    torch.cuda.synchronize()
    tfb = (time.perf_counter() - t0) / 5
    res["fwd_bwd"] = {"workload": "ellipsoid-m5-s16 (seed 16492)", "ms": round(tfb * 1e3, 3),
                      "backward_kernel_ms": round(float(np.mean(bw)), 4),
                      "grasps_per_s": round(db2.n_grasps / tfb, 1)}
    s2.close()
    return res


def size_sweep(torch, api, wl, sizes=(2048, 8192, 32768, 131072)):
    """The headline shape (5 contacts, 16 wrenches, ellipsoids) at several
    batch sizes: 8192 grasps are exactly one round of waves on the chip (the
    finalize's time is then its slowest waves'); larger batches run several
    rounds, which the hardware dispatcher balances."""
    out = {}
    stream = torch.cuda.current_stream()
    for G in sizes:
        b = wl.uniform_batch(16491, G, 5, 16, name="sweep")
        db = api.DeviceBatch(b)
        p = api.default_params(m_max=5, s_max=16)
        sv = api.Solver(p, stream=stream.cuda_stream)
        st = api.new_state(db.n_grasps, db.n_qps, 5)
        r = api.new_result(db.n_grasps, db.n_qps, 5)
        sv.solve(db, state=st, result=r)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record(stream)
        for _ in range(reps):
            sv.solve(db, state=st, result=r)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        conv = int(np.sum((r["status"].cpu().numpy() & api.ST_CONVERGED) != 0))
        out[str(G)] = {"qps": db.n_qps, "ms": round(ms, 3), "qps_per_s": round(conv / (ms / 1e3), 1),
                       "converged": conv}
        sv.close()
        del db, st, r
    return out


def descent_form(torch, api, wl, iters=20):
    """The bilevel loop on synthetic data (coarse stage on analytic objects):
    8192 floating 5-fingertip hands on ellipsoids, 16 wrenches each, `iters`
    gradient steps of w_qp sum_j Q_j + w_dist E^c_d in one call (per step:
    contact query, QP solve warm-started from the previous step, QP gradient,
    pose gradient, pose update), timed with events on the solver's stream;
    plus the per-launch times of the query and pose-gradient kernels."""
    hb = wl.hand_batch(16497, 8192, m=5, s=16)
    stream = torch.cuda.current_stream()
    sv = api.Solver(api.default_params(m_max=5, s_max=16), stream=stream.cuda_stream)
    dh = api.DeviceHand(hb)
    st = api.new_state(dh.n_grasps, dh.n_qps, 5)
    rs = api.new_result(dh.n_grasps, dh.n_qps, 5)
    rot0, trans0 = dh.rot.clone(), dh.trans.clone()
    sv.descend(dh, api.descent(iters=2), state=st, result=rs, trace=False)
    dh.rot.copy_(rot0)
    dh.trans.copy_(trans0)
    d = api.descent(iters=iters)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    rs, tr = sv.descend(dh, d, state=st, result=rs)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    trn = tr.cpu().numpy()
    conv = int(np.sum((rs["status"].cpu().numpy() & api.ST_CONVERGED) != 0))
    # the two hand kernels on their own (same stream)
    n = 50
    q = sv.contact_query(dh)
    e0.record(stream)
    for _ in range(n):
        sv.contact_query(dh, out=q)
    e1.record(stream)
    e1.synchronize()
    q_us = e0.elapsed_time(e1) / n * 1e3
    dP = torch.zeros((dh.n_grasps, 5, 3), device="cuda")
    e0.record(stream)
    for _ in range(n):
        sv.pose_gradient(dh, dP, dP, 1000.0, 0.01, 0.0)
    e1.record(stream)
    e1.synchronize()
    g_us = e0.elapsed_time(e1) / n * 1e3
    sv.close()
    # a small batch (64 hands): the step is launch-bound, so the descent
    # captured once in a hipGraph and replayed against eager launches
    # (a stream of its own: graphs are captured on a non-default stream)
    small = {}
    hs = wl.hand_batch(16498, 64, m=5, s=16)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    for label, flags in (("eager", 0), ("graph", api.F_GRAPH)):
        ss = api.Solver(api.default_params(m_max=5, s_max=16, flags_set=flags), stream=stream.cuda_stream)
        dhs = api.DeviceHand(hs)
        r0, t0_ = dhs.rot.clone(), dhs.trans.clone()
        sts = api.new_state(dhs.n_grasps, dhs.n_qps, 5)
        rss = api.new_result(dhs.n_grasps, dhs.n_qps, 5)
        ts = []
        for rep in range(4):
            with torch.cuda.stream(stream):
                dhs.rot.copy_(r0)
                dhs.trans.copy_(t0_)
            e0.record(stream)
            ss.descend(dhs, d, state=sts, result=rss, trace=False)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        small[label + "_ms_per_step"] = round(float(np.median(ts[1:])) / iters, 4)
        small[label + "_launches"] = ss.stats()["launches"]
        ss.close()
    return {"workload": "8192 floating hands x 5 fingertips on ellipsoids, 16 wrenches each (seed 16497)",
            "small_batch_64_hands": small,
            "iters": iters, "ms": round(ms, 3), "ms_per_step": round(ms / iters, 4),
            "grasp_steps_per_s": round(dh.n_grasps * iters / (ms / 1e3), 1),
            "qp_solves_per_s": round(dh.n_qps * iters / (ms / 1e3), 1),
            "last_step_converged": conv, "loss_first_mean": round(float(trn[0].mean()), 5),
            "loss_last_mean": round(float(trn[-1].mean()), 5),
            "frac_grasps_lowered": round(float(np.mean(trn[-1] < trn[0])), 4),
            "contact_query_kernel_us": round(q_us, 2), "pose_gradient_kernel_us": round(g_us, 2)}


def cone_form(torch, api, wl):
    """The exact circular friction cone of Eq. 1 on the headline grasps
    (8192 x 16 wrenches): ADMM with the truncated-cone projection and the FP64
    barrier polish; the finalize kernel's FP64 roofline; and the energy gap of
    the 8-facet pyramid the paper uses (its E is an upper bound of the cone's)."""
    b = wl.config(1)
    db = api.DeviceBatch(b)
    out = {}
    energies = {}
    for model in (api.CONE_CIRCULAR, api.CONE_PYRAMID8):
        p = api.default_params(m_max=5, s_max=16)
        p.friction_cone = model
        p.flags |= api.F_TIMING
        s = api.Solver(p)
        st = api.new_state(db.n_grasps, db.n_qps, 5, cone=model == api.CONE_CIRCULAR)
        r = api.new_result(db.n_grasps, db.n_qps, 5, polish_flops=True)
        s.solve(db, state=st, result=r)
        torch.cuda.synchronize()
        n = 5
        fin, adm = [], []
        t0 = time.perf_counter()
        for _ in range(n):
            s.solve(db, state=st, result=r)
            kt = s.kernel_times()
            fin.append(kt["finalize_ms"])
            adm.append(kt["admm_ms"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / n
        energies[model] = r["energy"].double().cpu().numpy()
        if model == api.CONE_CIRCULAR:
            conv = int(np.sum((r["status"].cpu().numpy() & api.ST_CONVERGED) != 0))
            pol = int(np.sum((r["status"].cpu().numpy() & api.ST_POLISHED) != 0))
            fin_ms = float(np.mean(fin))
            flops = float(np.sum(r["polish_flops"].double().cpu().numpy()))
            ach = flops / (fin_ms / 1e3) / 1e12
            out.update({"workload": "ellipsoid-m5-s16 (8192 grasps x 16 wrenches, seed 16491), exact cone",
                        "ms": round(ms, 3), "qps_per_s": round(conv / (ms / 1e3), 1), "converged": conv,
                        "polished": pol, "admm_ms": round(float(np.mean(adm)), 4), "finalize_ms": round(fin_ms, 4),
                        "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
                                     "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4),
                                     "traffic": measured_traffic("cone_finalize"),
                                     "kernel": "cone_finalize_kernel<5>", "kernel_dtype": "f64",
                                     "algorithmic_flops": flops}})
        s.close()
    ec, ep = energies[api.CONE_CIRCULAR], energies[api.CONE_PYRAMID8]
    gap = (ep - ec) / np.maximum(ec, 1e-12)
    out["pyramid_energy_gap"] = {"mean_rel": round(float(np.mean(gap)), 5),
                                 "median_rel": round(float(np.median(gap)), 5),
                                 "max_rel": round(float(np.max(gap)), 5),
                                 "grasps_pyramid_below_cone": int(np.sum(ep < ec * (1 - 1e-5)))}
    return out


# HBM bytes the fine-stage surrogate kernel must move: per contact R (36),
# T, c^f_w, p^f, p^c (12 each) read and dL/dR (36), dL/dT (12) written; per
# grasp the contact count and two weights read, Q' and E^f_d written.
DETACH_BYTES_PER_CONTACT = 84 + 48
DETACH_BYTES_PER_GRASP = 12 + 8
PEAK_HBM_GBS = 8000.0


def detach_form(torch, api, wl, large_only=False):
    """Fine-stage surrogate energies with Detach (Eq. 10-11) and their
    gradient: 2^20 grasps x 5 fingertips in one launch (HBM-bound), timed with
    events on the stream it runs on; plus the headline's 8192 grasps."""
    out = {}
    stream = torch.cuda.current_stream()
    sv = api.Solver(api.default_params(), stream=stream.cuda_stream)
    sizes = ((1 << 20, "large"),) if large_only else ((1 << 20, "large"), (8192, "headline_grasps"))
    for G, label in sizes:
        fc = api.DeviceFineContacts(wl.fine_contacts(16496, G, m=5))
        o = sv.detach_energy(fc)
        for _ in range(3):
            sv.detach_energy(fc, out=o)
        n = 20
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            sv.detach_energy(fc, out=o)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / n
        nbytes = G * 5 * DETACH_BYTES_PER_CONTACT + G * DETACH_BYTES_PER_GRASP
        gbs = nbytes / (ms / 1e3) / 1e9
        entry = {"workload": "%d grasps x 5 fingertips (seed 16496)" % G, "kernel_ms": round(ms, 5),
                 "grasps_per_s": round(G / (ms / 1e3), 1)}
        if label == "large":
            entry["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                 "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": measured_traffic("detach"),
                                 "kernel": "detach_kernel", "algorithmic_bytes": nbytes}
        out[label] = entry
        del fc, o
    sv.close()
    return out


def tuning(torch, api, db):
    """Headline solve time for each ADMM register budget (waves per SIMD)."""
    res = {}
    for occ in (1, 2, 3, 4):
        p = api.default_params(m_max=5, s_max=16)
        p.flags |= api.F_TIMING
        p.admm_waves = occ
        s = api.Solver(p)
        st = api.new_state(db.n_grasps, db.n_qps, 5)
        r = api.new_result(db.n_grasps, db.n_qps, 5)
        s.solve(db, state=st, result=r)
        torch.cuda.synchronize()
        ks = []
        for _ in range(5):
            s.solve(db, state=st, result=r)
            ks.append(s.kernel_times()["admm_ms"])
        res["admm_waves_%d_ms" % occ] = round(float(np.median(ks)), 4)
        s.close()
    # ADMM stopped at other tolerances (1e-5 = tol_rel; 1e30 = at its first
    # check), the FP64 polish lifting every QP to the 1e-5 bar (same final
    # criterion as the headline, which uses the pyramid's default 1e-1)
    for atol in (1e-5, 1e-3, 1e-2, 1e30):
        p = api.default_params(m_max=5, s_max=16)
        p.admm_tol = atol
        s = api.Solver(p)
        st = api.new_state(db.n_grasps, db.n_qps, 5)
        r = api.new_result(db.n_grasps, db.n_qps, 5)
        s.solve(db, state=st, result=r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            s.solve(db, state=st, result=r)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        conv = int(np.sum((r["status"].cpu().numpy() & api.ST_CONVERGED) != 0))
        res["admm_tol_%g" % atol] = {"ms": round(dt * 1e3, 4), "qps_per_s": round(conv / dt, 1),
                                     "converged": conv,
                                     "iters_mean": float(r["iters"].float().mean().item())}
        s.close()
    return res


def served(torch, wl, seconds, fifo_seconds):
    """Continuous batching vs FIFO plain launches on one Poisson stream (200
    requests/s, 50 forward+backward steps each, sizes log-U[16, 4096] grasps).
    The served form runs the first `seconds` of the stream; both forms run the
    same requests, those of the first `fifo_seconds` (the FIFO baseline
    serves about a tenth of the offered load, so the full window would take
    it many times longer).  Only converged QP solves are counted."""
    from paper_2412_16490_amd.serve import Server, serve_fifo_plain
    reqs = list(wl.request_stream(rate=200.0, duration=seconds))
    window = [r for r in reqs if r.arrival <= fifo_seconds]

    def run_served(rs):
        srv = Server(m_max=5, s_max=32, budget_bytes=4 << 30)
        srv.progress_every = 10.0
        st = srv.run(rs, realtime=True)
        srv.close()
        return {"qp_solves_per_s": round(st["qps_per_s"], 1), "converged": st["qp_solves_converged"],
                "qp_solves": st["qp_solves"], "offered_qp_solves_per_s": round(st["offered_qp_solves_per_s"], 1),
                "keeps_up": st["keeps_up"], "latency_p50_s": round(st["latency_p50_s"], 4),
                "latency_p99_s": round(st["latency_p99_s"], 4), "wall_s": round(st["wall_s"], 3),
                "ticks": st["ticks"], "queue_waiting_max": st["queue_waiting_max"],
                "queue_waiting_at": st["queue_waiting_at"],
                "around_solve_fraction": round(st["around_solve_fraction"], 4),
                "peak_device_bytes": st["peak_device_bytes"]}

    out = {}
    if seconds > fifo_seconds:
        out["served_full"] = {"stream": "%d requests over %.1f s, 50 steps" % (len(reqs), seconds),
                              **run_served(reqs)}
    out["served"] = {"stream": "%d requests over %.1f s, 50 steps (the window both forms run)" % (
        len(window), fifo_seconds), **run_served(window)}
    fifo = serve_fifo_plain(window, m_max=5, s_max=32, realtime=True)
    out["fifo_plain"] = {"stream": "the same %d requests" % fifo["requests"],
                         "qp_solves_per_s": round(fifo["qps_per_s"], 1), "converged": fifo["qp_solves_converged"],
                         "latency_p50_s": round(fifo["latency_p50_s"], 4),
                         "latency_p99_s": round(fifo["latency_p99_s"], 4), "wall_s": round(fifo["wall_s"], 3)}
    return out


def small_form(torch, api, wl, reps=20):
    """The 4-contact sphere workload (64 grasps x 6 wrenches = 384 QPs, tol
    1e-6): median and p99 of the device time of one solve's launches."""
    b = wl.config(0)
    db = api.DeviceBatch(b)
    p = api.default_params(m_max=4, s_max=6)
    p.flags |= api.F_TIMING
    p.tol_rel = 1e-6
    s = api.Solver(p)
    st = api.new_state(db.n_grasps, db.n_qps, 4)
    r = api.new_result(db.n_grasps, db.n_qps, 4)
    for _ in range(3):
        s.solve(db, state=st, result=r)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        s.solve(db, state=st, result=r)
        kt = s.kernel_times()
        ts.append(kt["admm_ms"] + kt["finalize_ms"])
    conv = int(np.sum((r["status"].cpu().numpy() & api.ST_CONVERGED) != 0))
    s.close()
    med = float(np.median(ts))
    return {"workload": "sphere-m4-s6 (64 grasps x 4 contacts x 6 wrenches, seed 16490, tol 1e-6)",
            "qps": int(db.n_qps), "converged": conv, "device_ms_median": round(med, 4),
            "device_ms_p99": round(float(np.percentile(ts, 99)), 4), "qps_per_s": round(conv / (med / 1e3), 1)}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch):
    """The FP64 oracle (as it stands) on the host: the cores this process is
    given (its CPU affinity, at most the 16-core share a GPU's job gets on a
    shared host), and one thread, over the same QPs."""
    import oracle
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    threads = max(1, min(affinity, 16))
    t0 = time.perf_counter()
    oracle.solve_batch(batch.counts, batch.woff, batch.points, batch.normals, batch.mu,
                       batch.wrench, nthreads=threads)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.solve_batch(batch.counts, batch.woff, batch.points, batch.normals, batch.mu,
                       batch.wrench, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": round(batch.n_qps / dt, 1), "unit": "QPs/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(), "logical_cpus_on_host": os.cpu_count(), "cpu_affinity": affinity,
            "value_1_thread": round(batch.n_qps / dt1, 1),
            "sample": "all %d QPs of the 8192-grasp workload: %.2f s wall on %d threads, %.2f s on 1 thread"
                      % (batch.n_qps, dt, threads, dt1)}


if __name__ == "__main__":
    main()
