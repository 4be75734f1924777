"""Short text summaries of rocprofv3 output (the rocpd SQLite databases).

  python -m paper_2412_16490_amd.profile_summary kernels DB --command CMD
      per-kernel call count, total / average / min / max duration

  python -m paper_2412_16490_amd.profile_summary counters DB --kernel SUBSTR [--kernel ...] --command CMD
      median per dispatch of every counter of a --pmc run (and the VALU busy
      fraction when SQ_ACTIVE_INST_VALU and GRBM_GUI_ACTIVE were collected)

  python -m paper_2412_16490_amd.profile_summary traffic --name NAME --kernel SUBSTR \\
      --fetch DB --write DB --copy-fetch DB --copy-write DB --copy-bytes N --command CMD
      HBM bytes per launch of the kernels whose name contains SUBSTR:
      FETCH_SIZE and WRITE_SIZE (KiB per dispatch, two counter runs), each
      scaled by what the same counter reads for a device copy of N bytes
      (the copy-calibration runs); prints the 'key: value' lines bench.py
      reads back (with the hash of the kernel sources they were taken on).

The output goes to stdout; profiles/ keeps it as text.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sqlite3
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")


# The sources each measured kernel is built and launched from: a traffic
# figure is reported only while these files are unchanged.
KERNEL_FILES = {
    "admm": ("bodex_math.h", "bodex_cone.h", "bodex_kernels.h", "k_admm.hip", "bodex_qp.hip"),
    "finalize": ("bodex_math.h", "bodex_cone.h", "bodex_gpolish.h", "bodex_kernels.h", "k_finalize.hip",
                 "k_finalize_sum.hip", "k_finalize_chunk.hip", "k_gpolish.hip", "bodex_qp.hip"),
    "cone_finalize": ("bodex_math.h", "bodex_cone.h", "bodex_kernels.h", "k_finalize_cone.hip", "bodex_qp.hip"),
    "detach": ("bodex_launch.h", "k_detach.hip"),
}


def kernel_source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in sorted(KERNEL_FILES[kernel]):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _durations(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration from kernels").fetchall()
    con.close()
    out = {}
    for name, d in rows:
        out.setdefault(name, []).append(float(d))
    return out


def kernels(db, command):
    d = _durations(db)
    total = sum(sum(v) for v in d.values())
    print("# kernel durations (rocprofv3 --kernel-trace --stats)")
    print("# command: %s" % command)
    print("# durations in microseconds")
    print("%-58s %6s %11s %10s %10s %10s %6s" % ("kernel", "calls", "total_us", "avg_us", "min_us", "max_us", "pct"))
    for name, v in sorted(d.items(), key=lambda kv: -sum(kv[1])):
        us = [x / 1e3 for x in v]
        print("%-58s %6d %11.1f %10.2f %10.2f %10.2f %6.2f" % (
            name[:58], len(v), sum(us), statistics.mean(us), min(us), max(us), 100.0 * sum(v) / total))


def _counter(db, counter, substr):
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, value from counters_collection where counter_name = ?",
                       (counter,)).fetchall()
    con.close()
    per = {}
    for did, name, val in rows:
        if substr in name:
            per[did] = per.get(did, 0.0) + float(val)
    return list(per.values())


def traffic(a):
    # --kernel may list several name substrings separated by '+': the launches
    # that together make one unit (their per-dispatch medians add)
    subs = [k.strip() for k in a.kernel.split("+") if k.strip()]
    fs = [_counter(a.fetch, "FETCH_SIZE", k) for k in subs]
    ws = [_counter(a.write, "WRITE_SIZE", k) for k in subs]
    cf = _counter(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
    cw = _counter(a.copy_write, "WRITE_SIZE", a.copy_kernel)
    kib = 1024.0
    sf = a.copy_bytes / (statistics.median(cf) * kib)
    sw = a.copy_bytes / (statistics.median(cw) * kib)
    f_kib = sum(statistics.median(v) for v in fs)
    w_kib = sum(statistics.median(v) for v in ws)
    fetch_b = f_kib * kib * sf
    write_b = w_kib * kib * sw
    print("# HBM traffic of %s (rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE)" % a.kernel)
    print("# command: %s" % a.command)
    print("# counters are KiB per dispatch; scaled by a %d-byte device copy (%s)" % (a.copy_bytes, a.copy_kernel))
    print("kernel: %s" % a.kernel)
    for k, fv, wv in zip(subs, fs, ws):
        print("part: %s  dispatches %d/%d  fetch_kib_median %.1f  write_kib_median %.1f" % (
            k, len(fv), len(wv), statistics.median(fv), statistics.median(wv)))
    print("fetch_kib_median: %.1f" % f_kib)
    print("write_kib_median: %.1f" % w_kib)
    print("copy_fetch_scale: %.4f" % sf)
    print("copy_write_scale: %.4f" % sw)
    print("fetch_bytes_per_launch: %.0f" % fetch_b)
    print("write_bytes_per_launch: %.0f" % write_b)
    print("bytes_per_launch: %.0f" % (fetch_b + write_b))
    print("source_hash: %s" % kernel_source_hash(a.name))


def counters(db, command, substrs):
    """Median per dispatch of every counter in a --pmc run, for the kernels
    whose names contain one of the substrings."""
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection").fetchall()
    con.close()
    per = {}
    for did, name, cname, val in rows:
        if any(sub in name for sub in substrs):
            per.setdefault(name, {}).setdefault(cname, {}).setdefault(did, 0.0)
            per[name][cname][did] += float(val)
    print("# rocprofv3 --pmc counters per dispatch (median over dispatches, summed over instances)")
    print("# command: %s" % command)
    for name in sorted(per):
        first = next(iter(per[name].values()))
        print("kernel: %s" % name.split("(")[0])
        print("dispatches: %d" % len(first))
        med = {c: statistics.median(v.values()) for c, v in per[name].items()}
        for cname in sorted(med):
            print("  %-24s %.4g" % (cname, med[cname]))
        if "SQ_ACTIVE_INST_VALU" in med and med.get("GRBM_GUI_ACTIVE"):
            # GRBM_GUI_ACTIVE sums the busy cycles of the 8 XCDs; a VALU
            # instruction occupies its SIMD 4 cycles
            print("  %-24s %.3f   (4 SQ_ACTIVE_INST_VALU / (1024 SIMDs x GRBM_GUI_ACTIVE / 8))" % (
                "valu_busy", 4.0 * med["SQ_ACTIVE_INST_VALU"] / (1024.0 * med["GRBM_GUI_ACTIVE"] / 8.0)))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("--command", required=True)
    c = sub.add_parser("counters")
    c.add_argument("db")
    c.add_argument("--kernel", action="append", required=True)
    c.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--name", required=True, choices=sorted(KERNEL_FILES))
    t.add_argument("--kernel", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--copy-kernel", default="copyBuffer")
    t.add_argument("--command", required=True)
    a = ap.parse_args()
    if a.what == "kernels":
        kernels(a.db, a.command)
    elif a.what == "counters":
        counters(a.db, a.command, a.kernel)
    else:
        traffic(a)


if __name__ == "__main__":
    main()
