"""Summaries of rocprofv3 result databases (rocpd SQLite).

  python -m paper_2011_11880_amd.rocprof_summary stats RUN_results.db [--match NAME]
      per-kernel dispatch count and duration statistics (microseconds)

  python -m paper_2011_11880_amd.rocprof_summary counters RUN_results.db --match NAME
      per-dispatch average of every counter collected for kernels whose name
      contains NAME (SQ counters are sums over the device)

  python -m paper_2011_11880_amd.rocprof_summary traffic \
        --fetch F.db --write W.db --copy-fetch CF.db --copy-write CW.db \
        --kernel NAME --copy-bytes BYTES --units U --out FILE.json [--last N]
      HBM bytes per dispatch of a kernel from FETCH_SIZE / WRITE_SIZE runs,
      each scaled by what the same counter reads for a plain copy kernel of
      known size (copy_bytes read and copy_bytes written per dispatch);
      --last N averages only the kernel's last N dispatches (the timed
      launches of a run that autotunes first), --first N its first N

  python -m paper_2011_11880_amd.rocprof_summary fp64 RUN_results.db \
        --kernel NAME --units U --out FILE.json [--last N]
      FP64 operations per dispatch from SQ_INSTS_VALU_FLOPS_FP64 (an
      instruction count per wavefront, FMA counted twice; x 64 lanes)
"""

from __future__ import annotations

import argparse
import json
import sqlite3
import sys


def kernel_stats(db, match=None):
    c = sqlite3.connect(db)
    rows = c.execute("select name, duration from kernels").fetchall()
    agg = {}
    for name, dur in rows:
        if match and match not in name:
            continue
        agg.setdefault(name, []).append(dur / 1000.0)
    out = []
    for name, d in agg.items():
        d.sort()
        out.append({"kernel": name, "calls": len(d), "total_us": sum(d),
                    "avg_us": sum(d) / len(d), "median_us": d[len(d) // 2],
                    "min_us": d[0], "max_us": d[-1]})
    out.sort(key=lambda r: -r["total_us"])
    return out


def counter_per_dispatch(db, counter, match, last=None, first=None):
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, dispatch_id, sum(value) from counters_collection "
                     "where counter_name = ? group by kernel_name, dispatch_id",
                     (counter,)).fetchall()
    rows = sorted((d, v) for name, d, v in rows if match in name)
    if first:
        rows = rows[:first]
    if last:
        rows = rows[-last:]
    vals = [v for _, v in rows]
    if not vals:
        raise SystemExit(f"no {counter} rows for kernels matching {match!r} in {db}")
    return sum(vals) / len(vals), len(vals)


def counters(db, match):
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, dispatch_id, counter_name, sum(value) from "
                     "counters_collection group by kernel_name, dispatch_id, counter_name").fetchall()
    agg = {}
    for name, _, counter, v in rows:
        if match in name:
            agg.setdefault(counter, []).append(v)
    if not agg:
        raise SystemExit(f"no counters for kernels matching {match!r} in {db}")
    return {k: (sum(v) / len(v), len(v)) for k, v in sorted(agg.items())}


def traffic(a):
    from .build import kernel_source_hash
    kib = 1024.0
    f_k, nf = counter_per_dispatch(a.fetch, "FETCH_SIZE", a.kernel, a.last, a.first)
    w_k, nw = counter_per_dispatch(a.write, "WRITE_SIZE", a.kernel, a.last, a.first)
    f_c, _ = counter_per_dispatch(a.copy_fetch, "FETCH_SIZE", a.copy_kernel)
    w_c, _ = counter_per_dispatch(a.copy_write, "WRITE_SIZE", a.copy_kernel)
    sf = a.copy_bytes / (f_c * kib)
    sw = a.copy_bytes / (w_c * kib)
    fetch = f_k * kib * sf
    write = w_k * kib * sw
    return {"kernel": a.kernel, "launch_units": a.units,
            "fetch_size_kib_per_dispatch": f_k, "write_size_kib_per_dispatch": w_k,
            "dispatches": [nf, nw],
            "copy_calibration": {"copy_bytes": a.copy_bytes,
                                 "fetch_size_kib": f_c, "write_size_kib": w_c,
                                 "fetch_scale": sf, "write_scale": sw},
            "hbm_read_bytes_per_launch": fetch, "hbm_write_bytes_per_launch": write,
            "hbm_bytes_per_launch": fetch + write,
            "kernel_source_sha256_16": kernel_source_hash(),
            "note": "FETCH_SIZE/WRITE_SIZE count L2-to-fabric traffic (Infinity Cache hits "
                    "included); scaled so that a plain copy reads and writes its own size"}


def fp64(a):
    from .build import kernel_source_hash
    n, nd = counter_per_dispatch(a.db, "SQ_INSTS_VALU_FLOPS_FP64", a.kernel, a.last)
    return {"kernel": a.kernel, "launch_units": a.units, "dispatches": nd,
            "sq_insts_valu_flops_fp64_per_dispatch": n,
            "fp64_flops_per_launch": 64.0 * n,
            "kernel_source_sha256_16": kernel_source_hash(),
            "note": "SQ_INSTS_VALU_FLOPS_FP64 counts ADD_F64 + MUL_F64 + 2 x FMA_F64 "
                    "instructions per wavefront; 64 lanes each, idle lanes included"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--match")
    cn = sub.add_parser("counters")
    cn.add_argument("db")
    cn.add_argument("--match", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "kernel", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--copy-kernel", default="copyBuffer")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--units", type=int, required=True)
    t.add_argument("--last", type=int, default=None)
    t.add_argument("--first", type=int, default=None)
    f = sub.add_parser("fp64")
    f.add_argument("db")
    for k in ("kernel", "out"):
        f.add_argument("--" + k, required=True)
    f.add_argument("--units", type=int, required=True)
    f.add_argument("--last", type=int, default=None)
    a = ap.parse_args(argv)
    if a.cmd == "fp64":
        d = fp64(a)
        with open(a.out, "w") as fh:
            json.dump(d, fh, indent=1)
        json.dump(d, sys.stdout, indent=1)
        print()
        return
    if a.cmd == "counters":
        for k, (avg, nd) in counters(a.db, a.match).items():
            print(f"{k:34s} {avg:20.1f}  ({nd} dispatches)")
        return
    if a.cmd == "stats":
        rows = kernel_stats(a.db, a.match)
        print(f"{'calls':>7} {'avg_us':>11} {'median_us':>11} {'min_us':>11} {'max_us':>11}  kernel")
        for r in rows:
            print(f"{r['calls']:7d} {r['avg_us']:11.3f} {r['median_us']:11.3f} "
                  f"{r['min_us']:11.3f} {r['max_us']:11.3f}  {r['kernel'][:100]}")
    else:
        d = traffic(a)
        with open(a.out, "w") as fh:
            json.dump(d, fh, indent=1)
        json.dump(d, sys.stdout, indent=1)
        print()


if __name__ == "__main__":
    main()
