#!/usr/bin/env python3
"""Throughput of FP64 residual + Jacobian evaluation on one MI355X.

Workload (default): a synthetic 70,000-bus grid with 88,207 branches shaped
like the paper's case study (Section IV-A), evaluated at 1000 random states.
One step = residual + Jacobian values at all 1000 states (the whole hot
path); inputs are resident in HBM before timing starts.  Two ways to run a
step are measured:

  batched  one launch over all 1000 states as instances
           (pf_eval_batch, instance-fastest layout, buses numbered
           breadth-first at setup; the input numbering beside it) -> headline value
  plain    1000 single-instance launches (pf_eval), each with its own
           state and output slot, replayed from a captured HIP graph

Prints one JSON line with the headline value, a roofline object for the
dominant kernel and the CPU oracle timed on a bounded sample.

The default run also summarises the other workloads under "others"; each
can be run alone with --config: c2 = 10,000-bus grid x 1024 scenario and N-1
instances; c3 = 256 grids of uneven size in one launch; c4 = adjoint (VJP)
with 64 cotangents on the 70,000-bus grid; newton = Newton power flow on the
70,000-bus grid with every step on the device; fdlf = fast decoupled power
flow on a meshed 70,000-bus grid; models = per-model cost (the 70k grid built
up model by model); newton_batch = N-1 contingency analysis (1024 Newton
solves at once) on the 10,000-bus grid; copy = HBM calibration.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "residual+Jacobian evals/s, 70k-bus FP64; batched vs plain; % HBM peak"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# schedules the autotuner picked on MI355X, keyed by GPU, kernel source and
# plan shape (a plan whose key is missing is tuned and appended)
TUNE_CACHE = os.path.join(ROOT, "paper_2011_11880_amd", "tune_cache.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def statics_bytes(info):
    """Setup-time arrays one launch reads: admittance entries (4 B column +
    2 x 8 B coefficients), per-bus slot maps and injections (40 B), per
    generator tables (32 B)."""
    return 20 * info["n_entries"] + 40 * info["n_bus"] + 32 * (info["n_pv"] + info["n_slack"])


def per_eval_bytes(n, nnz):
    """State read once, residual and Jacobian values written once."""
    return 8 * n + 8 * n + 8 * nnz


class Timer:
    def __init__(self, torch):
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.a.record()
        return self

    def __exit__(self, *e):
        self.b.record()
        self.torch.cuda.synchronize()
        self.ms = self.a.elapsed_time(self.b)


def time_ms(torch, fn, reps=10, warmup=2, batches=5):
    """Time of one fn(): the median over ``batches`` batches of the mean of
    ``reps`` back-to-back runs, each batch bracketed by events on the
    current stream (libpf launches on torch's current stream).  Running the
    launches back to back keeps the host's launch latency out of the
    figure, as a stream of evaluations would."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(batches):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b) / reps)
    ts.sort()
    return ts[len(ts) // 2]


def kernel_source_hash():
    from paper_2011_11880_amd.build import kernel_source_hash as h
    return h()


def measured_traffic(name, launch_units):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if d.get("launch_units") != launch_units:
        return None
    return d.get("hbm_bytes_per_launch")


def tune_cache(args):
    """The tune-cache file the autotuner reads and appends to; with --retune
    a fresh file under the system's temporary directory, so every schedule
    is searched again."""
    if getattr(args, "retune", False):
        import tempfile
        if not hasattr(args, "_fresh_cache"):
            args._fresh_cache = os.path.join(tempfile.mkdtemp(), "tune_cache.txt")
        return args._fresh_cache
    return TUNE_CACHE


def fp64_rate(name, launch_units, ms):
    """FP64 operations per launch of the dominant kernel from the committed
    rocprofv3 counter summary (64 x SQ_INSTS_VALU_FLOPS_FP64 per dispatch),
    if it was taken on the current kernel source, and the rate they give at
    the measured time against the 78.6 TFLOP/s FP64 vector peak."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return {"fp64_tflops": None}
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha256_16") != kernel_source_hash() or \
            d.get("launch_units") != launch_units:
        return {"fp64_tflops": None}
    flops = d["fp64_flops_per_launch"]
    rate = flops / (ms * 1e-3) / 1e12
    return {"fp64_flops_per_launch": flops, "fp64_tflops": rate,
            "fp64_frac": rate / FP64_PEAK_TFLOPS}


def host_cpu():
    """The host the CPU baselines ran on: usable cores and the processor model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"usable_cores": len(os.sched_getaffinity(0)), "cpus": os.cpu_count(), "model": model}


def cpu_baseline(net, states, seconds=12.0, max_states=1000):
    """The CPU oracle (plain C + scipy triplet assembly) on a bounded sample."""
    from oracle import oracle as O
    O.build()
    n_done = 0
    t0 = time.perf_counter()
    for y in states[:max_states]:
        O.residual(net, y)
        O.jacobian(net, y)
        n_done += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": n_done / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_done} of the {len(states)} states, residual + Jacobian "
                      f"(triplets summed into CSR), {dt:.1f} s",
            "host": host_cpu()}


def _oracle_share(task):
    """Worker process: the oracle's residual + Jacobian on a share of
    independent instances, until the share or the time budget ends.  An
    instance is (network, state) or, for a batched plan, (load scale row,
    PV scale row, outaged branch, state) applied to the base network."""
    base, items, seconds = task
    from oracle import oracle as O
    O.build()
    t0 = time.perf_counter()
    done = 0
    for it in items:
        if base is None:
            net, y = it
        else:
            ls, ps, outage, y = it
            net = base if outage < 0 else base.without_branch(int(outage))
            if ls is not None:
                net = net.copy()
                net.load_p = base.load_p * ls
                net.load_q = base.load_q * ls
                net.pv_p = base.pv_p * ps
        O.residual(net, y)
        O.jacobian(net, y)
        done += 1
        if time.perf_counter() - t0 > seconds:
            break
    return done, time.perf_counter() - t0


def cpu_baseline_parallel(base, items, seconds, what):
    """The CPU oracle over independent instances in one process per host core
    (at most 16), each timed by its own clock; throughput is the sum of the
    processes' rates (process start-up excluded)."""
    import multiprocessing as mp
    workers = max(1, min(16, len(os.sched_getaffinity(0)), len(items)))
    shares = [items[w::workers] for w in range(workers)]
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_share, [(base, sh, seconds) for sh in shares])
    done = sum(r[0] for r in res)
    rate = sum(r[0] / r[1] for r in res if r[1] > 0)
    return {"value": rate, "unit": "evals/s", "cores": workers, "kind": "oracle",
            "sample": f"{done} of the {len(items)} {what}, residual + Jacobian, "
                      f"{workers} processes, at most {seconds:.0f} s each",
            "host": host_cpu()}


def cpu_baseline_solve(run, what):
    """The CPU oracle's own solver loop (plain-C evaluation, scipy's sparse
    LU) timed once on the same case, one core.  ``run(O)`` returns the
    number of iterations and the final largest mismatch."""
    from oracle import oracle as O
    O.build()
    t0 = time.perf_counter()
    its, final = run(O)
    dt = time.perf_counter() - t0
    return {"total_ms": dt * 1e3, "iterations": int(its), "final_mismatch": float(final),
            "cores": 1,
            "kind": "oracle", "sample": what}


def run_c1(args, torch, dev):
    from paper_2011_11880_amd import synth
    from paper_2011_11880_amd.api import Plan

    S = args.states
    log(f"[bench] building 70k grid and {S} states")
    net = synth.grid_70k()
    Y = synth.random_states(net, S, seed=1001)
    res = {}

    # ---- batched: all states as instances of one launch; instance rows
    # padded to a multiple of 16 (128 B) so every 64-instance segment is
    # aligned.  The plan numbers the buses breadth-first at setup, so the
    # state rows a work item gathers are neighbours in memory; the states
    # are written in the plan's order before timing (the same launch on the
    # input numbering is reported beside it)
    LD = -(-S // 16) * 16
    bp = Plan(net, batch=dict(n_inst=S, inst_stride=LD), device=0, bus_order="locality")
    info = bp.info
    n, nnz = bp.n, bp.nnz
    Xh = np.zeros((n, LD))
    Xh[:, :S] = bp.to_plan(Y).T
    X = torch.from_numpy(Xh).to(dev)
    del Xh
    Fb = torch.empty((n, LD), dtype=torch.float64, device=dev)
    Jb = torch.empty((nnz, LD), dtype=torch.float64, device=dev)
    best = bp.autotune(X, Fb, Jb, reps=10, cache=tune_cache(args))
    log("[bench] batched schedule", best, "from the tune cache" if bp.tune_hit else "searched")
    hit_b = bp.tune_hit
    # each step replays a captured HIP graph holding the one batched launch
    # (the same launch eagerly is reported beside it)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())

    def captured(fn):
        fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                fn()
        torch.cuda.synchronize()
        return g

    def timed(g):
        for _ in range(args.warmup):
            g.replay()
        with Timer(torch) as t:
            for _ in range(args.steps):
                g.replay()
        return t.ms / args.steps

    log("[bench] batched timed (graph replay)")
    gb = captured(lambda: bp.eval_batch(X, Fb, Jb))
    ms_b = timed(gb)
    bytes_b = S * per_eval_bytes(n, nnz) + statics_bytes(info)
    for _ in range(args.warmup):
        bp.eval_batch(X, Fb, Jb)
    with Timer(torch) as te:
        for _ in range(args.steps):
            bp.eval_batch(X, Fb, Jb)
    ms_e = te.ms / args.steps
    res["batched"] = {"ms_per_step": ms_b, "evals_per_s": S / (ms_b * 1e-3),
                      "launch_bytes": bytes_b, "gbs": bytes_b / (ms_b * 1e-3) / 1e9,
                      "schedule": bp.schedule, "schedule_from_tune_cache": hit_b,
                      "launch": "HIP graph replay", "eager_ms_per_step": ms_e}
    res["batched"]["hbm_frac"] = res["batched"]["gbs"] / HBM_PEAK_GBS
    del gb
    res["batched"]["bus_order"] = "breadth-first at setup (states and outputs in the plan's order)"
    if args.headline_only:
        del Fb, Jb, X
        return _c1_out(args, torch, dev, net, Y, S, LD, n, nnz, res)
    # equation / Jacobian split of the same launch (Table III reports the two
    # separately): residual-only and Jacobian-only launches, each from its
    # own graph; algorithmic bytes read X once and write F or J
    bytes_f = S * 16 * n + statics_bytes(info)
    bytes_j = S * (8 * n + 8 * nnz) + statics_bytes(info)
    gf = captured(lambda: bp.eval_batch(X, Fb, None, want_J=False))
    ms_f = timed(gf)
    del gf
    gj = captured(lambda: bp.eval_batch(X, None, Jb, want_F=False))
    ms_j = timed(gj)
    del gj
    res["batched"]["residual_only_ms"] = ms_f
    res["batched"]["residual_only_hbm_frac"] = bytes_f / (ms_f * 1e-3) / 1e9 / HBM_PEAK_GBS
    res["batched"]["jacobian_only_ms"] = ms_j
    res["batched"]["jacobian_only_hbm_frac"] = bytes_j / (ms_j * 1e-3) / 1e9 / HBM_PEAK_GBS
    # context: the same outputs written in the same layout by torch's fill
    # kernel alone (no state reads, no arithmetic), a practical ceiling for
    # the launch's store stream (a non-zero value, so no memset node)
    def fill_outputs():
        Fb[:, :S].fill_(1.0)
        Jb[:, :S].fill_(1.0)

    gw = captured(fill_outputs)
    ms_w = timed(gw)
    del gw
    bytes_w = S * 8 * (n + nnz)
    res["batched"]["outputs_fill_ms"] = ms_w
    res["batched"]["outputs_fill_gbs"] = bytes_w / (ms_w * 1e-3) / 1e9
    res["batched"]["outputs_fill_over_fused"] = ms_w / ms_b
    log("[bench] batched", json.dumps(res["batched"]))
    del Fb, Jb, X
    # the same batch on the input bus numbering
    bl = Plan(net, batch=dict(n_inst=S, inst_stride=LD), device=0)
    Xh = np.zeros((n, LD))
    Xh[:, :S] = Y.T
    Xl = torch.from_numpy(Xh).to(dev)
    del Xh
    Fl = torch.empty((n, LD), dtype=torch.float64, device=dev)
    Jl = torch.empty((nnz, LD), dtype=torch.float64, device=dev)
    best_l = bl.autotune(Xl, Fl, Jl, reps=10, cache=tune_cache(args))
    gl = captured(lambda: bl.eval_batch(Xl, Fl, Jl))
    ms_l = timed(gl)
    del gl
    res["batched_input_order"] = {
        "ms_per_step": ms_l, "evals_per_s": S / (ms_l * 1e-3),
        "gbs": bytes_b / (ms_l * 1e-3) / 1e9,
        "hbm_frac": bytes_b / (ms_l * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "schedule": best_l, "schedule_from_tune_cache": bl.tune_hit}
    log("[bench] batched, input order", json.dumps(res["batched_input_order"]))
    del Xl, Fl, Jl, bl

    # ---- plain: one launch per state, distinct slots, captured graph
    if not args.no_plain:
        pp = Plan(net, device=0)
        Xs = torch.from_numpy(Y).to(dev)
        Fs = torch.empty((S, n), dtype=torch.float64, device=dev)
        Js = torch.empty((S, nnz), dtype=torch.float64, device=dev)
        best = pp.autotune(Xs[0], Fs[0], Js[0], reps=20, cache=tune_cache(args))
        log("[bench] plain schedule", best, "from the tune cache" if pp.tune_hit else "searched")
        for s in range(S):  # eager warmup
            pp.eval(Xs[s], Fs[s], Js[s])
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            with torch.cuda.graph(g, stream=st):
                for s in range(S):
                    pp.eval(Xs[s], Fs[s], Js[s])
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            g.replay()
        with Timer(torch) as tp:
            for _ in range(args.steps):
                g.replay()
        ms_p = tp.ms / args.steps
        bytes_p = per_eval_bytes(n, nnz) + statics_bytes(pp.info)
        res["plain"] = {"ms_per_step": ms_p, "evals_per_s": S / (ms_p * 1e-3),
                        "us_per_eval": ms_p * 1e3 / S, "launch_bytes": bytes_p,
                        "gbs": bytes_p * S / (ms_p * 1e-3) / 1e9, "schedule": pp.schedule}
        res["plain"]["hbm_frac"] = res["plain"]["gbs"] / HBM_PEAK_GBS
        log("[bench] plain", json.dumps(res["plain"]))
        # equation / Jacobian split (the paper's Table III reports the two
        # separately): the same 1000 evaluations as residual-only and
        # Jacobian-only launches, each replayed from its own graph
        for part, fn in (("residual_only", lambda s: pp.eval_residual(Xs[s], Fs[s])),
                         ("jacobian_only", lambda s: pp.eval_jacobian(Xs[s], Js[s]))):
            gp = torch.cuda.CUDAGraph()
            with torch.cuda.stream(st):
                with torch.cuda.graph(gp, stream=st):
                    for s in range(S):
                        fn(s)
            torch.cuda.synchronize()
            gp.replay()
            with Timer(torch) as tq:
                for _ in range(args.steps):
                    gp.replay()
            res["plain"][part + "_us"] = tq.ms * 1e3 / (args.steps * S)
            del gp
        log("[bench] plain split", res["plain"]["residual_only_us"], res["plain"]["jacobian_only_us"])
        # the same 1000 single-state launches spread round-robin over 4
        # streams inside one graph (fork/join), so that one launch's ramp-up
        # and drain overlap its neighbours'; evaluations only read the plan
        n_side = 4
        side = [torch.cuda.Stream() for _ in range(n_side)]
        gc = torch.cuda.CUDAGraph()
        events = []   # the fork/join events live as long as the graph
        with torch.cuda.stream(st):
            with torch.cuda.graph(gc, stream=st):
                events.append(torch.cuda.Event())
                events[0].record(st)
                for q in side:
                    q.wait_event(events[0])
                for s in range(S):
                    with torch.cuda.stream(side[s % n_side]):
                        pp.eval(Xs[s], Fs[s], Js[s])
                for q in side:
                    events.append(torch.cuda.Event())
                    events[-1].record(q)
                    st.wait_event(events[-1])
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            gc.replay()
        with Timer(torch) as tc:
            for _ in range(args.steps):
                gc.replay()
        ms_c = tc.ms / args.steps
        res["plain_4_streams"] = {"ms_per_step": ms_c, "evals_per_s": S / (ms_c * 1e-3),
                                  "us_per_eval": ms_c * 1e3 / S,
                                  "gbs": bytes_p * S / (ms_c * 1e-3) / 1e9}
        res["plain_4_streams"]["hbm_frac"] = res["plain_4_streams"]["gbs"] / HBM_PEAK_GBS
        log("[bench] plain 4 streams", json.dumps(res["plain_4_streams"]))
        del gc
        del events
        # per-launch floors for context, replayed the same way: an empty
        # launch (64 B fill) and a device copy moving the bytes of one
        # evaluation (half read, half written)
        half = int(bytes_p // 16)
        src = torch.randn((S, half), dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        tiny = torch.empty((S, 8), dtype=torch.float64, device=dev)
        for name, fn in (("empty_launch_us", lambda s: tiny[s].fill_(1.0)),
                         ("copy_same_bytes_us", lambda s: dst[s].copy_(src[s]))):
            for s in range(S):
                fn(s)
            torch.cuda.synchronize()
            gf = torch.cuda.CUDAGraph()
            with torch.cuda.stream(st):
                with torch.cuda.graph(gf, stream=st):
                    for s in range(S):
                        fn(s)
            torch.cuda.synchronize()
            gf.replay()
            with Timer(torch) as tf:
                for _ in range(args.steps):
                    gf.replay()
            res["plain"][name] = tf.ms * 1e3 / (args.steps * S)
            del gf
        log("[bench] plain floors", res["plain"]["empty_launch_us"], res["plain"]["copy_same_bytes_us"])
        del src, dst, tiny
        del g, Fs, Js, Xs
        # the same launches on a plan whose buses are numbered breadth-first
        # at setup (states converted to the plan's order beforehand)
        pl = Plan(net, device=0, bus_order="locality")
        Xl = torch.from_numpy(pl.to_plan(Y)).to(dev)
        Fl = torch.empty((S, n), dtype=torch.float64, device=dev)
        Jl = torch.empty((S, nnz), dtype=torch.float64, device=dev)
        best = pl.autotune(Xl[0], Fl[0], Jl[0], reps=20, cache=tune_cache(args))
        us1, us4 = time_plain_launches(torch, pl, Xl, Fl, Jl, args.steps, args.warmup)
        res["plain_locality_order"] = {
            "us_per_eval": us1, "evals_per_s": 1e6 / us1,
            "gbs": bytes_p / (us1 * 1e-6) / 1e9, "hbm_frac": bytes_p / (us1 * 1e-6) / 1e9 /
            HBM_PEAK_GBS, "us_per_eval_4_streams": us4,
            "hbm_frac_4_streams": bytes_p / (us4 * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "schedule": best, "schedule_from_tune_cache": pl.tune_hit}
        log("[bench] plain, locality order", json.dumps(res["plain_locality_order"]))
        del Xl, Fl, Jl

    return _c1_out(args, torch, dev, net, Y, S, LD, n, nnz, res)


def _c1_out(args, torch, dev, net, Y, S, LD, n, nnz, res):
    """The headline JSON object of the default workload (and the others'
    summaries unless --no-others)."""
    head = res["batched"]
    # overlay-free batches with an even instance count and pitch run the
    # two-instances-per-lane kernel
    head_kernel = "k_eval_batch2" if S % 2 == 0 and LD % 2 == 0 else "k_eval_batch"
    out = {
        "metric": METRIC, "value": head["evals_per_s"], "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "70k-bus synthetic grid (88,207 branches), residual + Jacobian "
                               f"values at {S} random states per step",
                   "n_bus": net.n_bus, "n_branch": net.n_branch, "n": n, "nnz": nnz,
                   "states": S, "variant": "batched (states as instances of one launch)",
                   "bus_order": "breadth-first at setup (PF_ORDER_LOCALITY)",
                   "instance_row_pitch": LD, "launch": "one HIP graph replay per step",
                   "schedule": head["schedule"],
                   "schedule_note": "one wavefront per work item (grid_blocks -1): the "
                                    "autotuner's persistent grid sizes measure slower"},
        "roofline": {"bound": "hbm", "kernel": head_kernel,
                     "achieved": head["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["hbm_frac"],
                     "traffic": measured_traffic(f"{head_kernel}_70k_x1000_traffic.json", S),
                     "bytes_per_launch": head["launch_bytes"],
                     "kernel_source_sha256_16": kernel_source_hash(),
                     **fp64_rate(f"{head_kernel}_70k_x1000_fp64.json", S, head["ms_per_step"])},
        "variants": res,
        "paper_context": {"evals_per_s": 294, "equation_ms": 0.6, "jacobian_ms": 2.8,
                          "note": "workflow 5 (serial + SIMD) of Table III on a 6-core Xeon "
                                  "W-2133, real 70k grid, Jacobian time incl. triplet assembly"},
    }
    if not args.no_cpu:
        log("[bench] cpu baseline")
        out["cpu_baseline"] = cpu_baseline(net, Y, seconds=args.cpu_seconds)
    if not args.no_others:
        out["others"] = {}
        for name, fn in (("scenarios_10k_x1024", run_c2), ("uneven_256_grids", run_c3),
                         ("adjoint_70k_k64", run_c4), ("newton_device_70k", run_newton),
                         ("fdlf_70k_meshed", run_fdlf), ("per_model_70k", run_models),
                         ("newton_batch_10k_n1", run_newton_batch)):
            log(f"[bench] {name}")
            out["others"][name] = fn(args, torch, dev, net70k=net,
                                     plain_us=res.get("plain", {}).get("us_per_eval"))
            log(f"[bench] {name}", json.dumps(out["others"][name]))
    return out


def time_plain_launches(torch, plan, Xs, Fs, Js, steps, warmup):
    """Microseconds per evaluation of len(Xs) single-instance launches (each
    state its own output slots) replayed from a captured graph, on one
    stream and spread round-robin over 4 streams (fork/join)."""
    S = Xs.shape[0]
    for s in range(S):
        plan.eval(Xs[s], Fs[s], Js[s])
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    side = [torch.cuda.Stream() for _ in range(4)]
    g1 = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        with torch.cuda.graph(g1, stream=st):
            for s in range(S):
                plan.eval(Xs[s], Fs[s], Js[s])
    g4 = torch.cuda.CUDAGraph()
    events = []   # the fork/join events live as long as the graph
    with torch.cuda.stream(st):
        with torch.cuda.graph(g4, stream=st):
            events.append(torch.cuda.Event())
            events[0].record(st)
            for q in side:
                q.wait_event(events[0])
            for s in range(S):
                with torch.cuda.stream(side[s % 4]):
                    plan.eval(Xs[s], Fs[s], Js[s])
            for q in side:
                events.append(torch.cuda.Event())
                events[-1].record(q)
                st.wait_event(events[-1])
    torch.cuda.synchronize()
    out = []
    for g in (g1, g4):
        for _ in range(warmup):
            g.replay()
        with Timer(torch) as t:
            for _ in range(steps):
                g.replay()
        out.append(t.ms * 1e3 / (steps * S))
    torch.cuda.synchronize()
    del g, g1, g4
    del events
    return out[0], out[1]


def run_c2(args, torch, dev, **kw):
    """10,000-bus grid, 1024 instances in one launch: 512 load/renewable
    scenarios and 512 N-1 contingencies, against the plain single-instance
    kernel on the same grid."""
    from paper_2011_11880_amd import synth
    from paper_2011_11880_amd.api import Plan
    net = synth.grid_10k()
    I = 1024
    ls = np.ones((I, net.n_load))
    ps = np.ones((I, net.n_pv))
    a, b = synth.batch_scenarios(net, 512, seed=2001)
    ls[:512], ps[:512] = a, b
    out = np.full(I, -1, np.int32)
    out[512:] = synth.contingencies(net, 512, seed=2002)
    bp = Plan(net, batch=dict(n_inst=I, load_scale=ls, pv_scale=ps, outage=out), device=0)
    Y = synth.random_states(net, I, seed=2003)
    X = torch.from_numpy(np.ascontiguousarray(Y.T)).to(dev)
    F = torch.empty((bp.n, I), dtype=torch.float64, device=dev)
    J = torch.empty((bp.nnz, I), dtype=torch.float64, device=dev)
    bp.autotune(X, F, J, reps=10, cache=tune_cache(args))
    hit = bp.tune_hit
    ms = time_ms(torch, lambda: bp.eval_batch(X, F, J), reps=20)
    nb = I * (per_eval_bytes(bp.n, bp.nnz) + 8 * (net.n_load + net.n_pv) + 4) + \
        statics_bytes(bp.info)
    pp = Plan(net, device=0)
    Xs = torch.from_numpy(Y[:64]).to(dev)
    Fs = torch.empty((64, pp.n), dtype=torch.float64, device=dev)
    Js = torch.empty((64, pp.nnz), dtype=torch.float64, device=dev)
    pp.autotune(Xs[0], Fs[0], Js[0], reps=20, cache=tune_cache(args))

    def plain64():
        for s in range(64):
            pp.eval(Xs[s], Fs[s], Js[s])
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    plain64()
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            plain64()
    torch.cuda.synchronize()
    ms_p = time_ms(torch, g.replay) / 64
    res = {"grid": "10,000 buses, 12,500 branches", "instances": I,
           "batched_ms": ms, "batched_evals_per_s": I / (ms * 1e-3),
           "batched_gbs": nb / (ms * 1e-3) / 1e9,
           "batched_hbm_frac": nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "batched_bytes_per_launch": nb,
           "batched_traffic": measured_traffic("k_eval_batch_10k_x1024_traffic.json", I),
           "plain_us_per_eval": ms_p * 1e3, "plain_evals_per_s": 1e3 / ms_p,
           "batched_over_plain": (I / ms) / (1.0 / ms_p), "schedule": bp.schedule,
           "schedule_from_tune_cache": hit}
    del g, F, J, X
    # the same batch with the buses numbered breadth-first at setup (the
    # overlays address loads, PV units and branches, which keep their order)
    bl = Plan(net, batch=dict(n_inst=I, load_scale=ls, pv_scale=ps, outage=out), device=0,
              bus_order="locality")
    Xl = torch.from_numpy(np.ascontiguousarray(bl.to_plan(Y).T)).to(dev)
    Fl = torch.empty((bl.n, I), dtype=torch.float64, device=dev)
    Jl = torch.empty((bl.nnz, I), dtype=torch.float64, device=dev)
    bl.autotune(Xl, Fl, Jl, reps=10, cache=tune_cache(args))
    ms_l = time_ms(torch, lambda: bl.eval_batch(Xl, Fl, Jl), reps=20)
    res["locality_order"] = {"batched_ms": ms_l, "batched_evals_per_s": I / (ms_l * 1e-3),
                             "batched_hbm_frac": nb / (ms_l * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "schedule": bl.schedule, "schedule_from_tune_cache": bl.tune_hit}
    del Xl, Fl, Jl, bl
    if not getattr(args, "no_cpu", False):
        log("[bench] c2 CPU oracle over instances")
        items = [(ls[k] if k < 512 else None, ps[k] if k < 512 else None, int(out[k]), Y[k])
                 for k in range(I)]
        res["cpu_baseline"] = cpu_baseline_parallel(net, items, 8.0, "instances")
    return res


def run_c3(args, torch, dev, **kw):
    """256 grids with bus counts log-uniform in [500, 20000], one launch."""
    from paper_2011_11880_amd import synth
    from paper_2011_11880_amd.api import Plan
    nets = synth.uneven_grids(256, seed=3000)
    mp = Plan.multi(nets, device=0)
    xs = np.concatenate([synth.random_states(n, seed=g) for g, n in enumerate(nets)])
    x = torch.from_numpy(xs).to(dev)
    F = torch.empty(mp.n, dtype=torch.float64, device=dev)
    J = torch.empty(mp.nnz, dtype=torch.float64, device=dev)
    best = mp.autotune(x, F, J, reps=10, cache=tune_cache(args))
    hit = mp.tune_hit
    ms = time_ms(torch, lambda: mp.eval(x, F, J), reps=20)
    # the same grids numbered breadth-first at setup
    ml = Plan.multi(nets, device=0, bus_order="locality")
    xl = torch.from_numpy(ml.to_plan(xs)).to(dev)
    best_l = ml.autotune(xl, F, J, reps=10, cache=tune_cache(args))
    ms_l = time_ms(torch, lambda: ml.eval(xl, F, J), reps=20)
    del ml, xl
    nb = per_eval_bytes(mp.n, mp.nnz) + statics_bytes(mp.info)
    res = {"grids": 256, "buses": int(sum(n.n_bus for n in nets)), "n": mp.n, "nnz": mp.nnz,
           "ms": ms, "grid_evals_per_s": 256 / (ms * 1e-3), "gbs": nb / (ms * 1e-3) / 1e9,
           "hbm_frac": nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": nb,
           "traffic": measured_traffic("k_eval_single_256_uneven_grids_traffic.json", 1),
           "autotuned_schedule": best, "schedule_from_tune_cache": hit,
           "locality_order": {"ms": ms_l, "grid_evals_per_s": 256 / (ms_l * 1e-3),
                              "hbm_frac": nb / (ms_l * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "autotuned_schedule": best_l}}
    if not getattr(args, "no_cpu", False):
        log("[bench] c3 CPU oracle over grids")
        off = np.cumsum([0] + [n.n_var for n in nets])
        items = [(n, xs[off[g]:off[g + 1]]) for g, n in enumerate(nets)]
        res["cpu_baseline"] = cpu_baseline_parallel(None, items, 8.0, "grids")
    return res


def run_c4(args, torch, dev, net70k=None, plain_us=None, **kw):
    """Adjoint on the 70,000-bus grid for 64 cotangents (state and parameter
    gradients), against one forward residual + Jacobian evaluation."""
    from paper_2011_11880_amd import synth
    from paper_2011_11880_amd.api import Plan
    net = net70k if net70k is not None else synth.grid_70k()
    p = Plan(net, device=0)
    K = 64
    x = torch.from_numpy(synth.random_states(net, seed=4000)).to(dev)
    W = torch.randn((p.n, K), dtype=torch.float64, device=dev,
                    generator=torch.Generator(device=dev).manual_seed(4001))
    gx = torch.empty((p.n, K), dtype=torch.float64, device=dev)
    gp = torch.empty((p.n_params, K), dtype=torch.float64, device=dev)
    ms = time_ms(torch, lambda: p.vjp(x, W, gx, gp))
    if plain_us is None:   # forward reference: one evaluation inside a captured graph
        F = torch.empty(p.n, dtype=torch.float64, device=dev)
        J = torch.empty(p.nnz, dtype=torch.float64, device=dev)
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        p.eval(x, F, J)
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            with torch.cuda.graph(g, stream=st):
                for _ in range(20):
                    p.eval(x, F, J)
        torch.cuda.synchronize()
        plain_us = time_ms(torch, g.replay) * 1e3 / 20
    ms_f = plain_us * 1e-3
    nb = K * (8 * p.n * 2 + 8 * p.n_params) + 8 * p.n + statics_bytes(p.info) + \
        64 * net.n_branch
    # the same adjoint with the buses numbered breadth-first at setup: state,
    # cotangent and gradient rows of neighbouring buses then sit together
    pl = Plan(net, device=0, bus_order="locality")
    perm = torch.from_numpy(pl.state_perm().astype(np.int64)).to(dev)
    xl = x[perm].contiguous()
    ms_l = time_ms(torch, lambda: pl.vjp(xl, W, gx, gp))
    pl.close()
    return {"cotangents": K, "vjp_ms": ms, "forward_us": plain_us,
            "vjp_over_forward": ms / ms_f, "vjp_per_cotangent_over_forward": ms / ms_f / K,
            "gbs": nb / (ms * 1e-3) / 1e9, "hbm_frac": nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "locality_order": {"vjp_ms": ms_l, "gbs": nb / (ms_l * 1e-3) / 1e9,
                               "hbm_frac": nb / (ms_l * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def manufactured_case(torch, dev, net, seed, ang=0.03, sigma=1e-4):
    """A solvable case on ``net``: a zero load at every bus without
    injection, a state y* (angles scaled by ``ang``), and loads, PV
    set-points and generator outputs shifted so that F(y*) = 0 (the residual
    from the library); the start is y* plus N(0, sigma) on angles and
    voltages and N(0, 2.5 sigma) on the generator variables."""
    from paper_2011_11880_amd import synth
    from paper_2011_11880_amd.api import Plan
    net = synth.fill_zero_injection_buses(net)
    N, NPV, NG = net.n_bus, net.n_pv, net.n_gen
    ystar = synth.random_states(net, seed=seed)
    ystar[:N] *= ang
    p0 = Plan(net, device=0)
    F0 = p0.eval_residual(torch.from_numpy(ystar).to(dev)).cpu().numpy()
    p0.close()
    has_load = np.zeros(N, bool)
    has_load[net.load_bus] = True
    net.load_p -= F0[net.load_bus]
    net.load_q -= F0[N + net.load_bus]
    pv_free = ~has_load[net.pv_bus]
    net.pv_p[pv_free] += F0[net.pv_bus[pv_free]]
    ystar[2 * N:2 * N + NPV][pv_free] += F0[N + net.pv_bus[pv_free]]
    sl_free = ~has_load[net.slack_bus]
    ystar[2 * N + NG:][sl_free] += F0[net.slack_bus[sl_free]]
    ystar[2 * N + NPV:2 * N + NG][sl_free] += F0[N + net.slack_bus[sl_free]]
    net.pv_v[:] = ystar[N + net.pv_bus]
    net.slack_v[:] = ystar[N + net.slack_bus]
    net.slack_theta[:] = ystar[net.slack_bus]
    rng = np.random.default_rng(seed + 1)
    y0 = ystar + np.concatenate([rng.normal(0, sigma, 2 * N),
                                 rng.normal(0, 2.5 * sigma, net.n_var - 2 * N)])
    return net, ystar, y0


def run_fdlf(args, torch, dev, **kw):
    """Fast decoupled power flow (XB) on a meshed, transmission-like 70,000-bus
    grid (175,000 branches, R/X in 0.05..0.3: the method's domain; on the
    paper-shaped grid it diverges), toward a manufactured solution, against
    device Newton on the same case."""
    from paper_2011_11880_amd import synth
    from paper_2011_11880_amd.api import Plan
    log("[bench] fdlf: meshed 70k grid and manufactured solution")
    net, ystar, y0 = manufactured_case(torch, dev, synth.grid_meshed(70000, 1100), 4200)
    p = Plan(net, device=0)
    x = torch.from_numpy(y0).to(dev)
    log("[bench] fdlf: B', B'' and their factorisations, first solve")
    r0 = p.fdlf(x, tol=1e-10, max_iter=60)   # builds and factorises B', B''
    log("[bench] fdlf: timed solves")
    reps = []
    for _ in range(3):
        x = torch.from_numpy(y0).to(dev)
        reps.append(p.fdlf(x, tol=1e-10, max_iter=60))
    r = min(reps, key=lambda q: q["t_total_s"])
    err = float(np.max(np.abs(x.cpu().numpy() - ystar)))
    it = r["iterations"]
    Bp, Bpp, _, _ = p.fdlf_matrices()
    log("[bench] fdlf: device Newton on the same case (host LU first)")
    xn = torch.from_numpy(y0).to(dev)
    lu = p.device_lu(xn)
    p.newton_device(xn, lu)
    xn = torch.from_numpy(y0).to(dev)
    rn = p.newton_device(xn, lu)
    cpu = None
    if not getattr(args, "no_cpu", False):
        log("[bench] fdlf: the oracle's fast decoupled method on the same case")

        def ora_fdlf(O):
            _, norms, iters = O.fdlf(net, y0, tol=1e-10, max_iter=60)
            return len(iters) - 1, norms[-1]
        cpu = cpu_baseline_solve(ora_fdlf, "the oracle's fast decoupled method (plain-C "
                                 "residuals, scipy LUs of B' and B'' once) on the same case")
    return {"grid": "70,000 buses, 175,000 branches (meshed), R/X 0.05..0.3",
            "cpu_baseline": cpu,
            "n": p.n, "nnz_bp": int(Bp.nnz), "nnz_bpp": int(Bpp.nnz),
            "setup_s": r0["t_setup_s"],
            "fdlf": {"iterations": it, "converged": r["converged"], "final_norm": r["norms"][-1],
                     "max_error_vs_solution": err, "total_ms": r["t_total_s"] * 1e3,
                     "residual_eval_ms_per_iter": r["t_eval_s"] * 1e3 / max(2 * it + 1, 1),
                     "half_steps_ms_per_iter": r["t_solve_s"] * 1e3 / max(it, 1)},
            "newton_device": {"iterations": rn["iterations"], "converged": rn["converged"],
                              "total_ms": rn["t_total_s"] * 1e3,
                              "solve_ms_per_iter": rn["t_solve_s"] * 1e3 / max(rn["iterations"], 1)}}


def run_newton(args, torch, dev, **kw):
    """Newton power flow on the 70,000-bus grid (a zero load added at every
    bus without injection) toward a manufactured solution y*: loads and
    generator set-points chosen so that F(y*) = 0, small angles at y*, start
    within 1e-4 of it.  Every step on the device (evaluation, norm,
    rocSOLVER re-factorisation along one host LU's pattern, triangular
    solves, update) against the same Newton with the host sparse solve."""
    from paper_2011_11880_amd import synth
    from paper_2011_11880_amd.api import Plan
    log("[bench] newton: 70k grid and manufactured solution")
    net, ystar, y0 = manufactured_case(torch, dev, synth.grid_70k(), 4100)
    N, NPV = net.n_bus, net.n_pv
    p = Plan(net, device=0)
    x = torch.from_numpy(y0).to(dev)
    t0 = time.perf_counter()
    lu = p.device_lu(x)
    t_lu = time.perf_counter() - t0
    p.newton_device(x, lu)  # warm-up (first rocSOLVER calls)
    reps = []
    for _ in range(3):
        x = torch.from_numpy(y0).to(dev)
        reps.append(p.newton_device(x, lu))
    rep = min(reps, key=lambda r: r["t_total_s"])
    err = float(np.max(np.abs(x.cpu().numpy() - ystar)))
    # the same Newton on this library's own factorisation (the batched LU
    # with the plan as its one instance)
    log("[bench] newton: device Newton on the library's own factorisation")
    x = torch.from_numpy(y0).to(dev)
    t0 = time.perf_counter()
    olu = p.batch_lu(x)
    t_olu = time.perf_counter() - t0
    p.newton_batch(x, olu, tol=1e-10, max_iter=12)  # warm-up
    oreps = []
    for _ in range(3):
        x = torch.from_numpy(y0).to(dev)
        oreps.append(p.newton_batch(x, olu, tol=1e-10, max_iter=12))
    orep = min(oreps, key=lambda r: r["t_total_s"])
    oerr = float(np.max(np.abs(x.cpu().numpy() - ystar)))
    oit = orep["iterations"]
    olu.close()
    log("[bench] newton: host-solve Newton")
    xh = torch.from_numpy(y0).to(dev)
    reph = p.newton(xh)
    it, ith = rep["iterations"], reph["iterations"]
    # reactive limits: 20 PV units capped 0.002 below their output at y*,
    # solved with the outer switching loop (a fresh host LU after each switch
    # on the device paths) and with the limits checked inside the iterations
    # (host solve; this library's factorisation along pivots that survive a
    # switch, one host LU for the run)
    q = ystar[2 * N:2 * N + NPV]
    pick = np.random.default_rng(4103).choice(NPV, 20, replace=False)
    qmin, qmax = q - 10.0, q + 10.0
    qmax[pick] = q[pick] - 0.002
    log("[bench] newton: with reactive limits")
    pq = Plan(net, device=0, q_limits=True)
    lim = {}
    for name, on_dev, inner in (("device", True, False), ("device_rocsolver", "rocsolver", False),
                                ("host_solve", False, False), ("device_inner", True, True),
                                ("device_rocsolver_inner", "rocsolver", True),
                                ("host_solve_inner", False, True)):
        pq.set_gen_modes(np.zeros(NPV, np.int32))
        x = torch.from_numpy(y0).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = pq.newton_qlim(x, qmin, qmax, device=on_dev, inner=inner,
                           max_iter=30 if inner else 10)
        t1 = time.perf_counter()
        lim[name] = {"converged": r["converged"], "outer_rounds": r["outer"],
                     "held_units": int(pq.gen_modes()[0].sum()),
                     "iterations": [rr["iterations"] for rr in r["rounds"]],
                     "total_ms": (t1 - t0) * 1e3}
        if inner:
            lim[name]["switched_at"] = [k for k, v in enumerate(r["rounds"][0]["switched"]) if v]
    pq.close()
    cpu = None
    if not getattr(args, "no_cpu", False):
        log("[bench] newton: the oracle's Newton on the same case")

        def ora_newton(O):
            _, norms, _ = O.newton(net, y0, tol=1e-10, max_iter=12)
            return len(norms) - 1, norms[-1]
        cpu = cpu_baseline_solve(ora_newton, "the oracle's Newton (plain-C evaluation, "
                                 "scipy SuperLU each iteration) on the same case")
    return {"grid": "70,000 buses, 88,207 branches, zero loads on empty buses",
            "cpu_baseline": cpu,
            "n": p.n, "nnz": p.nnz, "nnz_lu": lu.nnzT, "host_lu_s": t_lu,
            "device": {"iterations": it, "converged": rep["converged"],
                       "final_norm": rep["norms"][-1], "max_error_vs_solution": err,
                       "total_ms": rep["t_total_s"] * 1e3,
                       "eval_ms_per_iter": rep["t_eval_s"] * 1e3 / (it + 1),
                       "solve_ms_per_iter": rep["t_solve_s"] * 1e3 / max(it, 1)},
            "device_own_lu": {"iterations": oit, "converged": orep["n_converged"] == 1,
                              "max_error_vs_solution": oerr, "nnz_lu": orep["nnz_lu"],
                              "host_lu_s": t_olu, "total_ms": orep["t_total_s"] * 1e3,
                              "eval_ms_per_iter": orep["t_eval_s"] * 1e3 / (oit + 1),
                              "solve_ms_per_iter": orep["t_solve_s"] * 1e3 / max(oit, 1)},
            "host_solve": {"iterations": ith, "converged": reph["converged"],
                           "total_ms": reph["t_total_s"] * 1e3,
                           "eval_ms_per_iter": reph["t_eval_s"] * 1e3 / (ith + 1),
                           "solve_ms_per_iter": reph["t_solve_s"] * 1e3 / max(ith, 1)},
            "speedup_total": reph["t_total_s"] / rep["t_total_s"],
            "with_q_limits": lim}


def run_models(args, torch, dev, **kw):
    """Per-model cost on the GPU (the analogue of the paper's Table IV): the
    70k grid rebuilt model by model -- lines and the slack only, then with
    its 40,000 PQ loads, then its 3,500 shunts, then its 10,000 PV units (the
    full grid) -- each evaluated at 1000 states with the same kernels
    (batched launch, and 1000 single-instance launches in a graph).  The
    differences are what each model adds."""
    from paper_2011_11880_amd import synth
    from paper_2011_11880_amd.api import Plan
    full = synth.grid_70k()
    S = 1000
    Y = synth.random_states(full, S, seed=1001)
    N = full.n_bus
    e_i, e_d = np.zeros(0, np.int32), np.zeros(0)

    def variant(loads, shunts, pv):
        v = full.copy()
        if not loads:
            v.load_bus, v.load_p, v.load_q = e_i, e_d, e_d
        if not shunts:
            v.shunt_bus, v.shunt_g, v.shunt_b = e_i, e_d, e_d
        if not pv:
            v.pv_bus, v.pv_p, v.pv_v = e_i, e_d, e_d
        return v

    out = {}
    for name, v in (("line_slack", variant(False, False, False)),
                    ("+pq_loads", variant(True, False, False)),
                    ("+shunts", variant(True, True, False)),
                    ("+pv_units", variant(True, True, True))):
        # states of this variant: theta, V, then the generator variables
        Yv = np.concatenate([Y[:, :2 * N], Y[:, 2 * N + full.n_pv - v.n_pv:]], axis=1)
        bp = Plan(v, batch=dict(n_inst=S, inst_stride=1008), device=0)
        X = torch.from_numpy(np.ascontiguousarray(np.pad(Yv.T, ((0, 0), (0, 8))))).to(dev)
        Fb = torch.empty((bp.n, 1008), dtype=torch.float64, device=dev)
        Jb = torch.empty((bp.nnz, 1008), dtype=torch.float64, device=dev)
        ms_b = time_ms(torch, lambda: bp.eval_batch(X, Fb, Jb))
        del X, Fb, Jb
        pp = Plan(v, device=0)
        Xs = torch.from_numpy(Yv).to(dev)
        Fs = torch.empty((S, pp.n), dtype=torch.float64, device=dev)
        Js = torch.empty((S, pp.nnz), dtype=torch.float64, device=dev)
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        for k in range(S):
            pp.eval(Xs[k], Fs[k], Js[k])
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            with torch.cuda.graph(g, stream=st):
                for k in range(S):
                    pp.eval(Xs[k], Fs[k], Js[k])
        torch.cuda.synchronize()
        ms_p = time_ms(torch, g.replay, reps=5, warmup=1)
        del g, Xs, Fs, Js
        out[name] = {"n": pp.n, "nnz": pp.nnz, "batched_ms_1000": ms_b,
                     "plain_us_per_eval": ms_p * 1e3 / S}
        log("[bench] models", name, json.dumps(out[name]))
    return {"grid": "70,000-bus grid built up model by model, 1000 random states",
            "variants": out}


def run_newton_batch(args, torch, dev, **kw):
    """N-1 contingency analysis on the 10,000-bus grid: 1024 branch outages
    (non-bridges), each a Newton power flow warm-started at the base-case
    solution, all solved together (pf_newton_batch: one batched evaluation
    and one batched factorisation per iteration), against device Newton
    run instance by instance on a sample."""
    from paper_2011_11880_amd import synth
    from paper_2011_11880_amd.api import Plan
    log("[bench] newton batch: 10k grid, base solution, 1024 outages")
    net, ystar, _ = manufactured_case(torch, dev, synth.grid_10k(), 4300, sigma=0.0)
    I = 1024
    out = synth.contingencies(net, I, seed=2002)
    p = Plan(net, batch=dict(n_inst=I, outage=out), device=0)
    X0 = torch.from_numpy(p.to_batch(np.tile(ystar, (I, 1)))).to(dev)
    t0 = time.perf_counter()
    lu = p.batch_lu(X0)
    t_lu = time.perf_counter() - t0
    X = X0.clone()
    p.newton_batch(X, lu, tol=1e-10, max_iter=12)     # warm-up
    reps = []
    for _ in range(3):
        X = X0.clone()
        torch.cuda.synchronize()
        reps.append(p.newton_batch(X, lu, tol=1e-10, max_iter=12))
    r = min(reps, key=lambda q: q["t_total_s"])
    its = r["inst_iterations"]
    it = r["iterations"]
    log("[bench] newton batch: instance by instance on a sample")
    # each sampled outage solved alone on the device, with rocSOLVER's
    # re-factorisation and with this library's (the plan as one instance);
    # setup (host LU) excluded on both sides
    sample = np.linspace(0, I - 1, 16).astype(int)
    t_one, it_one, t_own, it_own = [], [], [], []
    for i in sample:
        v = net.without_branch(int(out[i]))
        q = Plan(v, device=0)
        x = torch.from_numpy(ystar).to(dev)
        luq = q.device_lu(x)
        q.newton_device(x, luq, tol=1e-10, max_iter=12)
        x = torch.from_numpy(ystar).to(dev)
        rq = q.newton_device(x, luq, tol=1e-10, max_iter=12)
        t_one.append(rq["t_total_s"])
        it_one.append(rq["iterations"])
        x = torch.from_numpy(ystar).to(dev)
        luo = q.batch_lu(x)
        q.newton_batch(x, luo, tol=1e-10, max_iter=12)
        x = torch.from_numpy(ystar).to(dev)
        ro = q.newton_batch(x, luo, tol=1e-10, max_iter=12)
        t_own.append(ro["t_total_s"])
        it_own.append(ro["iterations"])
        q.close()
    per_inst_ms = float(np.mean(t_one)) * 1e3
    per_own_ms = float(np.mean(t_own)) * 1e3
    best_ms = min(per_inst_ms, per_own_ms)
    cpu = None
    if not getattr(args, "no_cpu", False):
        log("[bench] newton batch: the oracle's Newton on the sampled outages")
        from oracle import oracle as O
        O.build()
        t_ora, it_ora = [], []
        for i in sample:
            v = net.without_branch(int(out[i]))
            t0 = time.perf_counter()
            _, norms, _ = O.newton(v, ystar, tol=1e-10, max_iter=12)
            t_ora.append(time.perf_counter() - t0)
            it_ora.append(len(norms) - 1)
        cpu = {"mean_ms_per_instance": float(np.mean(t_ora)) * 1e3,
               "extrapolated_total_ms": float(np.mean(t_ora)) * 1e3 * I,
               "mean_iterations": float(np.mean(it_ora)), "cores": 1, "kind": "oracle",
               "sample": f"the oracle's Newton (plain-C evaluation, scipy SuperLU each "
                         f"iteration) on the same {len(sample)} outages"}
    return {"grid": "10,000 buses, 12,500 branches; base case solved, 1024 N-1 outages",
            "instances": I, "nnz_lu": r["nnz_lu"], "host_lu_s": t_lu,
            "batched": {"iterations": it, "n_converged": r["n_converged"],
                        "steps_histogram": np.bincount(its).tolist(),
                        "total_ms": r["t_total_s"] * 1e3,
                        "eval_ms_per_iter": r["t_eval_s"] * 1e3 / (it + 1),
                        "factor_solve_ms_per_iter": r["t_solve_s"] * 1e3 / max(it, 1),
                        "us_per_instance": r["t_total_s"] * 1e6 / I},
            "one_by_one_device_newton": {"sample": len(sample),
                                         "mean_iterations": float(np.mean(it_one)),
                                         "mean_ms_per_instance": per_inst_ms,
                                         "extrapolated_total_ms": per_inst_ms * I},
            "one_by_one_own_factorisation": {"sample": len(sample),
                                             "mean_iterations": float(np.mean(it_own)),
                                             "mean_ms_per_instance": per_own_ms,
                                             "extrapolated_total_ms": per_own_ms * I},
            "cpu_baseline": cpu,
            "speedup": best_ms * I / (r["t_total_s"] * 1e3),
            "speedup_vs_rocsolver_one_by_one": per_inst_ms * I / (r["t_total_s"] * 1e3)}


def run_copy(args, torch, dev):
    """Calibration: a plain device-to-device copy of known size (torch's
    copy kernel), the reference for HBM byte counters; also reports the
    fill (write-only) and sum (read-only) bandwidth of the same buffer as
    practical ceilings."""
    nbytes = args.copy_mib << 20
    a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    with Timer(torch) as t:
        for _ in range(args.steps):
            b.copy_(a)
    ms = t.ms / args.steps
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    fill_ms = time_ms(torch, lambda: b.fill_(1.0))
    sum_ms = time_ms(torch, lambda: a.sum())
    return {"metric": "device copy bandwidth (read + write)", "value": gbs, "unit": "GB/s",
            "fill_gbs": nbytes / (fill_ms * 1e-3) / 1e9,
            "read_gbs": nbytes / (sum_ms * 1e-3) / 1e9,
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": {"workload": f"copy of {args.copy_mib} MiB",
                                            "bytes_read": nbytes, "bytes_written": nbytes}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c1",
                    choices=["c1", "c2", "c3", "c4", "newton", "fdlf", "models", "newton_batch",
                             "copy"])
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--states", type=int, default=1000)
    ap.add_argument("--retune", action="store_true",
                    help="search every schedule again instead of reading the tune cache")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="time the headline launch only (no splits, fill, input-order "
                         "variant or plain launches; for counter runs)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the scenario-batch, uneven-grid, adjoint and Newton summaries")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the evaluation runs on one GPU only; --gpus {args.gpus} is not "
              "supported (batches would shard by instance with no communication)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU available", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    out = {"c1": run_c1, "c2": run_c2, "c3": run_c3, "c4": run_c4, "newton": run_newton,
           "fdlf": run_fdlf, "models": run_models, "newton_batch": run_newton_batch,
           "copy": run_copy}[args.config](args, torch, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
