"""Benchmark: one step = the whole joint-cut HSF hot path on one GPU --
per-path half-state sweeps of both sides for all paths, then the path sum
into every output amplitude -- over a seeded synthetic circuit.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c2p|c2|c3|c5|qaoa]
    python bench.py --calibrate-copy      # a plain 1 GiB device copy, for counter scaling

The default workload is the largest single-GPU configuration: n = 34, cut
17|17, P = 4096 paths, all 2^34 amplitudes (128 GiB of complex64, resident
in HBM) in 16 row tiles of 2^13 rows.  A step sweeps all paths, splits both
operands into BF16 hi/lo planes once, and runs the split-BF16 x3 path sum on
every row tile; the same step with the plain FP32 path sum ("plain c64 HSF")
is timed beside it.

Prints one JSON line.  `value` is executed path-gate updates per second of
the whole step: fused ops applied to half-states as the sweeps run them (the
shared prefix once, each path-tree level once per state), divided by the
step time; logical updates (every path x every circuit op, the count a
per-path simulation does) are reported beside it.  Step times are the mean
over the timed steps, with std and median (the paper reports mean and std
of 5 runs).  The roofline object covers the dominant kernel, timed with HIP
events around each of its launches on the stream it runs on.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK = {"f32": 157.3, "bf16": 2500.0, "f64": 78.6}   # TFLOP/s, dense, MI355X datasheet
METRIC = "path-gate updates/s (%HBM peak) + path-sum TFLOP/s; vs plain c64 HSF at rel-L2\u22641e-5"

WORKLOADS = {
    # name: (generator, description)
    "c2p": ("c2p", "n=28 cut 14|14 depth-20 Haar+CZ brickwork, 5 joint blocks of rank 2 (P=32), complex64, "
                   "all 2^28 amplitudes"),
    "c2": ("c2", "n=28 cut 14|14 depth-20 Haar+CZ brickwork, 5 joint blocks of rank 4 (P=1024), complex64, "
                 "all 2^28 amplitudes"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _src_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2502_06959_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def _stats(xs):
    import numpy as np
    a = np.asarray(xs, dtype=np.float64)
    return {"mean": float(a.mean()), "std": float(a.std(ddof=1)) if len(a) > 1 else 0.0,
            "median": float(np.median(a)), "n": int(len(a))}


def _paths_ws(plan, n_paths):
    """Device workspace of hsf_run_paths over n_paths paths (the path-tree
    levels), or None when the sweep needs none."""
    import torch
    from paper_2502_06959_amd import hsf_workspace_size
    nbytes = hsf_workspace_size(plan.handle, 0, n_paths, 0)
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda") if nbytes else None


def _sweep_desc(plan, n_paths):
    """How the sweeps over n_paths paths run: path tree or flat, tile sizes."""
    tree, tiles = plan.sweep_form(n_paths)
    return {"form": "path tree" if tree else "flat", "tile_qubits": list(tiles)}


def _executed_ops(plan, side, n_paths):
    """Fused ops a sweep over all n_paths paths applies on one side: once per
    state of each path-tree level, or the shared prefix once and every
    per-path op on every path."""
    lv = plan.side_levels(side)
    if plan.sweep_form(n_paths)[0]:
        return sum(o * n for o, n in lv)
    return lv[0][0] + n_paths * sum(o for o, _ in lv[1:])


def _updates(plan):
    """(executed, logical) path-gate updates of one sweep over all paths."""
    ex = _executed_ops(plan, 0, plan.P) + _executed_ops(plan, 1, plan.P)
    lg = plan.P * (plan.side_stats(0)["ops_logical"] + plan.side_stats(1)["ops_logical"])
    return ex, lg


def _traffic_from_profiles(kernel, src_hash, workload):
    """HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE +
    WRITE_SIZE, copy-kernel calibrated), from profiles/traffic.md rows
    `| kernel | workload | source hash | bytes per launch | ...` taken on the
    current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        parts = [p.strip() for p in line.strip().strip("|").split("|")]
        if len(parts) >= 4 and parts[0] == kernel and parts[1] == workload and parts[2] == src_hash:
            try:
                return float(parts[3])
            except ValueError:
                return None
    return None


VALU_PEAK_TFLOPS = 78.6   # non-packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz


def _sweep_work_from_profiles(workload):
    """(HBM bytes, VALU flop) of one step's sweeps, measured with rocprofv3
    counters (profiles/sweeps_c4_qaoa.md rows `| workload | source hash |
    launches | ms | bytes | flop |`) on the current sweep sources; else None."""
    path = os.path.join(ROOT, "profiles", "sweeps_c4_qaoa.md")
    if not os.path.exists(path):
        return None
    src = _src_hash("sweep.hip", "plan.cpp")
    for line in open(path):
        parts = [p.strip() for p in line.strip().strip("|").split("|")]
        if len(parts) >= 6 and parts[0] == workload and parts[1] == src:
            try:
                return float(parts[4]), float(parts[5])
            except ValueError:
                return None
    return None


def _sweep_roofline(workload, sweep_ms):
    """Measured HBM traffic and VALU work of a step's sweeps over the live
    sweep time, as fractions of the HBM and non-packed FP32 VALU peaks; the
    bound named is the one the sweeps come closer to."""
    w = _sweep_work_from_profiles(workload)
    if w is None:
        return None
    nbytes, flop = w
    gbs = nbytes / (sweep_ms * 1e-3) / 1e9
    tfs = flop / (sweep_ms * 1e-3) / 1e12
    hbm_frac, alu_frac = gbs / HBM_PEAK_GBS, tfs / VALU_PEAK_TFLOPS
    return {"kernel": "sweep_pass", "bound": "hbm" if hbm_frac >= alu_frac else "alu",
            "hbm": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_frac, "traffic": nbytes},
            "alu": {"achieved": tfs, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": alu_frac, "flop": flop},
            "sweep_ms": sweep_ms,
            "note": "bytes and flop per step from rocprofv3 counters (profiles/sweeps_c4_qaoa.md), time live"}


def _host():
    """Host CPU model and thread count the oracle runs with."""
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return model, threads


def cpu_baseline(circuit, plan, budget_paths=None, rows=256):
    """The FP64 oracle (test infrastructure, untuned) on the host, on a
    bounded sample of the same workload: half-states of a sample of paths on
    both sides and the path sum of a sample of output rows over those paths,
    extrapolated linearly to all paths and rows (both costs are linear in
    each).  Returns the oracle's own executed path-gate updates per second
    (it runs every op on every path) and its extrapolated step time."""
    import numpy as np
    from oracle import hsf as ohsf
    P, na, nb = plan.P, plan.na, plan.nb
    n_s = min(P, budget_paths or max(1, min(P, (32 << 17) >> max(na, nb))))
    paths = np.linspace(0, P - 1, n_s).round().astype(np.int64)
    t0 = time.perf_counter()
    o = ohsf.plan(circuit)
    ta = time.perf_counter()
    a = ohsf.half_states(circuit, o, "A", paths=paths)
    b = ohsf.half_states(circuit, o, "B", paths=paths)
    tb = time.perf_counter()
    rows = min(rows, 1 << na)
    rr = np.arange(rows)
    reps = 0
    tr0 = time.perf_counter()
    while True:
        ohsf.amplitudes_rows(a, b, rr)
        reps += 1
        if time.perf_counter() - tr0 > 2.0:
            break
    t_rows = (time.perf_counter() - tr0) / reps
    scale = P / n_s
    t_step = (tb - ta) * scale + t_rows * ((1 << na) / rows) * scale
    logical = P * (plan.side_stats(0)["ops_logical"] + plan.side_stats(1)["ops_logical"])
    model, threads = _host()
    return {"value": logical / t_step, "unit": "path-gate updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": model,
            "sample": (f"oracle plan ({ta - t0:.3f} s) + half-states of {n_s} of {P} paths on both sides "
                       f"({tb - ta:.2f} s) + path sum of {rows} of {1 << na} output rows over those paths "
                       f"x{reps} ({t_rows * 1e3:.1f} ms each), extrapolated to all paths and rows; the oracle "
                       f"applies every op to every path, so its updates are the logical count"),
            "step_s_extrapolated": t_step}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS) + ["c3", "c4", "c5", "qaoa"])
    ap.add_argument("--mode", default="bf16x3", choices=["f32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain FP32 path sum")
    ap.add_argument("--plain-steps", type=int, default=None,
                    help="timed steps of the plain FP32 leg (default: all steps, at most 2 on c4)")
    ap.add_argument("--qaoa-instances", default=None,
                    help="comma-separated Table II names (q30-1, ...) to run with --workload qaoa (default: all 12)")
    ap.add_argument("--no-defer", action="store_true",
                    help="qaoa: keep side b's gates after its last factor slot in every path's half-state "
                         "instead of applying them once to the output rows")
    ap.add_argument("--no-standard", action="store_true",
                    help="--workload qaoa: skip the standard-cutting comparison runs")
    ap.add_argument("--no-tune", action="store_true",
                    help="--workload qaoa: keep the planner's sweep tile choice (no timing of 9/10/11-qubit tiles)")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="c2p / c2: also time the whole step replayed from a HIP graph")
    ap.add_argument("--tree", default="auto", choices=["auto", "on", "off"],
                    help="path-tree sweeps (one state per distinct leading-digit prefix)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_each_way": n * 4}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the build targets a single MI355X; multi-GPU path sharding is "
              "described in the design notes but not run. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.workload == "c5":
        return bench_c5(args)
    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "qaoa":
        return bench_qaoa(args)
    if args.workload == "c3":
        return bench_c3(args)
    return bench_full(args)


def _dominant_roofline(kind, kern, src, workload, per_launch, launch_ms):
    """Roofline object of the dominant kernel: `per_launch` algorithmic
    flops (kind mfma-*) or bytes (hbm) of one launch over its average
    event-timed duration."""
    if kind == "hbm":
        achieved = per_launch / (launch_ms * 1e-3) / 1e9
        bound, peak, unit = "hbm", HBM_PEAK_GBS, "GB/s"
    else:
        achieved = per_launch / (launch_ms * 1e-3) / 1e12
        bound, peak, unit = "mfma", MFMA_PEAK[kind.split("-")[1]], "TFLOP/s"
    return {"bound": bound, "kernel": kern, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": _traffic_from_profiles(kern, src, workload),
            "launch_ms": launch_ms, "per_launch": per_launch}


def bench_full(args):
    """c2p / c2: one plan, every output amplitude in one path-sum call."""
    import numpy as np
    import torch

    import circuitgen as cg
    from paper_2502_06959_amd import Plan
    gen, desc = WORKLOADS[args.workload]
    circuit = getattr(cg, gen)()
    t0 = time.perf_counter()
    plan = Plan(circuit, dtype="c64", tree=args.tree)
    plan_s = time.perf_counter() - t0
    P, na, nb = plan.P, plan.na, plan.nb
    A, B = plan.alloc_halves(P)
    out = torch.empty((1 << na, 1 << nb), dtype=torch.complex64, device="cuda")
    sw_ws = _paths_ws(plan, P)
    plan.run_paths(0, 1, A[:1], B[:1])        # tables to the device, prefix states: set-up, not timed
    torch.cuda.synchronize()
    cache = {}

    def run_mode(mode, steps, warmup):
        ws = None
        if mode == "bf16x3":
            from paper_2502_06959_amd import hsf_workspace_size
            ws = torch.empty(hsf_workspace_size(plan.handle, 1, P, 1), dtype=torch.uint8, device="cuda")

        def step(ev=None):
            if ev:
                ev[0].record()
            plan.run_paths(0, P, A, B, ws=sw_ws)
            if ev:
                ev[1].record()
            if mode == "bf16x3":
                plan.split_operands(A, B, ws=ws)
            if ev:
                ev[2].record()
            plan.amplitudes_full(A, B, mode="bf16x3_split" if mode == "bf16x3" else mode, out=out, ws=ws)
            if ev:
                ev[3].record()

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(evs[i])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        r = {"ms_per_step": wall * 1e3 / steps,
             "step_ms": _stats([e[0].elapsed_time(e[3]) for e in evs]),
             "sweeps_ms": _stats([e[0].elapsed_time(e[1]) for e in evs]),
             "split_ms": _stats([e[1].elapsed_time(e[2]) for e in evs]),
             "path_sum_ms": _stats([e[2].elapsed_time(e[3]) for e in evs])}
        if args.graph:
            # the same step captured once and replayed: no host enqueue, the
            # launches back to back on the device
            g = torch.cuda.CUDAGraph()
            cs = torch.cuda.Stream()
            cs.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(cs):
                step()
                torch.cuda.synchronize()
                with torch.cuda.graph(g, stream=cs):
                    step()
            torch.cuda.synchronize()
            for _ in range(warmup):
                g.replay()
            torch.cuda.synchronize()
            ge = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
            t0 = time.perf_counter()
            for i in range(steps):
                ge[i][0].record()
                g.replay()
                ge[i][1].record()
            torch.cuda.synchronize()
            r["graph"] = {"ms_per_step": (time.perf_counter() - t0) * 1e3 / steps,
                          "step_ms": _stats([e[0].elapsed_time(e[1]) for e in ge])}
            del g
        if not args.no_check:
            from oracle import hsf as ohsf
            if "oracle" not in cache:
                o = ohsf.plan(circuit)
                cache["oracle"] = (ohsf.half_states(circuit, o, "A"), ohsf.half_states(circuit, o, "B"))
            oa, ob = cache["oracle"]
            rows = np.random.default_rng(7).choice(1 << na, 32, replace=False)
            got = out[torch.from_numpy(rows).to("cuda")].cpu().numpy()
            r["rel_l2_sampled_rows"] = ohsf.rel_l2(got, ohsf.amplitudes_rows(oa, ob, rows))
        return r

    plain = None
    if not args.no_plain and args.mode != "f32":
        log("plain FP32 path sum")
        plain = run_mode("f32", args.plain_steps or args.steps, args.warmup)
    log(f"{args.mode} path sum")
    res_m = run_mode(args.mode, args.steps, args.warmup)
    ms_step = res_m["ms_per_step"]
    executed, logical = _updates(plan)
    flops = 8.0 * (1 << na) * (1 << nb) * P
    out_bytes = 8.0 * (1 << na) * (1 << nb)
    in_bytes = 8.0 * P * ((1 << na) + (1 << nb))
    sum_ms = res_m["path_sum_ms"]["mean"]
    if args.mode == "f32":
        kern = "pathsum_f32_lds" if P >= 64 else "pathsum_f32"
        roof = _dominant_roofline("mfma-f32", kern, _src_hash("pathsum.hip", "pathsum_lds.hip", "epilogue.h"),
                                  args.workload, flops, sum_ms)
    elif P >= 64:
        roof = _dominant_roofline("mfma-bf16", "pathsum_bf16x3_lds", _src_hash("pathsum_lds.hip", "epilogue.h"),
                                  args.workload, 3 * flops, sum_ms)
    else:
        # few paths: the split-BF16 sum is bound by its output write
        roof = _dominant_roofline("hbm", "pathsum_bf16x3_kernel", _src_hash("bf16x3.hip", "epilogue.h"),
                                  args.workload, out_bytes + in_bytes, sum_ms)
    res = {
        "metric": METRIC, "value": executed / (ms_step * 1e-3), "unit": "path-gate updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 (f32 sweeps, " + ("split-bf16x3" if args.mode == "bf16x3" else "f32") + " path sum)",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "paths": P, "n": plan.n, "cut": f"{nb}|{na}",
                   "path_sum": args.mode, "sweep": _sweep_desc(plan, P)},
        "updates": {"executed": executed, "logical": logical,
                    "logical_per_s": logical / (ms_step * 1e-3),
                    "note": "executed = fused ops applied as the sweeps run them (shared prefix once, each "
                            "path-tree level once per state); logical = every path x every circuit op"},
        "step_ms": res_m["step_ms"], "breakdown_ms": {"sweeps": res_m["sweeps_ms"], "split": res_m["split_ms"],
                                                      "path_sum": res_m["path_sum_ms"], "plan_host": plan_s * 1e3},
        "path_sum_tflops_fp32_equiv": flops / (sum_ms * 1e-3) / 1e12,
        "sweep_executed_updates_per_s": executed / (res_m["sweeps_ms"]["mean"] * 1e-3),
        "rel_l2_sampled_rows": res_m.get("rel_l2_sampled_rows"),
        "graph_replay": res_m.get("graph"),
        "plain_c64_hsf": None if plain is None else {
            "path_sum": "f32", "ms_per_step": plain["ms_per_step"], "step_ms": plain["step_ms"],
            "path_sum_ms": plain["path_sum_ms"], "rel_l2_sampled_rows": plain.get("rel_l2_sampled_rows"),
            "value": executed / (plain["ms_per_step"] * 1e-3), "speedup_of_chosen": plain["ms_per_step"] / ms_step},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline")
        res["cpu_baseline"] = cpu_baseline(circuit, plan)
        res["cpu_baseline"]["gpu_speedup"] = res["cpu_baseline"]["step_s_extrapolated"] / (ms_step * 1e-3)
    print(json.dumps(res), flush=True)


def bench_c5(args):
    """64 independent circuits (n 20..30, uneven cuts, depths and path counts):
    one tuned batch replayed from a HIP graph against per-circuit launches."""
    import numpy as np
    import torch

    import circuitgen as cg
    from paper_2502_06959_amd import Batch, Plan
    cs = cg.c5()
    plans = [Plan(c, tree=args.tree) for c in cs]
    b = Batch(plans)
    outs = b.alloc_outputs()
    mode = args.mode
    pol = b.tune(outs, mode=mode)
    executed = sum(_updates(p)[0] for p in plans)
    logical = sum(_updates(p)[1] for p in plans)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    ms = timed(lambda: b.run(outs, mode=mode, graph=True), args.steps, args.warmup)
    halves = [p.alloc_halves(p.P) for p in plans]
    sws = [_paths_ws(p, p.P) for p in plans]

    def per_circuit():
        for p, (A, B), o, w in zip(plans, halves, outs, sws):
            p.run_paths(0, p.P, A, B, ws=w)
            p.amplitudes_full(A, B, mode="f32", out=o)

    ms_plain = timed(per_circuit, max(1, args.steps // 2), 1)
    out_bytes = sum(8.0 * o.numel() for o in outs)
    res = {"metric": "path-gate updates/s (batch of 64 circuits)", "value": executed / (ms * 1e-3),
           "unit": "path-gate updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": f"c64 (f32 sweeps, {mode} path sum)", "data": "synthetic",
           "config": {"workload": "c5: 64 circuits, n 20..30, cut near n/2, depth 8..24, CZ/RZZ brick, "
                                  "joint blocks of 1-3 crossing gates, full states",
                      "circuits": len(plans), "paths_total": sum(p.P for p in plans),
                      "output_gib": out_bytes / 2 ** 30, "tuned_policy": pol},
           "updates": {"executed": executed, "logical": logical, "logical_per_s": logical / (ms * 1e-3)},
           "plain_per_circuit": {"ms_per_step": ms_plain, "path_sum": "f32",
                                 "speedup_of_batch": ms_plain / ms},
           "output_write_gbs": out_bytes / (ms * 1e-3) / 1e9}
    print(json.dumps(res), flush=True)


def bench_c3(args):
    """Gradient of L = sum_j |psi(x_j)|^2 over 1024 bitstrings with respect to
    all 708 angles of the n=30 variational circuit (P=256): one hsf_backward
    call per step, paths in chunks of 256.  The error is taken against the
    oracle's parameter-shift gradients of 16 sampled angles."""
    import numpy as np
    import torch

    import circuitgen as cg
    from paper_2502_06959_amd import Plan
    c = cg.c3()
    plan = Plan(c, tree=args.tree)
    x = torch.from_numpy(np.asarray(cg.c3_bitstrings(), dtype=np.uint64).astype(np.int64)).cuda()
    for _ in range(args.warmup):
        plan.backward(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g = plan.backward(x)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    t0 = time.perf_counter()
    L = plan.loss(x)
    torch.cuda.synchronize()
    ms_loss = (time.perf_counter() - t0) * 1e3
    err = None
    gold = os.path.join(ROOT, "tests", "golden", "c3.npz")
    gold_all = os.path.join(ROOT, "tests", "golden", "c3_grad.npz")
    if not args.no_check and os.path.exists(gold):
        z = np.load(gold)
        got = g.cpu().numpy()
        ref, ids = z["grad"], z["grad_ids"]
        if os.path.exists(gold_all):
            # the oracle's gradient for every angle
            ref, ids = np.load(gold_all)["grad"], np.arange(len(got))
        err = {"max_abs_over_max_ref": float(np.max(np.abs(got[ids] - ref)) / np.max(np.abs(ref))),
               "loss_rel": float(abs(L - float(z["loss"])) / float(z["loss"])), "grad_ids_checked": int(len(ids))}
    sa, sb = plan.side_stats(0), plan.side_stats(1)
    res = {"metric": "gradients/s (all 708 angles, 1024 bitstrings)", "value": 1e3 / ms, "unit": "gradients/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "c64 (f32 sweeps, f64 reductions)", "data": "synthetic",
           "config": {"workload": "c3: n=30 cut 15|15, 12 layers RY/RZ + RZZ brick, 4 blocks of 3 crossing RZZ "
                                  "(P=256), 708 parameters, loss over 1024 bitstrings",
                      "paths": plan.P, "params": plan.n_params, "sweep": _sweep_desc(plan, plan.P),
                      "ops_logical": [sa["ops_logical"], sb["ops_logical"]]},
           "forward_loss_ms": ms_loss, "error_vs_oracle": err}
    print(json.dumps(res), flush=True)


C4_DESC = ("c4: n=34 cut 17|17 depth-24 Haar+CZ brickwork, 6 joint blocks of rank 4 (P=4096), complex64, all 2^34 "
           "amplitudes resident in HBM (128 GiB) as 16 row tiles of 2^13 rows")


def bench_c4(args):
    """n=34, P=4096: sweeps of all paths, the split of both operands, then the
    path sum of every 2^13-row tile into one 2^17 x 2^17 output."""
    import numpy as np
    import torch

    import circuitgen as cg
    from paper_2502_06959_amd import Plan, hsf_norm2, hsf_workspace_size
    c = cg.c4()
    t0 = time.perf_counter()
    plan = Plan(c, tree=args.tree)
    plan_s = time.perf_counter() - t0
    P, na, nb = plan.P, plan.na, plan.nb
    A, B = plan.alloc_halves(P)
    rows = 1 << 13
    tiles = list(range(0, 1 << na, rows))
    log(f"c4: P={P}, allocating the {8 * (1 << (na + nb)) / 2**30:.0f} GiB output")
    out = torch.empty((1 << na, 1 << nb), dtype=torch.complex64, device="cuda")
    ws = torch.empty(hsf_workspace_size(plan.handle, 1, P, 1), dtype=torch.uint8, device="cuda")
    sw_ws = _paths_ws(plan, P)
    plan.run_paths(0, 1, A[:1], B[:1])        # tables to the device, prefix states: set-up, not timed
    torch.cuda.synchronize()
    gold = np.load(os.path.join(ROOT, "tests", "golden", "c4.npz"))
    xs = np.asarray(gold["x"], dtype=np.uint64)
    xs_dev = torch.from_numpy(xs.astype(np.int64)).cuda()

    def run_mode(mode, steps, warmup):
        def step(ev=None):
            if ev:
                ev["s"][0].record()
            plan.run_paths(0, P, A, B, ws=sw_ws)
            if ev:
                ev["s"][1].record()
            if mode == "bf16x3":
                plan.split_operands(A, B, ws=ws)
            if ev:
                ev["s"][2].record()
            for i, r0 in enumerate(tiles):
                if ev:
                    ev["t"][i][0].record()
                if mode == "bf16x3":
                    plan.amplitudes_full(A, B, rows=(r0, r0 + rows), mode="bf16x3_split", out=out[r0:r0 + rows],
                                         ws=ws)
                else:
                    plan.amplitudes_full(A, B, rows=(r0, r0 + rows), mode=mode, out=out[r0:r0 + rows])
                if ev:
                    ev["t"][i][1].record()
            if ev:
                ev["s"][3].record()

        for w in range(warmup):
            step()
            torch.cuda.synchronize()
            log(f"{mode}: warm-up step {w + 1}/{warmup} done")
        mk = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
        evs = [{"s": [mk() for _ in range(4)], "t": [[mk(), mk()] for _ in tiles]} for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(evs[i])
            if i % 5 == 4 or i == steps - 1:
                torch.cuda.synchronize()
                log(f"{mode}: timed step {i + 1}/{steps} done")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        e = lambda a, b: a.elapsed_time(b)  # noqa: E731
        r = {"ms_per_step": wall * 1e3 / steps,
             "step_ms": _stats([e(v["s"][0], v["s"][3]) for v in evs]),
             "sweeps_ms": _stats([e(v["s"][0], v["s"][1]) for v in evs]),
             "split_ms": _stats([e(v["s"][1], v["s"][2]) for v in evs]),
             "path_sum_ms": _stats([e(v["s"][2], v["s"][3]) for v in evs]),
             "tile_launch_ms": _stats([e(t[0], t[1]) for v in evs for t in v["t"]])}
        if not args.no_check:
            # the oracle's sampled amplitudes (rows of every tile) and the
            # norm of all 2^34 amplitudes the step left in HBM
            got = out.reshape(-1)[xs_dev].cpu().numpy().astype(np.complex128)
            r["rel_l2_vs_oracle_samples"] = float(np.linalg.norm(got - gold["psi"]) / np.linalg.norm(gold["psi"]))
            r["oracle_samples"] = int(len(xs))
            r["norm2_all_amplitudes"] = float(hsf_norm2(out.reshape(-1)).cpu().numpy()[0])
        return r

    plain = None
    if not args.no_plain and args.mode != "f32":
        n_plain = args.plain_steps or min(args.steps, 2)
        log(f"plain FP32 path sum: {n_plain} steps")
        plain = run_mode("f32", n_plain, 1 if args.warmup > 0 else 0)
    log(f"{args.mode} path sum: {args.steps} steps after {args.warmup} warm-up")
    res_m = run_mode(args.mode, args.steps, args.warmup)
    sum_err = None
    if not args.no_check:
        # one tile against the FP64 path sum of the same half-states: the
        # error of the path-sum arithmetic alone
        r0 = int((xs[0] >> np.uint64(nb)) // rows) * rows
        o64 = plan.amplitudes_full(A, B, rows=(r0, r0 + rows), mode="f64")
        d = hsf_norm2(out[r0:r0 + rows].reshape(-1), o64.reshape(-1)).cpu().numpy()
        ref = hsf_norm2(o64.reshape(-1)).cpu().numpy()[0]
        del o64
        sum_err = {"rel_l2_vs_fp64_path_sum": float(np.sqrt(d[1] / ref)), "tile_rows": [r0, r0 + rows]}
    ms_step = res_m["ms_per_step"]
    executed, logical = _updates(plan)
    flops = 8.0 * (1 << na) * (1 << nb) * P
    launch_flops = 8.0 * rows * (1 << nb) * P
    if args.mode == "bf16x3":
        # 3 BF16 products per FP32 product (hi.hi + hi.lo + lo.hi)
        roof = _dominant_roofline("mfma-bf16", "pathsum_bf16x3_lds", _src_hash("pathsum_lds.hip", "epilogue.h"),
                                  "c4", 3 * launch_flops, res_m["tile_launch_ms"]["mean"])
    else:
        roof = _dominant_roofline("mfma-f32", "pathsum_f32_lds", _src_hash("pathsum_lds.hip", "epilogue.h"),
                                  "c4", launch_flops, res_m["tile_launch_ms"]["mean"])
    sw_ms = res_m["sweeps_ms"]["mean"]
    res = {
        "metric": METRIC, "value": executed / (ms_step * 1e-3), "unit": "path-gate updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 (f32 sweeps, " + ("split-bf16x3" if args.mode == "bf16x3" else "f32") + " path sum)",
        "data": "synthetic",
        "config": {"workload": C4_DESC, "paths": P, "n": plan.n, "cut": f"{nb}|{na}", "path_sum": args.mode,
                   "row_tile": rows, "sweep": _sweep_desc(plan, P)},
        "updates": {"executed": executed, "logical": logical, "logical_per_s": logical / (ms_step * 1e-3),
                    "note": "executed = fused ops applied as the sweeps run them (shared prefix once, each "
                            "path-tree level once per state); logical = every path x every circuit op"},
        "step_ms": res_m["step_ms"],
        "breakdown_ms": {"sweeps": res_m["sweeps_ms"], "split": res_m["split_ms"], "path_sum": res_m["path_sum_ms"],
                         "path_sum_launch": res_m["tile_launch_ms"], "plan_host": plan_s * 1e3},
        "path_sum_tflops_fp32_equiv": flops / (res_m["path_sum_ms"]["mean"] * 1e-3) / 1e12,
        "sweep_executed_updates_per_s": executed / (sw_ms * 1e-3),
        "sweep_roofline": _sweep_roofline("c4", sw_ms),
        "error": {"vs_oracle_samples": res_m.get("rel_l2_vs_oracle_samples"),
                  "oracle_samples": res_m.get("oracle_samples"),
                  "norm2_all_amplitudes": res_m.get("norm2_all_amplitudes"), "path_sum": sum_err},
        "plain_c64_hsf": None if plain is None else {
            "path_sum": "f32", "steps": plain["step_ms"]["n"], "ms_per_step": plain["ms_per_step"],
            "step_ms": plain["step_ms"], "path_sum_launch_ms": plain["tile_launch_ms"],
            "path_sum_tflops": flops / (plain["path_sum_ms"]["mean"] * 1e-3) / 1e12,
            "frac_of_fp32_mfma_peak": flops / (plain["path_sum_ms"]["mean"] * 1e-3) / 1e12 / MFMA_PEAK["f32"],
            "rel_l2_vs_oracle_samples": plain.get("rel_l2_vs_oracle_samples"),
            "value": executed / (plain["ms_per_step"] * 1e-3), "speedup_of_chosen": plain["ms_per_step"] / ms_step},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a sample)")
        res["cpu_baseline"] = cpu_baseline(c, plan)
        res["cpu_baseline"]["gpu_speedup"] = res["cpu_baseline"]["step_s_extrapolated"] / (ms_step * 1e-3)
    print(json.dumps(res), flush=True)


# Table II shapes (Sec. V): name, community sizes, p_inter (p_intra 0.8), and
# the paper's own joint-cutting time with preprocessing and path count on a
# 16-core CPU (Table I), quoted as context
TABLE2 = [("q30-1", (15, 15), 0.10, 0.618, 11), ("q30-2", (15, 15), 0.15, 1.480, 12),
          ("q30-3", (15, 15), 0.17, 49.003, 17), ("q31-1", (15, 16), 0.10, 0.389, 10),
          ("q31-2", (15, 16), 0.15, 13.874, 15), ("q31-3", (15, 16), 0.17, 6.670, 14),
          ("q32-1", (16, 16), 0.10, 0.848, 11), ("q32-2", (16, 16), 0.11, 1.605, 12),
          ("q32-3", (16, 16), 0.12, 3.219, 13), ("q33-1", (16, 17), 0.10, 7.409, 14),
          ("q33-2", (16, 17), 0.11, 34.042, 16), ("q33-3", (16, 17), 0.12, 16.884, 15)]


def _first_amplitudes(plan, chunk, rows, mode, out):
    """Paths in chunks: sweeps, then the path sum of the first `rows` output
    rows accumulated over the chunks.  Returns device-event milliseconds
    for [p_lo, p_hi) (default all paths)."""
    import torch
    A, B = plan.alloc_halves(chunk)
    ws = _paths_ws(plan, chunk)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for p0 in range(0, plan.P, chunk):
        n = min(chunk, plan.P - p0)
        # side a only where the first `rows` rows are: its last pass runs only their tiles
        plan.run_paths(p0, p0 + n, A[:n], B[:n], ws=ws, rows=(0, rows))
        plan.amplitudes_full(A[:n], B[:n], n_paths=n, rows=(0, rows), mode=mode, out=out, accumulate=p0 > 0)
    # side b's deferred gates, once on the summed rows (no-op without deferral)
    plan.apply_b_suffix(out, rows)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def bench_qaoa(args):
    """Single-layer QAOA MaxCut on seeded SBM graphs of Table II's shapes:
    the first 10^6 amplitudes by joint cutting (cascade blocks from
    hsf_find_blocks) and by standard cutting (every crossing RZZ cut alone).
    Standard cutting with more than 2^16 paths is timed on one chunk of
    paths and scaled by the path count (marked "extrapolated")."""
    import numpy as np
    import torch

    import circuitgen as cg
    from paper_2502_06959_amd import Plan, joint_blocked
    mode = args.mode
    rows_out = []
    total_j = 0.0
    pick = set(args.qaoa_instances.split(",")) if args.qaoa_instances else None
    for i, (name, sizes, pout, paper_j, paper_log2p) in enumerate(TABLE2):
        if pick is not None and name not in pick:
            continue
        c = cg.qaoa_sbm(100 + i, sizes, 0.8, pout)
        t0 = time.perf_counter()
        r = joint_blocked(c)
        pj = Plan(r, tree=args.tree, defer_b_suffix=not args.no_defer)
        host_ms = (time.perf_counter() - t0) * 1e3
        rows = (10 ** 6 + (1 << pj.nb) - 1) >> pj.nb
        out = torch.empty((rows, 1 << pj.nb), dtype=torch.complex64, device="cuda")
        chunk = min(pj.P, 1 << 14)
        tile_choice, tune_ms = 0, 0.0
        if not args.no_tune:
            # tuner: the planner's own sweep tile choice (0) against tiles
            # forced to 9, 10 and 11 qubits, one warm and one timed run each,
            # outside the measured runs below
            t0 = time.perf_counter()
            best = None
            for tq in (0, 9, 10, 11):
                cand = pj if tq == 0 else Plan(r, tree=args.tree, defer_b_suffix=not args.no_defer, tile_qubits=tq)
                _first_amplitudes(cand, chunk, rows, mode, out)
                t_c = _first_amplitudes(cand, chunk, rows, mode, out)
                if best is None or t_c < best[0]:
                    best = (t_c, tq, cand)
            pj, tile_choice = best[2], best[1]
            tune_ms = (time.perf_counter() - t0) * 1e3
        _first_amplitudes(pj, chunk, rows, mode, out)            # warm-up
        j_ms = min(_first_amplitudes(pj, chunk, rows, mode, out) for _ in range(max(1, args.steps // 5)))
        total_j += j_ms
        std = dict(c)
        std["blocks"] = [[k] for k, g in enumerate(c["gates"])
                         if 0 < sum(q <= c["cut"] for q in g["q"]) < len(g["q"])]
        ps = Plan(std, tree=args.tree, defer_b_suffix=not args.no_defer)
        if args.no_standard:
            t_ms, t_kind = float("nan"), "skipped"
        elif ps.P <= (1 << 16):
            t_ms = _first_amplitudes(ps, min(ps.P, 1 << 14), rows, mode, out)
            t_kind = "measured"
        else:
            # one chunk of 2^14 paths, scaled to P_T
            sub = _PathWindow(ps, 1 << 14)
            _first_amplitudes(sub, 1 << 14, rows, mode, out)
            t_ms = _first_amplitudes(sub, 1 << 14, rows, mode, out) * (ps.P / float(1 << 14))
            t_kind = "extrapolated"
        rows_out.append({"circuit": name, "n": c["n"], "two_qubit_gates": c["meta"]["n_edges"],
                         "crossing": c["meta"]["n_cross"], "blocks": len(r["blocks"]),
                         "log2_paths_joint": int(pj.P).bit_length() - 1,
                         "log2_paths_standard": int(ps.P).bit_length() - 1,
                         "joint_ms": j_ms, "joint_host_plan_ms": host_ms,
                         "sweep_tile_qubits": tile_choice or "planner", "tune_ms": tune_ms,
                         "standard_ms": None if args.no_standard else t_ms, "standard_timing": t_kind,
                         "standard_over_joint": None if args.no_standard else t_ms / j_ms,
                         "paper_joint_cpu_s": paper_j, "paper_log2_paths_joint": paper_log2p})
        del out
        torch.cuda.empty_cache()
    res = {"metric": "QAOA first-10^6-amplitude time, 12 Table II shapes (joint cutting)", "value": total_j,
           "unit": "ms (sum over instances)", "n_gpus": 1, "steps": max(1, args.steps // 5), "warmup": 1,
           "ms_per_step": total_j, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": f"c64 (f32 sweeps, {mode} path sum)", "data": "synthetic",
           "config": {"workload": "qaoa: single-layer QAOA MaxCut on seeded SBM graphs, Table II sizes, "
                                  "p_intra 0.8, first 10^6 amplitudes",
                      "defer_b_suffix": not args.no_defer,
                      "sweep_tiles": "untuned (planner's estimate)" if args.no_tune else
                                     "tuned per instance: planner's estimate or 9/10/11-qubit tiles, "
                                     "timed before the measured runs; standard cutting untuned"},
           "instances": rows_out,
           "geomean_standard_over_joint": (float(np.exp(np.mean([np.log(x["standard_over_joint"]) for x in rows_out])))
                                           if not args.no_standard else None)}
    print(json.dumps(res), flush=True)


class _PathWindow:
    """The first `count` paths of a plan, seen as a plan of `count` paths."""

    def __init__(self, plan, count):
        self.plan, self.P = plan, count
        self.na, self.nb = plan.na, plan.nb

    def alloc_halves(self, n):
        return self.plan.alloc_halves(n)

    @property
    def handle(self):
        return self.plan.handle

    def run_paths(self, p0, p1, A, B, ws=None, rows=None):
        return self.plan.run_paths(p0, p1, A, B, ws=ws, rows=rows)

    def apply_b_suffix(self, out, rows=None):
        return self.plan.apply_b_suffix(out, rows)

    def amplitudes_full(self, *a, **k):
        return self.plan.amplitudes_full(*a, **k)


if __name__ == "__main__":
    main()
