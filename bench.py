"""Benchmark: one step = the whole joint-cut HSF hot path on one GPU --
per-path half-state sweeps of both sides for all paths, then the path sum
into every output amplitude -- over a seeded synthetic circuit.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2p] [--mode bf16x3|f32]
    python bench.py --calibrate-copy      # a plain 1 GiB device copy, for counter scaling

Prints one JSON line.  `value` is logical path-gate updates per second of
the whole step (paths x circuit ops of both sides, Schmidt-factor slots
included, divided by the step time) with the chosen path sum (split-BF16
x3); the same step with the plain FP32 path sum ("plain c64 HSF") is timed
beside it.  The path-sum TFLOP/s, the per-phase times, the roofline of the
dominant phase and the FP64 oracle's throughput on the host (bounded sample)
ride along.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK = {"f32": 157.3, "bf16x3": 2500.0, "f64": 78.6}   # TFLOP/s, dense, MI355X datasheet

WORKLOADS = {
    # name: (generator, description)
    "c2p": ("c2p", "n=28 cut 14|14 depth-20 Haar+CZ brickwork, 5 joint blocks of rank 2 (P=32), complex64, "
                   "all 2^28 amplitudes"),
    "c2": ("c2", "n=28 cut 14|14 depth-20 Haar+CZ brickwork, 5 joint blocks of rank 4 (P=1024), complex64, "
                 "all 2^28 amplitudes"),
}


def _src_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2502_06959_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


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


def _traffic_from_profiles(kernel, src_hash, workload):
    """HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE +
    WRITE_SIZE, copy-kernel calibrated), read from profiles/traffic.md if it
    was taken on the current kernel source and this workload; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.md")
    if not os.path.exists(path):
        return None
    head = open(path).readline()
    if not head.strip().endswith(f"workload {workload}"):
        return None
    for line in open(path):
        parts = line.strip().strip("|").split("|")
        parts = [p.strip() for p in parts]
        if len(parts) >= 4 and parts[0] == kernel and parts[1] == src_hash:
            try:
                return float(parts[2])
            except ValueError:
                return None
    return None


def cpu_baseline(circuit, plan_stats, P, na, nb, budget_s=20.0):
    """The FP64 oracle (test infrastructure, untuned) on the host: half-states
    of every path for both sides plus the path sum for a sample of output
    rows, extrapolated to the full step in the same unit as `value`."""
    import numpy as np
    from oracle import hsf as ohsf
    t0 = time.perf_counter()
    o = ohsf.plan(circuit)
    ta = time.perf_counter()
    a = ohsf.half_states(circuit, o, "A")
    b = ohsf.half_states(circuit, o, "B")
    tb = time.perf_counter()
    rows = 1024
    rr = np.arange(rows)
    reps = 0
    tr0 = time.perf_counter()
    while True:
        ohsf.amplitudes_rows(a, b, rr)
        reps += 1
        if time.perf_counter() - tr0 > min(5.0, budget_s / 4):
            break
    t_rows = (time.perf_counter() - tr0) / reps
    t_step = (tb - ta) + t_rows * ((1 << na) / rows)
    logical = P * (plan_stats[0] + plan_stats[1])
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": logical / t_step, "unit": "path-gate updates/s", "cores": cores, "kind": "oracle",
            "sample": (f"oracle plan + half-states of all {P} paths on both sides "
                       f"({tb - ta:.2f} s) + path sum of {rows} of {1 << na} output rows x{reps} "
                       f"({t_rows * 1e3:.1f} ms each), extrapolated to all rows; plan {ta - t0:.3f} s"),
            "step_s_extrapolated": t_step}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2p", choices=sorted(WORKLOADS) + ["c3", "c4", "c5", "qaoa"])
    ap.add_argument("--mode", default="bf16x3", choices=["f32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain FP32 path sum")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--c4-mode", default=None, choices=["f32", "bf16x3", "f64"])
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

    import numpy as np
    import torch

    import circuitgen as cg
    from paper_2502_06959_amd import Plan

    torch.cuda.set_device(0)
    if args.workload == "c5":
        return bench_c5(args)
    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "qaoa":
        return bench_qaoa(args)
    if args.workload == "c3":
        return bench_c3(args)
    gen, desc = WORKLOADS[args.workload]
    circuit = getattr(cg, gen)()
    t0 = time.perf_counter()
    plan = Plan(circuit, dtype="c64", tree=args.tree)
    plan_s = time.perf_counter() - t0
    P, na, nb = plan.P, plan.na, plan.nb
    sa, sb = plan.side_stats(0), plan.side_stats(1)
    A, B = plan.alloc_halves(P)
    out = torch.empty((1 << na, 1 << nb), dtype=torch.complex64, device="cuda")
    sw_ws = _paths_ws(plan, P)

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
            plan.amplitudes_full(A, B, mode=mode, out=out, ws=ws)
            if ev:
                ev[2].record()

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(evs[i])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sweep_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
        sum_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
        rel = None
        if not args.no_check:
            from oracle import hsf as ohsf
            if "oracle" not in cache:
                o = ohsf.plan(circuit)
                cache["oracle"] = (ohsf.half_states(circuit, o, "A"), ohsf.half_states(circuit, o, "B"))
            oa, ob = cache["oracle"]
            rows = np.random.default_rng(7).choice(1 << na, 32, replace=False)
            got = out[torch.from_numpy(rows).to("cuda")].cpu().numpy()
            rel = ohsf.rel_l2(got, ohsf.amplitudes_rows(oa, ob, rows))
        return wall * 1e3 / steps, sweep_ms, sum_ms, rel

    cache = {}
    plain = None
    if not args.no_plain and args.mode != "f32":
        p_ms, p_sw, p_sum, p_rel = run_mode("f32", args.steps, args.warmup)
        plain = {"path_sum": "f32", "ms_per_step": p_ms, "breakdown_ms": {"sweeps": p_sw, "path_sum": p_sum},
                 "rel_l2_sampled_rows": p_rel}
    ms_step, sweep_ms, sum_ms, rel = run_mode(args.mode, args.steps, args.warmup)

    logical_updates = P * (sa["ops_logical"] + sb["ops_logical"])
    flops = 8.0 * (1 << na) * (1 << nb) * P
    value = logical_updates / (ms_step * 1e-3)
    out_bytes = 8.0 * (1 << na) * (1 << nb)
    in_bytes = 8.0 * P * ((1 << na) + (1 << nb))

    # dominant kernel roofline
    if sum_ms >= sweep_ms:
        src = _src_hash("pathsum.hip", "bf16x3.hip", "epilogue.h")
        # the timed path-sum call: one MFMA kernel (FP32), or the split of both
        # operands plus the MFMA kernel (split-BF16 x3)
        many = P >= 64       # LDS-staged kernels from 64 paths on
        if args.mode == "f32":
            kern = "pathsum_f32_lds" if many else "pathsum_f32"
        else:
            kern = "split_chunked x2 + pathsum_bf16x3_lds" if many else "split_planes + pathsum_bf16x3_kernel"
        ach_tf = flops / (sum_ms * 1e-3) / 1e12
        if args.mode == "f32":
            bound, peak, unit, achieved = "mfma", MFMA_PEAK["f32"], "TFLOP/s", ach_tf
        else:
            # split-BF16 x3: 3 real BF16 products per FP32 product; bound by the output write
            t_mfma = 3 * flops / (MFMA_PEAK["bf16x3"] * 1e12)
            t_hbm = (out_bytes + in_bytes) / (HBM_PEAK_GBS * 1e9)
            if t_hbm >= t_mfma:
                bound, peak, unit = "hbm", HBM_PEAK_GBS, "GB/s"
                achieved = (out_bytes + in_bytes) / (sum_ms * 1e-3) / 1e9
            else:
                bound, peak, unit, achieved = "mfma", MFMA_PEAK["bf16x3"], "TFLOP/s", 3 * ach_tf
        traffic = _traffic_from_profiles(kern, src, args.workload)
    else:
        src = _src_hash("sweep.hip")
        kern = "sweep_pass<float> (all passes)"
        # ops are applied on-chip; the bound is the VALU (non-packed FP32:
        # 256 CU x 64 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s); a one-qubit
        # gate costs 14 flop per amplitude
        # ops executed: the per-path ones on every path, the shared prefix once
        ex_a, ex_b = _executed_ops(plan, 0, P), _executed_ops(plan, 1, P)
        fl = 14.0 * ((1 << na) * ex_a + (1 << nb) * ex_b)
        bound, peak, unit = "alu", 78.6, "TFLOP/s"
        achieved = fl / (sweep_ms * 1e-3) / 1e12
        traffic = _traffic_from_profiles(kern, src, args.workload)

    res = {
        "metric": "path-gate updates/s (%HBM peak) + path-sum TFLOP/s; vs plain c64 HSF at rel-L2<=1e-5",
        "value": value, "unit": "path-gate updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 (f32 sweeps, " + ("split-bf16x3" if args.mode == "bf16x3" else "f32") + " path sum)",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "paths": P, "n": plan.n, "cut": f"{nb}|{na}",
                   "path_sum": args.mode, "ops_logical": [sa["ops_logical"], sb["ops_logical"]],
                   "ops_fused": [sa["ops_fused"], sb["ops_fused"]], "sweep": _sweep_desc(plan, P),
                   # fused ops every path starts from (simulated once per plan and device)
                   "ops_shared": [sa["ops_shared"], sb["ops_shared"]]},
        "breakdown_ms": {"sweeps": sweep_ms, "path_sum": sum_ms, "plan_host": plan_s * 1e3},
        "path_sum_tflops": flops / (sum_ms * 1e-3) / 1e12,
        "sweep_updates_per_s": logical_updates / (sweep_ms * 1e-3),
        "sweep_hbm_equiv_pct": 100.0 * logical_updates * 2 * 8 * (1 << max(na, nb)) / (sweep_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "rel_l2_sampled_rows": rel,
        "plain_c64_hsf": None if plain is None else {**plain, "value": logical_updates / (plain["ms_per_step"] * 1e-3),
                                                     "speedup_of_chosen": plain["ms_per_step"] / ms_step},
        "roofline": {"bound": bound, "kernel": kern, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "traffic": traffic},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(circuit, (sa["ops_logical"], sb["ops_logical"]), P, na, nb)
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
    logical = sum(p.P * (p.side_stats(0)["ops_logical"] + p.side_stats(1)["ops_logical"]) for p in plans)

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
    res = {"metric": "path-gate updates/s (batch of 64 circuits)", "value": logical / (ms * 1e-3),
           "unit": "path-gate updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": f"c64 (f32 sweeps, {mode} path sum)", "data": "synthetic",
           "config": {"workload": "c5: 64 circuits, n 20..30, cut near n/2, depth 8..24, CZ/RZZ brick, "
                                  "joint blocks of 1-3 crossing gates, full states",
                      "circuits": len(plans), "paths_total": sum(p.P for p in plans),
                      "output_gib": out_bytes / 2 ** 30, "tuned_policy": pol},
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
    if not args.no_check and os.path.exists(gold):
        z = np.load(gold)
        got = g.cpu().numpy()[z["grad_ids"]]
        err = {"max_abs_over_max_ref": float(np.max(np.abs(got - z["grad"])) / np.max(np.abs(z["grad"]))),
               "loss_rel": float(abs(L - float(z["loss"])) / float(z["loss"])), "grad_ids_checked": int(len(got))}
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


def c4_errors(plan, A, B, tile, mode, rows):
    """Relative L2 error of one row tile in `mode` against the FP64 path sum
    of the same half-states (the path sum's own error), and of the oracle's
    sampled amplitudes that fall in that tile (the whole result's error)."""
    import numpy as np
    import torch

    from paper_2502_06959_amd import hsf_norm2
    g = np.load(os.path.join(ROOT, "tests", "golden", "c4.npz"))
    xs = np.asarray(g["x"], dtype=np.uint64)
    row_of = (xs >> np.uint64(plan.nb)).astype(np.int64)
    r0 = int(row_of[0] // rows) * rows
    sel = np.nonzero((row_of >= r0) & (row_of < r0 + rows))[0]
    plan.amplitudes_full(A, B, rows=(r0, r0 + rows), mode=mode, out=tile)
    o64 = plan.amplitudes_full(A, B, rows=(r0, r0 + rows), mode="f64")
    d = hsf_norm2(tile.reshape(-1), o64.reshape(-1)).cpu().numpy()
    ref = hsf_norm2(o64.reshape(-1)).cpu().numpy()[0]
    del o64
    col = (xs[sel] & np.uint64((1 << plan.nb) - 1)).astype(np.int64)
    idx = torch.from_numpy((row_of[sel] - r0) * (1 << plan.nb) + col).cuda()
    got = tile.reshape(-1)[idx].cpu().numpy().astype(np.complex128)
    want = g["psi"][sel]
    return {"vs_fp64_path_sum_rel_l2": float(np.sqrt(d[1] / ref)),
            "vs_oracle_rel_l2": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
            "oracle_samples": int(len(sel)), "tile_rows": [r0, r0 + rows]}


def bench_c4(args):
    """n=34 (P=4096): sweeps of all paths, then the path sum over every output
    row, streamed in row tiles through one reusable tile buffer, in the
    requested precision (f32, bf16x3 or f64)."""
    import numpy as np
    import torch

    import circuitgen as cg
    from paper_2502_06959_amd import Plan, hsf_workspace_size
    c = cg.c4()
    plan = Plan(c, tree=args.tree)
    A, B = plan.alloc_halves(plan.P)
    rows = 1 << 13
    mode = args.c4_mode or args.mode
    odt = torch.complex128 if mode == "f64" else torch.complex64
    tile = torch.empty((rows, 1 << plan.nb), dtype=odt, device="cuda")
    ws = None
    if mode == "bf16x3":
        ws = torch.empty(hsf_workspace_size(plan.handle, 1, plan.P, 1), dtype=torch.uint8, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    sw_ws = _paths_ws(plan, plan.P)
    plan.run_paths(0, 1, A[:1], B[:1])        # tables to the device, prefix states: set-up, not timed
    torch.cuda.synchronize()
    ev[0].record()
    plan.run_paths(0, plan.P, A, B, ws=sw_ws)
    ev[1].record()
    for r0 in range(0, 1 << plan.na, rows):
        plan.amplitudes_full(A, B, rows=(r0, r0 + rows), mode=mode, out=tile, ws=ws)
    ev[2].record()
    torch.cuda.synchronize()
    sw, ps = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    flops = 8.0 * (1 << plan.na) * (1 << plan.nb) * plan.P
    logical = plan.P * (plan.side_stats(0)["ops_logical"] + plan.side_stats(1)["ops_logical"])
    peak = {"f32": 157.3, "bf16x3": 2500.0 / 3, "f64": 78.6}[mode]
    err = None
    if not args.no_check:
        err = c4_errors(plan, A, B, tile, mode, rows)
    res = {"metric": "path-sum TFLOP/s (n=34, P=4096)", "value": flops / (ps * 1e-3) / 1e12, "unit": "TFLOP/s",
           "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": sw + ps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": mode, "data": "synthetic",
           "config": {"workload": "c4: n=34 cut 17|17 depth-24 Haar+CZ brickwork, 6 joint blocks of rank 4 "
                                  "(P=4096), all 2^34 amplitudes in 2^13-row tiles", "path_sum": mode,
                      "sweep": _sweep_desc(plan, plan.P)},
           "breakdown_ms": {"sweeps": sw, "path_sum": ps},
           "sweep_updates_per_s": logical / (sw * 1e-3),
           "mfma_frac_of_mode_peak": flops / (ps * 1e-3) / 1e12 / peak,
           "mode_peak_tflops": peak, "error": err}
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
        plan.run_paths(p0, p0 + n, A[:n], B[:n], ws=ws)
        plan.amplitudes_full(A[:n], B[:n], n_paths=n, rows=(0, rows), mode=mode, out=out, accumulate=p0 > 0)
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
    for i, (name, sizes, pout, paper_j, paper_log2p) in enumerate(TABLE2):
        c = cg.qaoa_sbm(100 + i, sizes, 0.8, pout)
        t0 = time.perf_counter()
        r = joint_blocked(c)
        pj = Plan(r, tree=args.tree)
        host_ms = (time.perf_counter() - t0) * 1e3
        rows = (10 ** 6 + (1 << pj.nb) - 1) >> pj.nb
        out = torch.empty((rows, 1 << pj.nb), dtype=torch.complex64, device="cuda")
        chunk = min(pj.P, 1 << 14)
        _first_amplitudes(pj, chunk, rows, mode, out)            # warm-up
        j_ms = min(_first_amplitudes(pj, chunk, rows, mode, out) for _ in range(max(1, args.steps // 5)))
        total_j += j_ms
        std = dict(c)
        std["blocks"] = [[k] for k, g in enumerate(c["gates"])
                         if 0 < sum(q <= c["cut"] for q in g["q"]) < len(g["q"])]
        ps = Plan(std, tree=args.tree)
        if ps.P <= (1 << 16):
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
                         "standard_ms": t_ms, "standard_timing": t_kind, "standard_over_joint": t_ms / j_ms,
                         "paper_joint_cpu_s": paper_j, "paper_log2_paths_joint": paper_log2p})
        del out
        torch.cuda.empty_cache()
    res = {"metric": "QAOA first-10^6-amplitude time, 12 Table II shapes (joint cutting)", "value": total_j,
           "unit": "ms (sum over instances)", "n_gpus": 1, "steps": max(1, args.steps // 5), "warmup": 1,
           "ms_per_step": total_j, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": f"c64 (f32 sweeps, {mode} path sum)", "data": "synthetic",
           "config": {"workload": "qaoa: single-layer QAOA MaxCut on seeded SBM graphs, Table II sizes, "
                                  "p_intra 0.8, first 10^6 amplitudes"},
           "instances": rows_out,
           "geomean_standard_over_joint": float(np.exp(np.mean([np.log(x["standard_over_joint"]) for x in rows_out])))}
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

    def run_paths(self, p0, p1, A, B, ws=None):
        return self.plan.run_paths(p0, p1, A, B, ws=ws)

    def amplitudes_full(self, *a, **k):
        return self.plan.amplitudes_full(*a, **k)


if __name__ == "__main__":
    main()
