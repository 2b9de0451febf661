#!/usr/bin/env python3
"""Benchmark: forward + readout + adjoint backward of a parameterised circuit.

One step = one pass of the whole hot path over one batch: gate-matrix cache
evaluation, product-state init (angle embedding), every gate of the circuit,
<Z_i> readout, and the adjoint backward giving all weight and input
gradients of L = sum_{b,i} <Z_i>_b. Inputs for every step are generated
beforehand and resident in HBM; each step draws fresh inputs and perturbed
weights (as an optimizer step would), so nothing can be cached across steps.

Default workload: 20 qubits, batch 64, embedding + 10 layers of
[RX, RY, RZ on every qubit; CZ ladder], complex64, fused method. The plain
per-gate method is timed beside it on the same inputs, and the CPU oracle is
timed on a bounded sample.

Prints one JSON line (rank 0, single GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TF = 157.3    # MI355X FP32 vector, TFLOP/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=15)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="w20_b64_ladder")
    ap.add_argument("--per-gate-steps", type=int, default=3)
    ap.add_argument("--cpu-samples", type=int, default=4,
                    help="batch samples the oracle is timed on (0 = skip)")
    ap.add_argument("--fuse-width", type=int, default=None)
    ap.add_argument("--tile-qubits", type=int, default=None)
    ap.add_argument("--low-qubits", type=int, default=None)
    ap.add_argument("--mfma", type=int, choices=range(8), default=None,
                    help="2x2 products on the matrix cores, bits: 1 forward, 2 backward psi, 4 backward lambda")
    ap.add_argument("--bwd-gate-by-gate", type=int, choices=(0, 1), default=None)
    ap.add_argument("--pack-beam", type=int, default=None)
    ap.add_argument("--uneven-steps", type=int, default=15,
                    help="timed steps of the 512-circuit uneven set (0 = skip)")
    ap.add_argument("--pass-copy", type=int, choices=(0, 1), default=1,
                    help="time each generated pass's loads and stores alone (qsv_pass_copy)")
    ap.add_argument("--launch-log", default=None,
                    help="after the per-gate steps, run one more with one profile record per "
                         "launch and write the records (kernel.class, bytes, ms) here as JSON, "
                         "for matching per-dispatch counters to gate classes")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--mode", choices=("bench", "copy"), default="bench",
                    help="copy: time a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.launch_log and args.per_gate_steps <= 0:
        ap.error("--launch-log needs --per-gate-steps > 0")
    return args


def copy_rate(reps=5):
    """A plain device-to-device copy of 1 GiB, `reps` times: read + write bytes
    over the best time, the on-box reference rate for HBM-bound kernels."""
    import torch
    n = 1 << 28  # float32 elements = 1 GiB
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del a, b
    return {"bytes_read": 4 * n, "bytes_written": 4 * n, "ms": [round(x, 4) for x in ms],
            "gbs": round(8 * n / (min(ms) / 1e3) / 1e9, 1)}


def copy_calibration(args):
    """The copy above as its own run: the reference for scaling rocprofv3's
    FETCH_SIZE / WRITE_SIZE to bytes."""
    print(json.dumps(dict(mode="copy", **copy_rate())), flush=True)


def family(name):
    """Per-pass generated kernels (qsv_f<i>, qsv_b<i>) grouped by direction."""
    if re.fullmatch(r"qsv_f\d+", name):
        return "pass_fwd(generated)"
    if re.fullmatch(r"qsv_b\d+", name):
        return "pass_bwd(generated)"
    return name


def families(stats):
    out = {}
    for k, v in stats.items():
        f = out.setdefault(family(k), {"launches": 0, "total_ms": 0.0, "bytes": 0.0, "flops": 0.0})
        for key in f:
            f[key] += v[key]
    return out


def counters_summary(workload, kernel, sha):
    """From the committed counter summary of this workload, if it was taken on
    the same generated source: HBM bytes per launch of `kernel` and the
    per-kernel instruction mix / unit occupancy ({} if absent). Returns
    (traffic or None, source or reason, util)."""
    path = os.path.join(ROOT, "profiles", f"{workload}_counters.md")
    if not os.path.exists(path):
        return None, "no counter summary", {}
    m = re.search(r"```json\s*(\{.*?\})\s*```", open(path).read(), re.S)
    if not m:
        return None, "no json block in counter summary", {}
    d = json.loads(m.group(1))
    if d.get("codegen_sha1") != sha:
        return None, "kernel source changed since the counters were taken", {}
    util = d.get("util", {})
    by = d.get("traffic_by_kernel", {})
    if kernel not in by:
        return None, f"no counters for {kernel}", util
    return by[kernel], os.path.relpath(path, ROOT), util


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def run_steps(plan, ws_inputs, g, state, E, gw, gx, steps, warmup, torch):
    """Warm up, then time `steps` steps without instrumentation (the step time),
    then the same steps again with the library's HIP events around every
    launch (per-kernel durations, algorithmic bytes and flops): the events add
    a few microseconds per launch, which would otherwise count in the step.
    Returns (ms_per_step, per-kernel stats, per-step ms)."""
    B = state.shape[0]
    n = len(ws_inputs)

    def step(r):
        w, x = ws_inputs[r % n]
        plan.forward_expval(w, x, B, state, E)
        plan.backward(w, x, state, g, gw=gw, gx=gx)

    for r in range(warmup):
        step(r)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i, r in enumerate(range(warmup, warmup + steps)):
        step(r)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    total_ms = ev[0].elapsed_time(ev[-1])
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    plan.profile(True)
    plan.profile_read()  # drop anything recorded before
    for r in range(warmup, warmup + steps):
        step(r)
    torch.cuda.synchronize()
    stats = plan.profile_read()
    plan.profile(False)
    return total_ms / steps, stats, step_ms


# LDS reserved per workgroup by the copy measurement: 0, then 6, 5, 4, 3 and 2
# tiles per compute unit (160 KB each)
COPY_LDS = (0, 24576, 32768, 40960, 53248, 65536)


def pass_copies(plan, info, B, state, stats, torch, reps=3):
    """Every generated pass beside a plain copy of its own memory accesses: the
    same loads and stores on the same arrays (the state; psi and lambda in the
    backward workspace) through the same tiles, with no arithmetic
    (qsv_pass_copy), at several residencies (LDS reserved per workgroup), timed
    with events on the stream the passes run on; the fastest residency is kept.
    copy_over_pass near 1 means the pass takes as long as its accesses alone.
    Runs after the timed steps: it overwrites the state and the workspace."""
    stream = torch.cuda.current_stream()
    passes = {}
    for which, count, prefix in ((0, info["n_fwd_passes"], "qsv_f"), (1, info["n_bwd_passes"], "qsv_b")):
        for i in range(count):
            name = f"{prefix}{i}"
            if name not in stats:
                return None  # not the generated kernels (table-driven passes)
            by_lds = []
            for lds in COPY_LDS:
                plan.pass_copy(which, i, B, state, lds)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    plan.pass_copy(which, i, B, state, lds)
                e1.record(stream)
                e1.synchronize()
                by_lds.append(round(e0.elapsed_time(e1) * 1e3 / reps, 1))
            copy_us = min(by_lds)
            pass_us = stats[name]["total_ms"] / stats[name]["launches"] * 1e3
            passes[name] = {"pass_us": round(pass_us, 1), "copy_us": copy_us,
                            "copy_lds": COPY_LDS[by_lds.index(copy_us)], "copy_us_by_lds": by_lds,
                            "copy_over_pass": round(copy_us / pass_us, 4)}
    sum_copy = sum(v["copy_us"] for v in passes.values()) / 1e3
    sum_pass = sum(v["pass_us"] for v in passes.values()) / 1e3
    return {"lds_sweep": list(COPY_LDS), "passes": passes, "copy_ms_per_step": round(sum_copy, 3),
            "pass_ms_per_step": round(sum_pass, 3), "copy_over_pass": round(sum_copy / sum_pass, 4)}


def graph_steps(plan, runs, g, state, E, gw, gx, steps, warmup, torch, binding):
    """The same steps replayed from one captured HIP graph (qsv_graph_create):
    every step copies its fresh weights and inputs into the captured buffers,
    then launches the graph. Returns ms per step and the last step's
    expectations, which must equal the eager step's on the same inputs."""
    dev = state.device
    B = state.shape[0]
    wbuf = torch.empty_like(runs[0][0])
    xbuf = torch.empty_like(runs[0][1])
    Eg = torch.empty_like(E)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    graph = binding.StepGraph(plan, wbuf, xbuf, B, state, Eg, g, gw, gx, stream)
    n = len(runs)
    with torch.cuda.stream(stream):
        for r in range(warmup):
            wbuf.copy_(runs[r % n][0])
            xbuf.copy_(runs[r % n][1])
            graph.launch()
    stream.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        t0.record(stream)
        for r in range(warmup, warmup + steps):
            wbuf.copy_(runs[r % n][0])
            xbuf.copy_(runs[r % n][1])
            graph.launch()
        t1.record(stream)
    stream.synchronize()
    del graph
    return t0.elapsed_time(t1) / steps, Eg


def step_spread(ms_list):
    """Mean, min and standard deviation of per-step times (ms)."""
    import statistics
    return {"mean": round(statistics.fmean(ms_list), 4), "min": round(min(ms_list), 4),
            "std": round(statistics.pstdev(ms_list), 4) if len(ms_list) > 1 else 0.0}


def opts_summary(opts):
    """Tuned options as reported: the option dict, or for options chosen per
    circuit how many circuits took each option set."""
    if "per_circuit" not in opts:
        return opts
    import collections
    cnt = collections.Counter(json.dumps(o, sort_keys=True) for o in opts["per_circuit"])
    return {"per_circuit": [{"opts": json.loads(k), "circuits": n} for k, n in cnt.most_common()]}


def bench_uneven(args, torch, dev, binding, inputs):
    """512 circuits of 8..18 qubits and 2..12 random layers, batch 1 each, in
    one multi-circuit plan: options from the tuner, the whole step (forward +
    readout + adjoint) replayed as one captured HIP graph. Fresh perturbed
    weights every step are copied into the captured buffer inside the timed
    region. Reported beside the main line; not its value."""
    import numpy as np

    from paper_2404_09213_amd import tune
    cs = inputs.uneven_set(512, seed=1004)
    space = {"fuse_width": [1, 2, 3], "tile_qubits": [10, 11, 12], "low_qubits": [3, 4, 5],
             "splitter": [0, 1]}
    tr = tune.tune(cs, 1, multi=True, space=space, top=3, steps=3, log=lambda m: log(args, m))
    t_plan = time.perf_counter()
    plan = binding.MultiPlan(cs, **tr["opts"])
    plan_ms = (time.perf_counter() - t_plan) * 1e3
    n_runs = args.warmup + args.uneven_steps
    runs = []
    for r in range(n_runs):
        ws = [inputs.draw_angles(c, 1, 1004 + i, run=r + 1)[0] for i, c in enumerate(cs)]
        runs.append(torch.from_numpy(np.concatenate(ws).astype(np.float32)).to(dev))
    nw = plan.n_weights
    wbuf = torch.empty(nw, dtype=torch.float32, device=dev)
    xbuf = torch.empty((1, 0), dtype=torch.float32, device=dev)
    state = torch.empty((1, plan.state_len), dtype=torch.complex64, device=dev)
    E = torch.empty((1, plan.n_out), dtype=torch.float64, device=dev)
    g = torch.ones((1, plan.n_out), dtype=torch.float64, device=dev)
    gw = torch.empty(max(nw, 1), dtype=torch.float64, device=dev)
    gx = torch.empty((1, 1), dtype=torch.float64, device=dev)

    # eager, profiled: algorithmic bytes per step and the per-kernel split
    eager = [(w, xbuf) for w in runs]
    ems, stats, _ = run_steps(plan, eager, g, state, E, gw, gx, args.uneven_steps, args.warmup, torch)
    step_bytes = sum(v["bytes"] for v in stats.values()) / args.uneven_steps

    torch.cuda.synchronize()
    stream = torch.cuda.Stream(device=dev)
    graph = binding.StepGraph(plan, wbuf, xbuf, 1, state, E, g, gw, gx, stream)
    with torch.cuda.stream(stream):
        for r in range(args.warmup):
            wbuf.copy_(runs[r])
            graph.launch()
    stream.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        t0.record(stream)
        for r in range(args.warmup, n_runs):
            wbuf.copy_(runs[r])
            graph.launch()
        t1.record(stream)
    stream.synchronize()
    gms = t0.elapsed_time(t1) / args.uneven_steps
    # the last replay against eager calls on the same weights
    st_e, E_e = plan.forward_expval(runs[-1], xbuf, 1)
    torch.cuda.synchronize()
    same = bool(torch.equal(E_e, E))
    del graph
    out = {"circuits": len(cs), "n_qubits": [min(c.n_qubits for c in cs), max(c.n_qubits for c in cs)],
           "n_gates": sum(len(c.gates) for c in cs), "n_weights": nw,
           "evals_per_s": round(len(cs) / (gms / 1e3), 1), "ms_per_step": round(gms, 4),
           "eager_ms_per_step": round(ems, 4),
           "alg_gbs": round(step_bytes / (gms / 1e3) / 1e9, 1),
           "opts": opts_summary(tr["opts"]), "tune_seconds": tr["seconds"], "plan_ms": round(plan_ms, 1),
           "graph_equals_eager": same,
           # per kernel over the profiled steps: time, and algorithmic rates
           "kernels": {k: {"launches": v["launches"], "ms": round(v["total_ms"], 3),
                           "tflops": round(v["flops"] / (v["total_ms"] * 1e9), 2) if v["total_ms"] > 0 else None,
                           "gbs": round(v["bytes"] / (v["total_ms"] * 1e6), 1) if v["total_ms"] > 0 else None}
                       for k, v in stats.items()}}
    log(args, f"[bench] uneven: {out}")
    return out


def main():
    args = parse()
    if args.mode == "copy":
        copy_calibration(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "libqsv runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2404_09213_amd import binding, inputs

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    dev = torch.device("cuda:0")
    circ, B, seed = inputs.workload(args.workload)
    W = circ.n_qubits
    opts = {k: v for k, v in (("fuse_width", args.fuse_width), ("tile_qubits", args.tile_qubits),
                              ("low_qubits", args.low_qubits), ("mfma", args.mfma),
                              ("bwd_gate_by_gate", args.bwd_gate_by_gate),
                              ("pack_beam", args.pack_beam)) if v is not None}
    t_plan = time.perf_counter()
    fused = binding.Plan(W, circ.gates, circ.n_weights, circ.n_inputs, method="fused", **opts)
    plan_ms = (time.perf_counter() - t_plan) * 1e3
    per_gate = binding.Plan(W, circ.gates, circ.n_weights, circ.n_inputs, method="per_gate")
    info = fused.info()
    log(args, f"[bench] {args.workload}: W={W} B={B} gates={len(circ.gates)} plan={info}")

    # inputs for every step, resident on the device before timing
    n_runs = args.warmup + args.steps
    runs = []
    for r in range(n_runs):
        w, x = inputs.draw_angles(circ, B, seed, run=r + 1)
        runs.append((torch.from_numpy(w).to(dev), torch.from_numpy(x).to(dev)))
    g = torch.ones((B, W), dtype=torch.float64, device=dev)   # L = sum_{b,i} <Z_i>
    state = torch.empty((B, 1 << W), dtype=torch.complex64, device=dev)
    E = torch.empty((B, W), dtype=torch.float64, device=dev)
    gw = torch.empty((max(circ.n_weights, 1),), dtype=torch.float64, device=dev)
    gx = torch.empty((B, max(circ.n_inputs, 1)), dtype=torch.float64, device=dev)

    ms, stats, step_ms = run_steps(fused, runs, g, state, E, gw, gx, args.steps, args.warmup, torch)
    spread = step_spread(step_ms)
    E_eager = E.clone()
    gms, E_graph = graph_steps(fused, runs, g, state, E, gw, gx, args.steps, args.warmup, torch, binding)
    graph = {"ms_per_step": round(gms, 4), "evals_per_s": round(B / (gms / 1e3), 2),
             "equals_eager": bool(torch.equal(E_graph, E_eager))}
    log(args, f"[bench] fused, replayed from a HIP graph: {gms:.3f} ms/step")
    copy_gbs = copy_rate()["gbs"]  # on-box reference rate for HBM-bound kernels
    log(args, f"[bench] fused: {ms:.3f} ms/step")
    fam = families(stats)
    for k, v in sorted(list(fam.items()) + [kv for kv in stats.items() if family(kv[0]) != kv[0]],
                       key=lambda kv: -kv[1]["total_ms"]):
        log(args, f"   {k:16s} launches={v['launches']:6d} ms={v['total_ms']:9.3f} "
                  f"GB/s={v['bytes'] / max(v['total_ms'], 1e-9) / 1e6:8.1f} "
                  f"TF/s={v['flops'] / max(v['total_ms'], 1e-9) / 1e9:7.2f}")

    # parity spot check of the last timed step (sample 0) against the oracle
    check = None
    if args.cpu_samples > 0:
        from oracle import oracle as orc
        w_last, x_last = runs[(args.warmup + args.steps - 1) % n_runs]
        w64 = w_last.cpu().numpy().astype(np.float64)
        x64 = x_last.cpu().numpy().astype(np.float64)
        ref_E = orc.expval(W, orc.forward(W, circ.gates, w64, x64[:1], 1))
        check = {"sample": 0, "expval_max_abs_err": float(np.abs(E[:1].cpu().numpy() - ref_E).max())}

    # plain per-gate method on the same inputs
    pg = None
    if args.per_gate_steps > 0:
        pms, pstats, _ = run_steps(per_gate, runs, g, state, E, gw, gx, args.per_gate_steps, 1, torch)
        pbytes = sum(v["bytes"] for v in pstats.values()) / args.per_gate_steps
        pg = {"ms_per_step": round(pms, 3), "evals_per_s": round(B / (pms / 1e3), 2),
              "hbm_gbs": round(pbytes / (pms / 1e3) / 1e9, 1),
              "hbm_frac": round(pbytes / (pms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
              "launches_per_step": int(sum(v["launches"] for v in pstats.values()) // args.per_gate_steps),
              "copy_gbs": copy_gbs,
              # per gate class: algorithmic GB/s, as a fraction of the 8 TB/s peak and of the copy
              "kernels": {k: {"launches": v["launches"], "ms": round(v["total_ms"], 3),
                              "gbs": round(v["bytes"] / (v["total_ms"] / 1e3) / 1e9, 1),
                              "hbm_frac": round(v["bytes"] / (v["total_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                              "copy_frac": round(v["bytes"] / (v["total_ms"] / 1e3) / 1e9 / copy_gbs, 4)}
                          for k, v in sorted(pstats.items()) if v["total_ms"] > 0}}
        log(args, f"[bench] per-gate: {pms:.3f} ms/step  {pg}")
        if args.launch_log:
            w, x = runs[0]
            per_gate.profile(2)
            per_gate.profile_launches()
            per_gate.forward_expval(w, x, B, state, E)
            per_gate.backward(w, x, state, g, gw=gw, gx=gx)
            torch.cuda.synchronize()
            launches = per_gate.profile_launches()
            per_gate.profile(False)
            with open(args.launch_log, "w") as f:
                json.dump({"workload": args.workload, "method": "per_gate", "launches": launches}, f)

    uneven = bench_uneven(args, torch, dev, binding, inputs) if args.uneven_steps > 0 else None
    copies = pass_copies(fused, info, B, state, stats, torch) if args.pass_copy else None

    # roofline of the dominant kernel (largest share of the timed region)
    dom_name, dom = max(stats.items(), key=lambda kv: kv[1]["total_ms"])
    gbs = dom["bytes"] / (dom["total_ms"] / 1e3) / 1e9
    tfs = dom["flops"] / (dom["total_ms"] / 1e3) / 1e12
    hbm_frac, alu_frac = gbs / HBM_PEAK_GBS, tfs / FP32_VECTOR_PEAK_TF
    sha = hashlib.sha1(binding.qsv_plan_codegen_source(fused.handle).encode()).hexdigest()
    traffic, traffic_src, util = counters_summary(args.workload, dom_name, sha)
    dfam = fam[family(dom_name)]
    if hbm_frac >= alu_frac:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(tfs, 3), "peak": FP32_VECTOR_PEAK_TF,
                "unit": "TFLOP/s", "frac": round(alu_frac, 4)}
    roof.update({"kernel": dom_name, "launches": dom["launches"],
                 "avg_launch_ms": round(dom["total_ms"] / dom["launches"], 4),
                 "alg_bytes_per_launch": dom["bytes"] / dom["launches"],
                 "alg_flops_per_launch": dom["flops"] / dom["launches"],
                 "hbm_frac": round(hbm_frac, 4), "alu_frac": round(alu_frac, 4),
                 "family": family(dom_name),
                 "family_ms_per_step": round(dfam["total_ms"] / args.steps, 4),
                 "family_alu_tflops": round(dfam["flops"] / (dfam["total_ms"] / 1e3) / 1e12, 3),
                 "family_hbm_gbs": round(dfam["bytes"] / (dfam["total_ms"] / 1e3) / 1e9, 1),
                 "traffic": None if traffic is None else round(traffic, 1),
                 "traffic_source": traffic_src, "codegen_sha1": sha,
                  # counter-derived, same source hash: vector instructions issued per SIMD
                 # per cycle, and the fraction of cycles the matrix cores were busy
                 "valu_issue": util.get(dom_name, {}).get("valu_issue"),
                 "mfma_busy": util.get(dom_name, {}).get("mfma_busy"),
                 # the same pass's loads and stores alone in a plain copy kernel
                 # (qsv_pass_copy), and that time over the pass's own
                 "copy_ms": None if not copies or dom_name not in copies["passes"] else
                 round(copies["passes"][dom_name]["copy_us"] / 1e3, 4),
                 "copy_over_pass": None if not copies or dom_name not in copies["passes"] else
                 copies["passes"][dom_name]["copy_over_pass"]})
    # the generated kernels that issue matrix instructions (forward 2x2 products),
    # from the same counter summary: matrix instructions per wave, busy fractions,
    # and the matrix-core busy fraction weighted by this run's kernel times
    mc = {k: v for k, v in util.items() if v.get("mfma_insts_per_wave")}
    matrix_cores = None
    if mc:
        wt = {k: stats[k]["total_ms"] for k in mc if k in stats}
        tot = sum(wt.values())
        matrix_cores = {"kernels": mc, "source": traffic_src if traffic is not None else
                        os.path.join("profiles", f"{args.workload}_counters.md"),
                        "mfma_busy_time_weighted": round(sum(mc[k]["mfma_busy"] * w for k, w in wt.items()) / tot, 4)
                        if tot and all("mfma_busy" in mc[k] for k in wt) else None}

    # CPU oracle on a bounded sample of the same workload
    cpu = None
    if args.cpu_samples > 0:
        from oracle import oracle as orc
        ns = min(args.cpu_samples, B)
        w0, x0 = runs[0]
        w64 = w0.cpu().numpy().astype(np.float64)
        x64 = x0.cpu().numpy()[:ns].astype(np.float64)
        threads = len(os.sched_getaffinity(0))
        t = time.perf_counter()
        orc.adjoint(W, circ.gates, w64, x64, ns, np.ones((ns, W)))
        dt = time.perf_counter() - t
        cpu = {"value": round(ns / dt, 4), "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": f"{ns} of {B} samples of the same workload, complex128 forward + adjoint, "
                         f"OMP_NUM_THREADS={os.environ.get('OMP_NUM_THREADS', 'unset')}",
               "seconds": round(dt, 2)}
        log(args, f"[bench] cpu oracle: {cpu}")

    out = {
        "metric": "fwd+adjoint circuit evals/s & HBM GB/s, fused vs per-gate, 20q batch 64",
        "value": round(B / (ms / 1e3), 2),
        "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "step_ms": spread,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic: seeded inputs x~U(-pi,pi), weights~U(0,2pi), fresh per step",
        "config": {"workload": args.workload, "n_qubits": W, "batch": B,
                   "n_gates": len(circ.gates), "n_weights": circ.n_weights,
                   "method": "fused", "fuse_width": info["fuse_width"],
                   "tile_qubits": info["tile_qubits"], "low_qubits": info["low_qubits"],
                   "pack_beam": opts.get("pack_beam", binding.qsv_default_opts().pack_beam),
                   "fwd_passes": info["n_fwd_passes"], "bwd_passes": info["n_bwd_passes"],
                   "plan_ms": round(plan_ms, 2)},
        "per_gate": pg,
        "speedup_fused_vs_per_gate": round(pg["ms_per_step"] / ms, 2) if pg else None,
        # the same steps replayed from one captured HIP graph (fresh inputs copied in)
        "graph": graph,
        # per kernel (and per family of generated pass kernels): algorithmic GB/s,
        # as a fraction of the 8 TB/s peak and of the 1 GiB copy timed in this run
        "copy_gbs": copy_gbs,
        "kernels": {k: {"launches": v["launches"], "ms": round(v["total_ms"], 3),
                        "gbs": round(v["bytes"] / max(v["total_ms"], 1e-9) / 1e6, 1),
                        "hbm_frac": round(v["bytes"] / max(v["total_ms"], 1e-9) / 1e6 / HBM_PEAK_GBS, 4),
                        "copy_frac": round(v["bytes"] / max(v["total_ms"], 1e-9) / 1e6 / copy_gbs, 4)}
                    for k, v in list(fam.items()) + [kv for kv in stats.items()
                                                     if family(kv[0]) != kv[0]]},
        "roofline": roof,
        "pass_copy": copies,
        "matrix_cores": matrix_cores,
        "cpu_baseline": cpu,
        "check": check,
        "uneven": uneven,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
