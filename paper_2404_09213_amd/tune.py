"""Choice of fusion width k, tile qubits m, low qubits c and splitter for a circuit.

Section "Circuit Splitting" leaves the block size to the user (it suggests
small widths) and notes that the split is made once, when the circuit is
built. Here the choice is made once per (circuit, batch, device): every
candidate plan is built on the host and ranked by the library's cost model
(qsv_plan_estimate); the best few are then timed on the device (one full
step each: forward + readout + adjoint backward) and the fastest wins. For
many circuits in one plan, one more timed candidate gives every circuit the
options the model ranks best for it alone (qsv_plan_multi_each). Results
are kept in a JSON file (path from the `cache` argument or the QSV_TUNE_CACHE
environment variable) keyed by a hash of the gate lists, the batch and the
device architecture, so later runs skip the timing.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

from . import binding

HBM_GBS = 6500.0      # sustained HBM rate assumed by the cost model, GB/s
ALU_TFLOPS = 70.0     # sustained non-packed float32 rate, TFLOP/s
LAUNCH_US = 4.0       # per kernel launch


def _key(circuits, batch, arch, space):
    h = hashlib.sha1()
    for c in circuits:
        h.update(repr((c.n_qubits, c.n_weights, c.n_inputs, tuple(map(tuple, c.gates)))).encode())
    h.update(repr((int(batch), arch, sorted(space.items()))).encode())
    return h.hexdigest()


def default_space(circuits, multi):
    wmax = max(c.n_qubits for c in circuits)
    mmax = 12 if multi else 14
    tiles = [m for m in range(8, mmax + 1) if m <= max(wmax, 8)]
    return {"fuse_width": [1, 2, 3, 4, 5, 6], "tile_qubits": tiles, "low_qubits": [3, 4, 5, 6],
            "splitter": [0, 1]}


def per_circuit_choice(circuits, batch, space, threads=None):
    """Options of each circuit of a multi-circuit plan by the cost model alone:
    the candidate of `space` with the lowest estimate for a single plan of that
    circuit (launch costs left out: the circuits share their launches).
    Planning runs in the library, outside the interpreter lock, so the
    circuits are spread over a few threads."""
    from concurrent.futures import ThreadPoolExecutor
    names = sorted(space)
    combos = [dict(zip(names, v)) for v in itertools.product(*(space[n] for n in names))]
    combos = [o for o in combos if o.get("low_qubits", 0) < o.get("tile_qubits", 99)]

    def best(c):
        top = None
        seen = set()
        for o in combos:
            # tiles at least as wide as the circuit all clamp to its width
            key = tuple(sorted({**o, "tile_qubits": min(o.get("tile_qubits", 12), c.n_qubits)}.items()))
            if key in seen:
                continue
            seen.add(key)
            p = binding.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method="fused", codegen=0, **o)
            e = binding.qsv_plan_estimate(p.handle, batch, HBM_GBS, ALU_TFLOPS, 0.0)
            del p
            if top is None or e < top[0]:
                top = (e, o)
        return top[1]

    if threads is None:
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(best, circuits))


def _make(circuits, multi, opts):
    if multi:
        return binding.MultiPlan(circuits, **opts)
    c = circuits[0]
    return binding.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, **opts)


def _time_step(plan, batch, steps, torch, dev):
    """Mean milliseconds of one forward + readout + backward with fixed angles."""
    import numpy as np
    rng = np.random.default_rng(0)
    w = torch.from_numpy(rng.uniform(0, 2 * np.pi, plan.n_weights).astype(np.float32)).to(dev)
    x = torch.from_numpy(rng.uniform(-np.pi, np.pi, (batch, plan.n_inputs)).astype(np.float32)).to(dev)
    g = torch.ones((batch, plan.n_out), dtype=torch.float64, device=dev)
    st = plan.forward(w, x, batch)   # first use: tables, generated kernels
    E = plan.expval(st)
    plan.backward(w, x, st, g)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.forward(w, x, batch, st)
        plan.expval(st, E)
        plan.backward(w, x, st, g)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(circuits, batch, *, multi=None, space=None, top=4, steps=3, cache=None, device="cuda:0",
         log=None, per_circuit=True):
    """Pick fuse_width / tile_qubits / low_qubits for `circuits` at `batch`.

    circuits: one Circuit or a list (a list of more than one means a
    multi-circuit plan unless multi=False). For a multi-circuit plan the timed
    candidates also include options chosen per circuit by the model
    (per_circuit_choice; opts = {"per_circuit": [one dict per circuit]}, for
    MultiPlan). Returns a dict with the chosen options ("opts"), the model's
    estimate and the measured step time of every timed candidate ("timed"),
    and whether it came from the cache.
    """
    import torch
    if not isinstance(circuits, (list, tuple)):
        circuits = [circuits]
    if multi is None:
        multi = len(circuits) > 1
    space = space or default_space(circuits, multi)
    dev = torch.device(device)
    arch = torch.cuda.get_device_properties(dev).gcnArchName
    key = _key(circuits, batch, arch, space)
    path = cache or os.environ.get("QSV_TUNE_CACHE")
    db = {}
    if path and os.path.exists(path):
        with open(path) as f:
            db = json.load(f)
        if key in db:
            out = dict(db[key])
            out["cached"] = True
            return out

    t0 = time.perf_counter()
    ranked = []
    seen = set()
    names = sorted(space)
    for vals in itertools.product(*(space[n] for n in names)):
        opts = dict(zip(names, vals))
        if opts.get("low_qubits", 0) >= opts.get("tile_qubits", 99):
            continue
        plan = _make(circuits, multi, opts)
        info = plan.info()
        # options that lead to the same schedule (tile clamped to the width, ...)
        sig = (info["fuse_width"], info["tile_qubits"], info["low_qubits"], info["n_fwd_passes"],
               info["n_bwd_passes"], info["n_fwd_stages"], info["n_bwd_stages"], info["n_blocks"],
               opts.get("splitter", 0))
        if sig in seen:
            continue
        seen.add(sig)
        est = binding.qsv_plan_estimate(plan.handle, batch, HBM_GBS, ALU_TFLOPS, LAUNCH_US)
        ranked.append((est, opts))
        del plan
    ranked.sort(key=lambda r: r[0])
    host_s = time.perf_counter() - t0
    # the library defaults are always among the timed candidates
    d = binding.qsv_default_opts()
    dflt = {n: getattr(d, n) for n in names}
    pick = ranked[:max(1, top)]
    if all(o != dflt for _, o in pick):
        plan = _make(circuits, multi, dflt)
        pick.append((binding.qsv_plan_estimate(plan.handle, batch, HBM_GBS, ALU_TFLOPS, LAUNCH_US), dflt))
        del plan
    if multi and per_circuit:
        # one more candidate: every circuit with the options the model ranks best
        # for it, at the widest tile of the space (the multi-circuit kernels run
        # 256 threads per item whatever the tile, so narrower tiles leave lanes idle)
        t1 = time.perf_counter()
        pc_space = dict(space)
        if "tile_qubits" in pc_space:
            pc_space["tile_qubits"] = [max(pc_space["tile_qubits"])]
        opts = {"per_circuit": per_circuit_choice(circuits, batch, pc_space)}
        plan = _make(circuits, multi, opts)
        pick.append((binding.qsv_plan_estimate(plan.handle, batch, HBM_GBS, ALU_TFLOPS, LAUNCH_US), opts))
        del plan
        host_s += time.perf_counter() - t1

    timed = []
    for est, opts in pick:
        plan = _make(circuits, multi, opts)
        ms = _time_step(plan, batch, steps, torch, dev)
        timed.append({"opts": opts, "est_ms": round(est / 1e3, 4), "ms": round(ms, 4)})
        if log:
            shown = "per circuit" if "per_circuit" in opts else opts
            log(f"[tune] {shown} est={est / 1e3:.3f} ms measured={ms:.3f} ms")
        del plan
    best = min(timed, key=lambda r: r["ms"])
    out = {"opts": best["opts"], "ms": best["ms"], "timed": timed, "n_candidates": len(ranked),
           "host_seconds": round(host_s, 2), "seconds": round(time.perf_counter() - t0, 2),
           "arch": arch, "batch": int(batch)}
    if path:
        db[key] = out
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, path)
    out = dict(out)
    out["cached"] = False
    return out
