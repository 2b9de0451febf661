"""Summaries of rocprofv3 CSV output (`-f csv`) for this library's kernels.

    python -m paper_2404_09213_amd.profread stats DIR
        per-kernel calls / total / average duration from *kernel_stats.csv
    python -m paper_2404_09213_amd.profread counters DIR [KERNEL_REGEX]
        per-kernel mean counter value per dispatch from *counter_collection.csv
    python -m paper_2404_09213_amd.profread traffic FETCH_DIR WRITE_DIR COPY_FETCH_DIR \\
            COPY_WRITE_DIR COPY_BYTES KERNEL
        HBM bytes per dispatch of KERNEL from FETCH_SIZE / WRITE_SIZE (KiB per
        dispatch), each scaled by what the same counter reads for a plain
        device copy of COPY_BYTES bytes read and written; prints JSON
    python -m paper_2404_09213_amd.profread traffic_all FETCH_DIR WRITE_DIR COPY_FETCH_DIR \\
            COPY_WRITE_DIR COPY_BYTES KERNEL_REGEX
        the same for every kernel matching KERNEL_REGEX
    python -m paper_2404_09213_amd.profread per_gate FETCH_DIR WRITE_DIR COPY_FETCH_DIR \
            COPY_WRITE_DIR COPY_BYTES LAUNCH_LOG
        HBM bytes of every launch of one per-gate step, matched to the gate
        class of the launch from bench.py's --launch-log file, and summed per
        class against the algorithmic bytes; prints JSON
    python -m paper_2404_09213_amd.profread util SQ_DIR [KERNEL_REGEX]
        per kernel from one SQ + GRBM counter pass: vector and matrix
        instructions per wave, matrix-core busy fraction, vector
        instructions issued per SIMD per cycle and matrix FLOPs (see util());
        prints JSON
"""
from __future__ import annotations

import collections
import csv
import glob
import json
import os
import re
import sys


def _one(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def short(name):
    """Kernel name without its argument list, return type and vector-type
    spelling: 'void k_pg_adj<HIP_vector_type<float, 2u> >(...)' -> 'k_pg_adj<float2>'."""
    n = name.split("(")[0].strip()
    if n.startswith("void "):
        n = n[5:]
    return re.sub(r"HIP_vector_type<(\w+), (\d)u>\s*", r"\1\2", n).replace("> >", ">>").replace(" >", ">")


def kernel_stats(d):
    rows = []
    with open(_one(d, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append({"name": short(r["Name"]), "calls": int(r["Calls"]),
                         "total_us": float(r["TotalDurationNs"]) / 1e3,
                         "avg_us": float(r["AverageNs"]) / 1e3,
                         "percent": float(r["Percentage"])})
    return rows


def counter_means(d, kernel_regex=None):
    """{(kernel, counter): (dispatches, mean value per dispatch)}"""
    agg = collections.defaultdict(list)
    rx = re.compile(kernel_regex) if kernel_regex else None
    with open(_one(d, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            k = short(r["Kernel_Name"])
            if rx and not rx.fullmatch(k):
                continue
            agg[(k, r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in agg.items()}


def _copy_kib(d, counter):
    m = counter_means(d, r"__amd_rocclr_copyBuffer")
    return m[("__amd_rocclr_copyBuffer", counter)][1]


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, kernel):
    fk = counter_means(fetch_dir, re.escape(kernel))[(kernel, "FETCH_SIZE")]
    wk = counter_means(write_dir, re.escape(kernel))[(kernel, "WRITE_SIZE")]
    cf = _copy_kib(copy_fetch_dir, "FETCH_SIZE")
    cw = _copy_kib(copy_write_dir, "WRITE_SIZE")
    fetch_scale = copy_bytes / (cf * 1024.0)
    write_scale = copy_bytes / (cw * 1024.0)
    return {"kernel": kernel, "dispatches": fk[0], "fetch_kib": fk[1], "write_kib": wk[1],
            "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
            "fetch_scale": round(fetch_scale, 4), "write_scale": round(write_scale, 4),
            "traffic_bytes": fk[1] * 1024.0 * fetch_scale + wk[1] * 1024.0 * write_scale}


N_CU = 256          # MI355X compute units
N_SIMD = 4 * N_CU   # four SIMDs per CU
N_XCD = 8           # GRBM_GUI_ACTIVE comes back summed over the eight XCDs


def util(sq_dir, kernel_regex=None):
    """Per-kernel instruction mix and unit occupancy from one counter pass.

    GRBM_GUI_ACTIVE / N_XCD is the dispatch's length in GPU cycles (checked
    against its timestamps: 2.0-2.2 cycles per ns under load), so
      mfma_busy  = SQ_VALU_MFMA_BUSY_CYCLES / (cycles x SIMDs),
      valu_issue = vector (non-matrix) instructions per SIMD per cycle,
    and mfma_flops = SQ_INSTS_VALU_MFMA_MOPS_F32 x 512 (the counter
    definitions' MfmaFlopsF32)."""
    m = counter_means(sq_dir, kernel_regex)
    out = {}
    for k in sorted({k for (k, _) in m}):
        g = lambda c: m.get((k, c), (0, None))[1]
        waves, gui = g("SQ_WAVES"), g("GRBM_GUI_ACTIVE")
        row = {"dispatches": m.get((k, "SQ_WAVES"), (0, 0))[0]}
        if waves:
            for c, name in (("SQ_INSTS_VALU", "valu_insts_per_wave"), ("SQ_INSTS_MFMA", "mfma_insts_per_wave"),
                            ("SQ_INSTS_LDS", "lds_insts_per_wave")):
                if g(c) is not None:
                    row[name] = round(g(c) / waves, 1)
        if gui:
            cyc = gui / N_XCD
            row["cycles"] = round(cyc)
            if g("SQ_VALU_MFMA_BUSY_CYCLES") is not None:
                row["mfma_busy"] = round(g("SQ_VALU_MFMA_BUSY_CYCLES") / (cyc * N_SIMD), 4)
            if g("SQ_INSTS_VALU") is not None:
                row["valu_issue"] = round((g("SQ_INSTS_VALU") - (g("SQ_INSTS_MFMA") or 0)) / (cyc * N_SIMD), 4)
        if g("SQ_INSTS_VALU_MFMA_MOPS_F32") is not None:
            row["mfma_flops"] = g("SQ_INSTS_VALU_MFMA_MOPS_F32") * 512
        out[k] = row
    return out


def traffic_all(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, kernel_regex):
    """traffic() for every kernel matching kernel_regex: {kernel: bytes per dispatch}."""
    fk = counter_means(fetch_dir, kernel_regex)
    wk = counter_means(write_dir, kernel_regex)
    fetch_scale = copy_bytes / (_copy_kib(copy_fetch_dir, "FETCH_SIZE") * 1024.0)
    write_scale = copy_bytes / (_copy_kib(copy_write_dir, "WRITE_SIZE") * 1024.0)
    out = {}
    for (k, c), (n, v) in fk.items():
        if c == "FETCH_SIZE" and (k, "WRITE_SIZE") in wk:
            out[k] = v * 1024.0 * fetch_scale + wk[(k, "WRITE_SIZE")][1] * 1024.0 * write_scale
    return {"fetch_scale": round(fetch_scale, 4), "write_scale": round(write_scale, 4),
            "traffic_by_kernel": {k: round(v, 1) for k, v in sorted(out.items())}}


def dispatches(d, counter):
    """[(short kernel name, value)] of one counter, in dispatch order."""
    rows = []
    with open(_one(d, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                rows.append((int(r["Dispatch_Id"]), short(r["Kernel_Name"]), float(r["Counter_Value"])))
    rows.sort()
    return [(k, v) for _, k, v in rows]


def _base(name):
    """Kernel family of a dispatch or of a library record: 'k_pg_adj_vec',
    'k_pg_adj<float2>' and 'k_pg_adj.sign' all give 'k_pg_adj'."""
    n = name.split(".")[0].split("<")[0]
    return n[:-4] if n.endswith("_vec") else n


def _match_last(disp, want):
    """Index in disp (library kernels only, in order) where the last run of
    the families in want starts."""
    fam = [_base(k) for k, _ in disp]
    n = len(want)
    for i in range(len(fam) - n, -1, -1):
        if fam[i:i + n] == want:
            return i
    raise ValueError("the launch log's kernel sequence does not occur in the counter dispatches")


def per_gate(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, launch_log):
    """Per-launch HBM bytes (FETCH_SIZE, WRITE_SIZE scaled as in traffic())
    of the last per-gate step in the two counter runs, with each launch's gate
    class and algorithmic bytes from the library's per-launch record of the
    same step (bench.py --launch-log), and the per-class sums."""
    with open(launch_log) as f:
        log = json.load(f)["launches"]
    want = [_base(r["name"]) for r in log]
    fetch_scale = copy_bytes / (_copy_kib(copy_fetch_dir, "FETCH_SIZE") * 1024.0)
    write_scale = copy_bytes / (_copy_kib(copy_write_dir, "WRITE_SIZE") * 1024.0)
    runs = []
    for d, c, sc in ((fetch_dir, "FETCH_SIZE", fetch_scale), (write_dir, "WRITE_SIZE", write_scale)):
        disp = [(k, v) for k, v in dispatches(d, c) if k.startswith("k_")]
        i = _match_last(disp, want)
        runs.append([v * 1024.0 * sc for _, v in disp[i:i + len(want)]])
    launches, classes = [], {}
    for r, fb, wb in zip(log, runs[0], runs[1]):
        launches.append({"name": r["name"], "alg_bytes": r["bytes"], "fetch_bytes": round(fb, 1),
                         "write_bytes": round(wb, 1)})
        c = classes.setdefault(r["name"], {"launches": 0, "alg_bytes": 0.0, "fetch_bytes": 0.0,
                                           "write_bytes": 0.0})
        c["launches"] += 1
        c["alg_bytes"] += r["bytes"]
        c["fetch_bytes"] += fb
        c["write_bytes"] += wb
    for c in classes.values():
        c["traffic_over_alg"] = round((c["fetch_bytes"] + c["write_bytes"]) / c["alg_bytes"], 3) \
            if c["alg_bytes"] > 0 else None
    return {"fetch_scale": round(fetch_scale, 4), "write_scale": round(write_scale, 4),
            "classes": dict(sorted(classes.items())), "launches": launches}


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        rows = sorted(kernel_stats(argv[1]), key=lambda r: -r["total_us"])
        print("| kernel | calls | total us | avg us | % |\n|---|---|---|---|---|")
        for r in rows:
            print(f"| {r['name']} | {r['calls']} | {r['total_us']:.1f} | {r['avg_us']:.1f} | "
                  f"{r['percent']:.2f} |")
    elif len(argv) >= 2 and argv[0] == "counters":
        m = counter_means(argv[1], argv[2] if len(argv) > 2 else None)
        print("| kernel | counter | dispatches | mean per dispatch |\n|---|---|---|---|")
        for (k, c), (n, v) in sorted(m.items()):
            print(f"| {k} | {c} | {n} | {v:.6g} |")
    elif len(argv) >= 2 and argv[0] == "util":
        print(json.dumps(util(argv[1], argv[2] if len(argv) > 2 else None), indent=1))
    elif len(argv) == 7 and argv[0] == "traffic_all":
        print(json.dumps(traffic_all(argv[1], argv[2], argv[3], argv[4], float(argv[5]), argv[6]), indent=1))
    elif len(argv) == 7 and argv[0] == "per_gate":
        r = per_gate(argv[1], argv[2], argv[3], argv[4], float(argv[5]), argv[6])
        print(json.dumps({k: v for k, v in r.items() if k != "launches"}, indent=1))
    elif len(argv) == 7 and argv[0] == "traffic":
        print(json.dumps(traffic(argv[1], argv[2], argv[3], argv[4], float(argv[5]), argv[6])))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
