"""Host tests of the rocprofv3 CSV readers (synthetic CSV files) and of the
per-launch profiling mode's argument checks."""
import csv
import json

import pytest

from paper_2404_09213_amd import binding, inputs, profread

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(d, rows, counter):
    d.mkdir()
    with open(d / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, FIELDS)
        w.writeheader()
        # written out of dispatch order: the reader sorts by Dispatch_Id
        for i, (name, v) in reversed(list(enumerate(rows))):
            w.writerow({k: 0 for k in FIELDS} | {"Dispatch_Id": i + 1, "Kernel_Name": name,
                                                 "Counter_Name": counter, "Counter_Value": v})


def test_per_gate_matches_the_last_step_and_scales_by_the_copy(tmp_path):
    copy = "__amd_rocclr_copyBuffer(...)"
    _write(tmp_path / "cf", [(copy, 2048.0)], "FETCH_SIZE")   # 2 MiB counted for 1 MiB read
    _write(tmp_path / "cw", [(copy, 512.0)], "WRITE_SIZE")    # 0.5 MiB counted for 1 MiB written
    step = ["void k_coef(float const*)", "k_pg_apply_vec(HIP_vector_type<float, 2u>*, int)",
            "void k_pg_adj<HIP_vector_type<float, 2u> >(HIP_vector_type<float, 2u>*)",
            "k_pg_adj_vec(HIP_vector_type<float, 2u>*, int)"]
    torch_k = "void at::native::elementwise_kernel<128, 4>(int)"
    fetch = [(torch_k, 1.0)] + [(k, 10.0) for k in step] + [(torch_k, 1.0)] + \
            [(k, 100.0 + i) for i, k in enumerate(step)]
    write = [(k, 20.0) for k in step] + [(torch_k, 3.0)] + [(k, 200.0 + i) for i, k in enumerate(step)]
    _write(tmp_path / "f", fetch, "FETCH_SIZE")
    _write(tmp_path / "w", write, "WRITE_SIZE")
    log = tmp_path / "launches.json"
    names = ["k_coef", "k_pg_apply.sign", "k_pg_adj.1q", "k_pg_adj.1q"]
    with open(log, "w") as f:
        json.dump({"launches": [{"name": n, "bytes": 1000.0, "ms": 0.1, "flops": 0.0} for n in names]}, f)
    r = profread.per_gate(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                          str(tmp_path / "cw"), float(1 << 20), str(log))
    assert r["fetch_scale"] == 0.5 and r["write_scale"] == 2.0
    got = [(x["name"], x["fetch_bytes"], x["write_bytes"]) for x in r["launches"]]
    assert got == [(n, (100.0 + i) * 1024 * 0.5, (200.0 + i) * 1024 * 2.0) for i, n in enumerate(names)]
    adj = r["classes"]["k_pg_adj.1q"]
    assert adj["launches"] == 2 and adj["alg_bytes"] == 2000.0
    assert adj["traffic_over_alg"] == pytest.approx((102 + 103) * 512 / 2000 + (202 + 203) * 2048 / 2000, rel=1e-3)
    # a log whose sequence is absent is an error, not a silent mismatch
    with open(log, "w") as f:
        json.dump({"launches": [{"name": "k_grad_reduce", "bytes": 1.0}]}, f)
    with pytest.raises(ValueError):
        profread.per_gate(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                          str(tmp_path / "cw"), float(1 << 20), str(log))


def test_profile_modes_are_checked():
    c = inputs.rx_ry_rz_cz_ladder(6, 1)
    p = binding.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method="per_gate")
    L = binding.lib()
    assert L.qsv_profile_enable(p.handle, 3) == -1
    assert L.qsv_profile_enable(p.handle, -1) == -1
    p.profile(2)
    assert p.profile_launches() == []   # nothing launched yet
    p.profile(False)


@pytest.mark.gpu
def test_per_launch_records_match_the_totals():
    """Mode 2 gives one record per launch, in launch order, that sums to the
    per-kernel totals of mode 1 for the same step."""
    import collections

    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    c = inputs.rx_ry_rz_cz_ladder(8, 2)
    B = 4
    p = binding.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method="per_gate")
    w, x = inputs.draw_angles(c, B, 5)
    wt = torch.from_numpy(w).to(dev)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    g = torch.ones((B, c.n_qubits), dtype=torch.float64, device=dev)

    def step():
        st, E = p.forward_expval(wt, xt, B)
        p.backward(wt, xt, st, g)
        torch.cuda.synchronize()

    print("[profile] per-gate ladder 8 qubits, batch 4", flush=True)
    step()
    p.profile(True)
    p.profile_read()
    step()
    tot = p.profile_read()
    p.profile(2)
    step()
    recs = p.profile_launches()
    p.profile(False)
    assert recs and recs[0]["name"] == "k_coef"
    per = collections.defaultdict(lambda: [0, 0.0])
    for r in recs:
        per[r["name"]][0] += 1
        per[r["name"]][1] += r["bytes"]
        assert r["ms"] >= 0.0
    assert set(per) == set(tot)
    for k, v in tot.items():
        assert per[k][0] == v["launches"], k
        assert per[k][1] == pytest.approx(v["bytes"], rel=1e-12), k
    # forward gate launches come before every adjoint launch
    names = [r["name"] for r in recs]
    last_fwd = max(i for i, n in enumerate(names) if n.startswith("k_pg_apply"))
    first_adj = min(i for i, n in enumerate(names) if n.startswith("k_pg_adj"))
    assert last_fwd < first_adj
