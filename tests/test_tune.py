"""Cost model (host) and option tuner (device)."""
import itertools
import json

import numpy as np
import pytest

from paper_2404_09213_amd import binding as B
from paper_2404_09213_amd import inputs as I


def _est(plan, batch):
    return B.qsv_plan_estimate(plan.handle, batch, 6500.0, 70.0, 4.0)


def test_estimate_orders_methods_and_scales_with_batch():
    c, batch, _ = I.workload("w20_b64_ladder")
    fused = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs)
    pg = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method="per_gate")
    ef, ep = _est(fused, batch), _est(pg, batch)
    assert 0 < ef < ep
    # the per-gate method moves 16 B per changed amplitude per gate: its
    # estimate is at least those bytes at the assumed rate
    amps = batch * (1 << c.n_qubits)
    assert ep >= 16.0 * amps * 0.25 * len(c.gates) / 6500e3
    # launch cost only: a tiny batch is dominated by it, a big one scales
    assert _est(fused, 2 * batch) > 1.9 * ef - 4.0 * 200
    assert B.qsv_plan_estimate(fused.handle, 1, 1e12, 1e12, 4.0) >= 4.0 * (
        fused.info()["n_fwd_passes"] + fused.info()["n_bwd_passes"])


def test_estimate_rejects_bad_rates():
    c = I.rx_ry_rz_cz_ladder(6, 1)
    p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs)
    for args in [(8, 0.0, 1.0, 1.0), (8, 1.0, -1.0, 1.0), (8, 1.0, 1.0, -1.0), (0, 1.0, 1.0, 1.0)]:
        with pytest.raises(RuntimeError):
            B.qsv_plan_estimate(p.handle, *args)


def test_estimate_multi_is_sum_of_parts_order():
    rng = np.random.default_rng(3)
    cs = [I.random_layers(int(n), 3, rng) for n in (8, 10, 12)]
    mp = B.MultiPlan(cs)
    parts = [B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, codegen=0) for c in cs]
    em = B.qsv_plan_estimate(mp.handle, 1, 6500.0, 70.0, 0.0)
    es = sum(B.qsv_plan_estimate(p.handle, 1, 6500.0, 70.0, 0.0) for p in parts)
    assert em == pytest.approx(es, rel=1e-9)


@pytest.mark.gpu
def test_tune_picks_timed_best_and_caches(tmp_path):
    from paper_2404_09213_amd import tune
    print("tune w12 ladder batch 16", flush=True)
    c = I.rx_ry_rz_cz_ladder(12, 3)
    path = str(tmp_path / "tune.json")
    space = {"fuse_width": [1, 3], "tile_qubits": [10, 12], "low_qubits": [4]}
    r = tune.tune(c, 16, space=space, top=2, steps=2, cache=path)
    assert not r["cached"]
    assert r["ms"] == min(t["ms"] for t in r["timed"])
    assert r["opts"] in [t["opts"] for t in r["timed"]]
    with open(path) as f:
        assert len(json.load(f)) == 1
    r2 = tune.tune(c, 16, space=space, top=2, steps=2, cache=path)
    assert r2["cached"] and r2["opts"] == r["opts"]


def test_per_circuit_choice_never_estimates_worse_than_one_global_choice():
    # The multi estimate without launch costs is the sum over circuits, so
    # choosing each circuit's options by its own estimate can only lower it.
    from paper_2404_09213_amd import tune
    cs = I.uneven_set(24, seed=77)
    space = {"fuse_width": [1, 2, 3], "tile_qubits": [10, 12], "low_qubits": [3, 4], "splitter": [0, 1]}
    per = tune.per_circuit_choice(cs, 1, space, threads=4)
    assert len(per) == len(cs) and all(set(o) == set(space) for o in per)
    mp = B.MultiPlan(cs, per_circuit=per)
    e_per = B.qsv_plan_estimate(mp.handle, 1, tune.HBM_GBS, tune.ALU_TFLOPS, 0.0)
    names = sorted(space)
    for vals in itertools.product(*(space[n] for n in names)):
        o = dict(zip(names, vals))
        mg = B.MultiPlan(cs, **o)
        e = B.qsv_plan_estimate(mg.handle, 1, tune.HBM_GBS, tune.ALU_TFLOPS, 0.0)
        assert e_per <= e * (1 + 1e-12), o


@pytest.mark.gpu
def test_tune_multi_times_a_per_circuit_candidate(tmp_path):
    from paper_2404_09213_amd import tune
    print("tune 12 mixed circuits with a per-circuit candidate", flush=True)
    cs = I.uneven_set(12, seed=78, qmax=14)
    space = {"fuse_width": [1, 2], "tile_qubits": [10, 12], "low_qubits": [4]}
    r = tune.tune(cs, 1, multi=True, space=space, top=1, steps=2, cache=str(tmp_path / "t.json"))
    assert any("per_circuit" in t["opts"] for t in r["timed"])
    assert r["ms"] == min(t["ms"] for t in r["timed"])
