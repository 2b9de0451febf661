"""28 qubits, batch 1 (2 GiB of complex64 amplitudes): the 6-layer RY/RZ/CNOT-ring
circuit with an angle-embedding layer, forward + readout + adjoint backward of
L = sum_i <Z_i>, against the oracle's values stored in golden/w28_b1_ring.json
(written by golden/make_w28_golden.py, which calls only the oracle; it takes
about 14 minutes of CPU, so the values are stored rather than recomputed).
"""
import json
import os

import numpy as np
import pytest

from paper_2404_09213_amd import inputs as I

from .helpers import AMP_TOL, EXP_TOL, grad_close, gpu_run

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "w28_b1_ring.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_golden_matches_workload_definition():
    """The stored file belongs to the current workload (sizes, seed) and is sane."""
    d = _golden()
    c, batch, seed = I.workload("w28_b1_ring")
    assert (d["workload"], d["seed"], batch) == ("w28_b1_ring", seed, 1)
    assert len(d["expval"]) == c.n_qubits == 28
    assert len(d["grad_weights"]) == c.n_weights
    assert len(d["grad_inputs"]) == c.n_inputs
    assert all(abs(e) <= 1.0 for e in d["expval"])
    amps = np.array(d["amps_re"]) + 1j * np.array(d["amps_im"])
    assert np.all(np.abs(amps) <= 1.0)


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["fused", "fused_tables", "per_gate"])
def test_w28_b1_ring_against_stored_oracle(method):
    import torch
    d = _golden()
    c, batch, seed = I.workload("w28_b1_ring")
    w, x = I.draw_angles(c, batch, seed)
    g = np.ones((batch, c.n_qubits))
    opts = {"fused": {"method": "fused"}, "fused_tables": {"method": "fused", "codegen": 0},
            "per_gate": {"method": "per_gate"}}[method]
    print(f"[w28] method={method}", flush=True)
    got = gpu_run(c, w, x, batch, g, **opts)
    E = got["E"].cpu().numpy()[0]
    assert np.abs(E - np.array(d["expval"])).max() <= EXP_TOL
    idx = torch.tensor(d["amp_indices"], device=got["state"].device)
    amps = got["state"][0].index_select(0, idx).cpu().numpy()
    ref = np.array(d["amps_re"]) + 1j * np.array(d["amps_im"])
    assert np.abs(amps - ref).max() <= AMP_TOL
    ok, rel = grad_close(got["gw"].cpu().numpy(), d["grad_weights"])
    assert ok, ("weights", rel)
    ok, rel = grad_close(got["gx"].cpu().numpy()[0], d["grad_inputs"])
    assert ok, ("inputs", rel)
    del got
    torch.cuda.empty_cache()
