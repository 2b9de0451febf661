"""The allocation-free forward + readout (qsv_forward_expval_noalloc) against
qsv_forward_expval, through the C ABI.

Both run the same kernels on the same inputs, so states and expectations must
agree bit for bit; the allocation-free call only moves the workspace into the
library's own device array. Two calls in a row, the second with a smaller
batch, check that a call does not depend on what the previous one left there.
"""
import numpy as np
import pytest

from paper_2404_09213_amd import binding, inputs


def _plan(circ, **opts):
    return binding.Plan(circ.n_qubits, circ.gates, circ.n_weights, circ.n_inputs, **opts)


def test_noalloc_rejects_oversized_calls_before_any_device_work():
    # 28 qubits at batch 4: the readout partials alone are 4 x 2^16 x 28 float64
    # (58.7 MB), above the 16 MiB array; the size check comes before any device call
    c = inputs.ry_rz_cnot_ring(28, 1)
    p = _plan(c)
    need = binding.qsv_workspace_size(p.handle, 4, binding.OP_FORWARD_EXPVAL)
    assert need > 16 * 1024 * 1024
    L = binding.lib()
    fake = 256  # never dereferenced: the call must return before touching memory
    rc = L.qsv_forward_expval_noalloc(p.handle, fake, fake, 4, fake, fake, None)
    assert rc == -5  # QSV_ERR_TOO_BIG
    assert b"scratch" in L.qsv_last_error()
    rc = L.qsv_forward_expval_noalloc(p.handle, fake, fake, 0, fake, fake, None)
    assert rc == -1  # batch <= 0
    rc = L.qsv_forward_expval_noalloc(p.handle, fake, fake, 2, None, fake, None)
    assert rc == -1  # null state


CASES = [
    ("ladder_fused", lambda: inputs.rx_ry_rz_cz_ladder(10, 3), {"method": "fused"}),
    ("mixed_fused_small_tiles",
     lambda: inputs.random_mixed(9, 60, np.random.default_rng(31), n_inputs=3, p_input=0.2),
     {"method": "fused", "tile_qubits": 6, "low_qubits": 2}),
    ("ring_tables", lambda: inputs.ry_rz_cnot_ring(8, 2), {"method": "fused", "codegen": 0}),
    ("ring_per_gate", lambda: inputs.ry_rz_cnot_ring(7, 2), {"method": "per_gate"}),
]


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,opts", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_forward_expval(name, make, opts):
    import torch
    dev = torch.device("cuda:0")
    c = make()
    p = _plan(c, **opts)
    for call, batch in enumerate((6, 3)):  # second call smaller than the first
        w, x = inputs.draw_angles(c, batch, 500 + call)
        wt = torch.from_numpy(w).to(dev)
        xt = torch.from_numpy(x).to(dev)
        if call == 0:
            # before any call on this device the plan has no tables: refused
            st = torch.empty((batch, 1 << c.n_qubits), dtype=torch.complex64, device=dev)
            E = torch.empty((batch, c.n_qubits), dtype=torch.float64, device=dev)
            with pytest.raises(binding.QsvError) as ei:
                p.forward_expval_noalloc(wt, xt, batch, st, E)
            assert ei.value.code == -1
        ref_st, ref_E = p.forward_expval(wt, xt, batch)
        st = torch.full((batch, 1 << c.n_qubits), float("nan"), dtype=torch.complex64, device=dev)
        E = torch.full((batch, c.n_qubits), float("nan"), dtype=torch.float64, device=dev)
        p.forward_expval_noalloc(wt, xt, batch, st, E)
        torch.cuda.synchronize()
        assert torch.equal(st, ref_st), f"{name} call {call}: states differ"
        assert torch.equal(E, ref_E), f"{name} call {call}: expectations differ"
