"""qsv_pass_copy: the memory accesses of a fused pass alone (its loads and stores
in a plain copy kernel).

The copy must touch exactly the amplitudes the pass does, through the same
tiles: values read are written back unchanged, the first backward pass writes
its input to both arrays (so every amplitude of lambda is written once, with
the value at the same index of psi), and the first forward pass, which builds
the product state without reading, writes zeros everywhere.
"""
import numpy as np
import pytest

from paper_2404_09213_amd import binding, inputs


def _plan(circ, **opts):
    return binding.Plan(circ.n_qubits, circ.gates, circ.n_weights, circ.n_inputs, **opts)


def test_pass_copy_rejects_bad_calls_before_any_device_work():
    L = binding.lib()
    fake = 256  # never dereferenced: every call below returns before a launch
    c = inputs.ry_rz_cnot_ring(12, 2)
    pg = _plan(c, method="per_gate")
    assert L.qsv_pass_copy(pg.handle, 0, 0, 2, fake, None, 0, 0, None) == -1
    assert b"fused" in L.qsv_last_error()
    p = _plan(c, method="fused", tile_qubits=8)
    info = p.info()
    need = binding.qsv_workspace_size(p.handle, 2, binding.OP_BACKWARD)
    assert L.qsv_pass_copy(p.handle, 2, 0, 2, fake, fake, need, 0, None) == -1
    assert L.qsv_pass_copy(p.handle, 0, info["n_fwd_passes"], 2, fake, None, 0, 0, None) == -1
    assert L.qsv_pass_copy(p.handle, 1, -1, 2, fake, fake, need, 0, None) == -1
    assert L.qsv_pass_copy(p.handle, 0, 0, 0, fake, None, 0, 0, None) == -1
    assert L.qsv_pass_copy(p.handle, 0, 1, 2, None, None, 0, 0, None) == -1
    assert L.qsv_pass_copy(p.handle, 1, 1, 2, fake, None, 0, 0, None) == -1  # a backward pass needs the workspace
    assert L.qsv_pass_copy(p.handle, 1, 1, 2, fake, fake, need - 1, 0, None) == -1
    assert L.qsv_pass_copy(p.handle, 0, 1, 2, fake + 4, None, 0, 0, None) == -1  # misaligned
    assert L.qsv_pass_copy(p.handle, 0, 1, 2, fake, None, 0, 65537, None) == -1  # LDS beyond 64 KiB


CASES = [
    # (name, circuit, options): tiles of 4 to 10 qubits over 9-14-qubit states,
    # with low qubits (16-byte pairs) and with none (single amplitudes)
    ("ring12_t8", lambda: inputs.ry_rz_cnot_ring(12, 3), {"tile_qubits": 8}),
    ("ring14_t10", lambda: inputs.ry_rz_cnot_ring(14, 3), {"tile_qubits": 10}),
    ("ladder13_t9_low0", lambda: inputs.rx_ry_rz_cz_ladder(13, 2), {"tile_qubits": 9, "low_qubits": 0}),
    ("ring9_t4", lambda: inputs.ry_rz_cnot_ring(9, 2), {"tile_qubits": 4, "low_qubits": 1}),
]

# Where qsv_backward keeps psi and lambda in its workspace: psi right after the
# gate matrices (the forward workspace), lambda 4 KiB + 256 bytes past the end of
# psi's 256-byte-aligned extent.
LAMBDA_SKEW = 4096 + 256


@pytest.mark.gpu
@pytest.mark.parametrize("name,make,opts", CASES, ids=[c[0] for c in CASES])
def test_pass_copy_touches_each_amplitude_once(name, make, opts):
    import torch

    dev = torch.device("cuda:0")
    c = make()
    p = _plan(c, method="fused", **opts)
    info = p.info()
    B = 3
    n = 1 << c.n_qubits
    g = torch.Generator().manual_seed(7)
    ref_a = torch.randn((B, n), dtype=torch.complex64, generator=g)
    ref_b = torch.randn((B, n), dtype=torch.complex64, generator=g)
    nan = torch.full((B, n), complex(float("nan"), float("nan")), dtype=torch.complex64)
    ws = p.workspace(B, binding.OP_BACKWARD, dev)
    mats = binding.qsv_workspace_size(p.handle, B, binding.OP_FORWARD)
    nbytes = B * n * 8
    psi = ws[mats:mats + nbytes].view(torch.complex64).view(B, n)
    lo = mats + (nbytes + 255) // 256 * 256 + LAMBDA_SKEW
    lam = ws[lo:lo + nbytes].view(torch.complex64).view(B, n)
    assert info["n_bwd_passes"] > 1  # the first backward pass then writes psi and lambda
    for i in range(info["n_fwd_passes"]):
        print(f"[pass_copy] {name} forward pass {i}", flush=True)
        st = (nan if i == 0 else ref_a).to(dev)
        p.pass_copy(0, i, B, st, lds_bytes=(0, 40960)[i % 2])
        torch.cuda.synchronize()
        assert torch.equal(st.cpu(), torch.zeros_like(ref_a) if i == 0 else ref_a)
    for i in range(info["n_bwd_passes"]):
        print(f"[pass_copy] {name} backward pass {i}", flush=True)
        st = ref_a.to(dev)
        if i == 0:
            psi.copy_(nan.to(dev))
            lam.copy_(nan.to(dev))
        else:
            psi.copy_(ref_a.to(dev))
            lam.copy_(ref_b.to(dev))
        p.pass_copy(1, i, B, st, lds_bytes=(0, 40960)[i % 2])
        torch.cuda.synchronize()
        assert torch.equal(st.cpu(), ref_a)
        assert torch.equal(psi.cpu(), ref_a)
        assert torch.equal(lam.cpu(), ref_a if i == 0 else ref_b)
