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
    assert L.qsv_pass_copy(pg.handle, 0, 0, 2, fake, fake, 0, None) == -1
    assert b"fused" in L.qsv_last_error()
    p = _plan(c, method="fused", tile_qubits=8)
    info = p.info()
    assert L.qsv_pass_copy(p.handle, 2, 0, 2, fake, fake, 0, None) == -1
    assert L.qsv_pass_copy(p.handle, 0, info["n_fwd_passes"], 2, fake, fake, 0, None) == -1
    assert L.qsv_pass_copy(p.handle, 1, -1, 2, fake, fake, 0, None) == -1
    assert L.qsv_pass_copy(p.handle, 0, 0, 0, fake, fake, 0, None) == -1
    assert L.qsv_pass_copy(p.handle, 0, 1, 2, None, None, 0, None) == -1
    assert L.qsv_pass_copy(p.handle, 1, 1, 2, fake, None, 0, None) == -1  # a backward pass needs lambda
    assert L.qsv_pass_copy(p.handle, 0, 1, 2, fake + 4, None, 0, None) == -1  # misaligned
    assert L.qsv_pass_copy(p.handle, 0, 1, 2, fake, None, 65537, None) == -1  # LDS beyond 64 KiB


CASES = [
    # (name, circuit, options): tiles of 8 and 10 qubits over 12-14-qubit states,
    # with 4 low qubits (16-byte pairs) and with none (single amplitudes)
    ("ring12_t8", lambda: inputs.ry_rz_cnot_ring(12, 3), {"tile_qubits": 8}),
    ("ring14_t10", lambda: inputs.ry_rz_cnot_ring(14, 3), {"tile_qubits": 10}),
    ("ladder13_t9_low0", lambda: inputs.rx_ry_rz_cz_ladder(13, 2), {"tile_qubits": 9, "low_qubits": 0}),
]


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
    assert info["n_bwd_passes"] > 1  # the first backward pass then writes lambda
    for which, count in ((0, info["n_fwd_passes"]), (1, info["n_bwd_passes"])):
        for i in range(count):
            print(f"[pass_copy] {name} which={which} pass={i}", flush=True)
            first = i == 0
            a = (nan if (which == 0 and first) else ref_a).to(dev)
            b = (nan if (which == 1 and first) else ref_b).to(dev)
            p.pass_copy(which, i, B, a, b, lds_bytes=(0, 40960)[i % 2])
            torch.cuda.synchronize()
            a, b = a.cpu(), b.cpu()
            if which == 0 and first:
                assert torch.equal(a, torch.zeros_like(a))
            else:
                assert torch.equal(a, ref_a)
            if which == 1:
                if first:
                    assert torch.equal(b, ref_a)
                else:
                    assert torch.equal(b, ref_b)
            else:
                assert torch.equal(b, ref_b)
