"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Amplitudes and <Z_i> within 1e-5 max-abs; gradients within 1e-4 relative
(normwise and per entry with a floor, see helpers.grad_close). Both methods
(fused tiles and the plain per-gate method) and several tile shapes.
"""
import math

import numpy as np
import pytest
import torch  # noqa: F401  (import once at collection, outside per-test time limits)

from paper_2404_09213_amd import inputs as I

from .helpers import AMP_TOL, EXP_TOL, grad_close, gpu_run, oracle_run

pytestmark = pytest.mark.gpu

# fused = generated per-plan kernels; fused_tables = table-driven kernels; per_gate = plain
# method; fused_gbg = generated kernels with the backward uncomputing gate by gate (no
# 1-qubit chain products) and every 2x2 on the vector ALU (no matrix cores)
METHODS = ["fused", "fused_tables", "per_gate", "fused_gbg"]
_METHOD_OPTS = {"fused": {"method": "fused", "codegen": 1},
                "fused_tables": {"method": "fused", "codegen": 0},
                "per_gate": {"method": "per_gate"},
                "fused_gbg": {"method": "fused", "codegen": 1, "bwd_gate_by_gate": 1, "mfma": 0}}


def _opts(method, **extra):
    o = dict(_METHOD_OPTS[method])
    o.update(extra)
    return o


def _check(circ, batch, seed, orc, method, grads=True, **opts):
    w, x = I.draw_angles(circ, batch, seed)
    g = I.draw_grad_out(circ, batch, seed) if grads else None
    print(f"[parity] {circ.name} B={batch} seed={seed} method={method} opts={opts}", flush=True)
    got = gpu_run(circ, w, x, batch, g, **_opts(method, **opts))
    ref = oracle_run(orc, circ, w, x, batch, g)
    amp = np.abs(got["state"].cpu().numpy() - ref["state"]).max()
    e = np.abs(got["E"].cpu().numpy() - ref["E"]).max()
    e2 = np.abs(got["E_fused"].cpu().numpy() - ref["E"]).max()
    assert amp <= AMP_TOL, amp
    assert e <= EXP_TOL, e
    assert e2 <= EXP_TOL, ("forward_expval", e2)
    if grads:
        ok, rel = grad_close(got["gw"].cpu().numpy(), ref["gw"])
        assert ok, ("weights", rel)
        if circ.n_inputs:
            ok, rel = grad_close(got["gx"].cpu().numpy(), ref["gx"])
            assert ok, ("inputs", rel)
    return got, ref


@pytest.mark.parametrize("method", METHODS)
def test_bell_and_ghz(orc, method):
    for W in (2, 3, 6, 13):
        c = I.Circuit(W, name=f"ghz{W}")
        c.fixed("H", 0)
        for q in range(W - 1):
            c.fixed("CNOT", q, q + 1)
        got = gpu_run(c, np.zeros(0, np.float32), np.zeros((1, 0), np.float32), 1, **_opts(method))
        st = got["state"].cpu().numpy()[0]
        r = 1 / math.sqrt(2)
        assert abs(st[0] - r) < 1e-6 and abs(st[-1] - r) < 1e-6
        assert np.abs(st[1:-1]).max() < 1e-7
        assert np.abs(got["E"].cpu().numpy()).max() < 1e-6


@pytest.mark.parametrize("method", METHODS)
def test_small_workload_w6_b8(orc, method):
    c, batch, seed = I.workload("w6_b8_ring")
    _check(c, batch, seed, orc, method)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("W,ng,seed", [(1, 20, 1), (2, 40, 2), (3, 60, 3), (4, 80, 4), (5, 90, 5),
                                       (7, 120, 6), (9, 150, 7), (11, 150, 8), (13, 120, 9)])
def test_random_mixed(orc, method, W, ng, seed):
    rng = np.random.default_rng(seed)
    c = I.random_mixed(W, ng, rng, n_inputs=3, p_input=0.2)
    _check(c, 3, seed, orc, method)


@pytest.mark.parametrize("method", ["fused", "fused_tables"])
@pytest.mark.parametrize("k,m,cq", [(2, 4, 0), (3, 5, 1), (4, 6, 2), (5, 8, 3), (6, 9, 4),
                                    (5, 10, 5), (3, 11, 6), (5, 12, 5), (1, 12, 11), (16, 12, 0)])
def test_fused_tile_shapes(orc, method, k, m, cq):
    rng = np.random.default_rng(100 + m)
    c = I.random_mixed(13, 160, rng, n_inputs=4, p_input=0.2)
    _check(c, 2, 100 + m, orc, method, fuse_width=k, tile_qubits=m, low_qubits=cq)


@pytest.mark.parametrize("k,m,cq", [(1, 13, 5), (1, 14, 6), (2, 13, 4), (5, 14, 3)])
def test_generated_large_tiles(orc, k, m, cq):
    # 512- and 1024-thread tiles (generated kernels only)
    rng = np.random.default_rng(200 + m)
    c = I.random_mixed(16, 140, rng, n_inputs=3, p_input=0.2)
    _check(c, 2, 200 + m, orc, "fused", fuse_width=k, tile_qubits=m, low_qubits=cq)
    _check(I.rx_ry_rz_cz_ladder(16, 3), 2, 7, orc, "fused", fuse_width=k, tile_qubits=m, low_qubits=cq)


@pytest.mark.parametrize("method", METHODS)
def test_ladder_and_ring_small(orc, method):
    _check(I.rx_ry_rz_cz_ladder(14, 4), 3, 1003, orc, method)
    _check(I.ry_rz_cnot_ring(13, 4), 3, 1002, orc, method)


@pytest.mark.parametrize("method", METHODS)
def test_random_layers(orc, method):
    rng = np.random.default_rng(1004)
    for _ in range(3):
        n = int(rng.integers(8, 15))
        L = int(rng.integers(2, 13))
        c = I.random_layers(n, L, rng)
        _check(c, 1, 1004, orc, method)


@pytest.mark.parametrize("method", METHODS)
def test_product_state_closed_form_w20(method):
    # Ladder ansatz without entanglers: <Z_i> = cos(x_i + a_i) cos(theta_i) ... composed per
    # layer; with one layer the closed form is exact at any size.
    W = 20
    c = I.rx_ry_rz_cz_ladder(W, 1)
    c.gates = [g for g in c.gates if g[0] != "CZ"]
    w, x = I.draw_angles(c, 4, 77)
    got = gpu_run(c, w, x, 4, np.ones((4, W)), **_opts(method))
    w64, x64 = w.astype(np.float64), x.astype(np.float64)
    a = w64.reshape(W, 3)[:, 0][None, :]
    th = w64.reshape(W, 3)[:, 1][None, :]
    E = np.cos(x64 + a) * np.cos(th)
    assert np.abs(got["E"].cpu().numpy() - E).max() < EXP_TOL
    gx = -np.sin(x64 + a) * np.cos(th)
    ok, rel = grad_close(got["gx"].cpu().numpy(), gx)
    assert ok, rel
    gw = np.stack([(-np.sin(x64 + a) * np.cos(th)).sum(0), (-np.cos(x64 + a) * np.sin(th)).sum(0),
                   np.zeros(W)], axis=1).reshape(-1)
    assert np.abs(got["gw"].cpu().numpy() - gw).max() < 1e-4 * np.abs(gw).max()


def _sampled_full_size(orc, name, method, samples, **extra):
    """Full-size workload in the benchmark's launch configuration; the oracle
    recomputes selected samples one by one. Weight gradients are linear in the
    upstream gradient g, so zeroing g outside the selected samples makes the
    GPU's batch-summed weight gradient comparable with the oracle's."""
    c, batch, seed = I.workload(name)
    w, x = I.draw_angles(c, batch, seed)
    g = np.zeros((batch, c.n_qubits))
    g[samples] = I.draw_grad_out(c, batch, seed)[samples]
    print(f"[parity] {name} sampled {samples} method={method} {extra}", flush=True)
    got = gpu_run(c, w, x, batch, g, **_opts(method, **extra))
    ref = oracle_run(orc, c, w, x[samples], len(samples), g[samples])
    st = got["state"].cpu().numpy()[samples]
    assert np.abs(st - ref["state"]).max() <= AMP_TOL
    assert np.abs(got["E"].cpu().numpy()[samples] - ref["E"]).max() <= EXP_TOL
    assert np.abs(got["E_fused"].cpu().numpy()[samples] - ref["E"]).max() <= EXP_TOL
    ok, rel = grad_close(got["gw"].cpu().numpy(), ref["gw"])
    assert ok, ("weights", rel)
    ok, rel = grad_close(got["gx"].cpu().numpy()[samples], ref["gx"])
    assert ok, ("inputs", rel)
    # samples with g = 0 have zero input gradients
    others = [b for b in range(batch) if b not in samples]
    assert np.abs(got["gx"].cpu().numpy()[others]).max() == 0.0


@pytest.mark.parametrize("method", METHODS)
def test_full_size_w20_b64_sampled(orc, method):
    _sampled_full_size(orc, "w20_b64_ladder", method, [0, 37, 63])


@pytest.mark.parametrize("method", METHODS)
def test_full_size_w16_b256_sampled(orc, method):
    _sampled_full_size(orc, "w16_b256_ring", method, [0, 101, 255])


@pytest.mark.parametrize("method", ["fused", "fused_tables"])
def test_full_size_w16_b256_blocks_of_5_sampled(orc, method):
    # the 16-qubit workload as specified: split into blocks of up to 5 qubits
    _sampled_full_size(orc, "w16_b256_ring", method, [3, 200], fuse_width=5)


@pytest.mark.parametrize("method", METHODS)
def test_bitwise_deterministic(orc, method):
    # Two runs of the same plan give identical bits (no atomics on result paths).
    c = I.rx_ry_rz_cz_ladder(16, 3)
    w, x = I.draw_angles(c, 4, 5)
    g = I.draw_grad_out(c, 4, 5)
    a = gpu_run(c, w, x, 4, g, **_opts(method))
    b = gpu_run(c, w, x, 4, g, **_opts(method))
    assert np.array_equal(a["state"].cpu().numpy(), b["state"].cpu().numpy())
    assert np.array_equal(a["gw"].cpu().numpy(), b["gw"].cpu().numpy())
    assert np.array_equal(a["gx"].cpu().numpy(), b["gx"].cpu().numpy())


def test_generated_equals_table_driven_state():
    # Both fused kernel families apply the same ops in the same order per
    # amplitude (they differ only in float32 contraction order).
    c = I.ry_rz_cnot_ring(14, 3)
    w, x = I.draw_angles(c, 3, 9)
    a = gpu_run(c, w, x, 3, **_opts("fused"))
    b = gpu_run(c, w, x, 3, **_opts("fused_tables"))
    assert np.abs(a["state"].cpu().numpy() - b["state"].cpu().numpy()).max() < 2e-6


@pytest.mark.parametrize("method", ["fused", "fused_tables", "per_gate"])
def test_weight_remap(orc, method):
    """Weights enter as pi tanh(w) (section "Additional Optimizations");
    gradients with respect to the raw weights."""
    rng = np.random.default_rng(91)
    c = I.random_mixed(9, 120, rng, n_inputs=3, p_input=0.2)
    B = 3
    w, x = I.draw_angles(c, B, 91)
    w = (w - np.float32(math.pi)) * np.float32(0.8)  # raw weights over [-2.5, 2.5]
    g = I.draw_grad_out(c, B, 91)
    print(f"[parity] weight remap {method}", flush=True)
    got = gpu_run(c, w, x, B, g, **_opts(method, weight_remap=1))
    gw, gx, st = orc.adjoint_remapped(c.n_qubits, c.gates, w.astype(np.float64),
                                      x.astype(np.float64), B, g, want_state=True)
    assert np.abs(got["state"].cpu().numpy() - st).max() <= AMP_TOL
    assert np.abs(got["E"].cpu().numpy() - orc.expval(c.n_qubits, st)).max() <= EXP_TOL
    ok, rel = grad_close(got["gw"].cpu().numpy(), gw)
    assert ok, ("weights", rel)
    ok, rel = grad_close(got["gx"].cpu().numpy(), gx)
    assert ok, ("inputs", rel)


# -- multi-qubit gates: CRY, CRZ, Toffoli (CCX), CCZ, CCRX ----------------------

@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("W,ng,seed", [(3, 60, 71), (6, 120, 72), (9, 150, 73), (13, 150, 74)])
def test_controlled_kinds(orc, method, W, ng, seed):
    rng = np.random.default_rng(seed)
    c = I.random_mixed(W, ng, rng, n_inputs=3, p_input=0.3, kinds=I.ALL_KINDS)
    _check(c, 3, seed, orc, method)


@pytest.mark.parametrize("method", ["fused", "fused_tables"])
@pytest.mark.parametrize("W,m,cq", [(9, 4, 1), (11, 6, 2), (13, 8, 3)])
def test_controlled_kinds_small_tiles(orc, method, W, m, cq):
    """Small tiles put controls and targets outside the registers and the tile."""
    rng = np.random.default_rng(100 + W)
    c = I.random_mixed(W, 120, rng, n_inputs=2, p_input=0.3, kinds=I.ALL_KINDS)
    _check(c, 2, 100 + W, orc, method, tile_qubits=m, low_qubits=cq)


@pytest.mark.parametrize("method", METHODS)
def test_toffoli_truth_table(method):
    W = 5
    for order in [(0, 1, 2), (4, 0, 3), (2, 4, 0)]:
        c0, c1, t = order
        for bits in range(32):
            circ = I.Circuit(W, name="toffoli")
            for q in range(W):
                if (bits >> (W - 1 - q)) & 1:
                    circ.fixed("X", q)
            circ.fixed("CCX", c0, c1, t)
            got = gpu_run(circ, np.zeros(0, np.float32), np.zeros((1, 0), np.float32), 1, **_opts(method))
            st = got["state"].cpu().numpy()[0]
            b = [(bits >> (W - 1 - q)) & 1 for q in range(W)]
            if b[c0] and b[c1]:
                b[t] ^= 1
            want = sum(v << (W - 1 - q) for q, v in enumerate(b))
            assert st[want] == 1 and np.count_nonzero(st) == 1, (order, bits)


@pytest.mark.parametrize("method", ["fused", "fused_tables"])
@pytest.mark.parametrize("k", [1, 3, 5])
def test_dag_splitter(orc, method, k):
    """Plans split by the dependency-graph list scheduler (splitter = 1)."""
    rng = np.random.default_rng(200 + k)
    for c in (I.random_layers(12, 6, rng),
              I.random_mixed(10, 150, rng, n_inputs=2, p_input=0.3, kinds=I.ALL_KINDS),
              I.rx_ry_rz_cz_ladder(14, 3)):
        _check(c, 2, 200 + k, orc, method, fuse_width=k, splitter=1)


@pytest.mark.parametrize("method", ["fused", "fused_tables"])
@pytest.mark.parametrize("beam", [0, 64])
def test_pass_packing_beams(orc, method, beam):
    """Pass schedules from the plain program-order greedy (pack_beam = 0) and
    from a wider search than the default, on a ladder, a ring and a random
    circuit, at two tile shapes."""
    rng = np.random.default_rng(300 + beam)
    for c, m, cq in ((I.rx_ry_rz_cz_ladder(14, 4), 10, 3), (I.ry_rz_cnot_ring(12, 4), 8, 2),
                     (I.random_mixed(11, 160, rng, n_inputs=2, p_input=0.3, kinds=I.ALL_KINDS), 9, 2)):
        _check(c, 2, 300 + beam, orc, method, pack_beam=beam, tile_qubits=m, low_qubits=cq)


C128_TOL = 1e-12   # max-abs on amplitudes and <Z_i> with complex128 amplitudes
C128_GRAD = 1e-10  # relative on gradients


@pytest.mark.parametrize("case", ["w6_b8_ring", "mixed_all_kinds_w7", "mixed_inputs_w9"])
def test_c128_plain_method(orc, case):
    """The plain method instantiated for complex128 amplitudes and float64 gate
    matrices (the oracle's own precision): amplitudes and <Z_i> within 1e-12
    of the complex128 oracle, gradients within 1e-10 relative."""
    rng = np.random.default_rng(91)
    if case == "w6_b8_ring":
        c, batch, seed = I.workload("w6_b8_ring")
    elif case == "mixed_all_kinds_w7":
        c, batch, seed = I.random_mixed(7, 120, rng, kinds=I.ALL_KINDS), 3, 92
    else:
        c, batch, seed = I.random_mixed(9, 150, rng, n_inputs=4, p_input=0.3), 5, 93
    w, x = I.draw_angles(c, batch, seed)
    g = I.draw_grad_out(c, batch, seed)
    print(f"[parity] c128 {case} B={batch}", flush=True)
    got = gpu_run(c, w, x, batch, g, method="per_gate", amp_dtype="c128")
    assert got["state"].dtype == torch.complex128
    ref = oracle_run(orc, c, w, x, batch, g)
    assert np.abs(got["state"].cpu().numpy() - ref["state"]).max() <= C128_TOL
    assert np.abs(got["E"].cpu().numpy() - ref["E"]).max() <= C128_TOL
    assert np.abs(got["E_fused"].cpu().numpy() - ref["E"]).max() <= C128_TOL
    ok, rel = grad_close(got["gw"].cpu().numpy(), ref["gw"], tol=C128_GRAD)
    assert ok, ("weights", rel)
    if c.n_inputs:
        ok, rel = grad_close(got["gx"].cpu().numpy(), ref["gx"], tol=C128_GRAD)
        assert ok, ("inputs", rel)
