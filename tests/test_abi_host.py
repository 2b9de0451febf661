"""Host-side tests of libqsv (no GPU): exported symbols, argument validation,
and the planner's split / schedule invariants checked with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2404_09213_amd import binding as B
from paper_2404_09213_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2404_09213_amd import build_lib
        build_lib.build()
    return B.lib()


def header_functions():
    txt = open(os.path.join(ROOT, "include", "qsv.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qsv_\w+)\s*\(", txt)))


def test_exports_every_declared_function(lib):
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)


def _plan_rc(W, gates, n_w=4, n_in=2, opts=None):
    arr = (B.qsv_gate * max(len(gates), 1))(*[B.qsv_gate(*g) for g in gates])
    h = ctypes.c_void_p()
    rc = B.lib().qsv_plan(W, arr, len(gates), n_w, n_in, ctypes.byref(opts) if opts else None,
                          ctypes.byref(h))
    if rc == 0:
        B.qsv_plan_destroy(h)
    return rc


@pytest.mark.parametrize("W,gate,code", [
    (3, (99, 0, -1, 0, -1), -3),          # unknown kind
    (3, (-1, 0, -1, 0, -1), -3),
    (3, (0, 3, -1, 0, -1), -2),           # qubit >= W
    (3, (0, -1, -1, 0, -1), -2),
    (3, (7, 1, 1, 0, -1), -2),            # CNOT on one qubit
    (3, (8, 0, 5, 0, -1), -2),            # CZ target out of range
    (3, (4, 0, -1, 1, 4), -4),            # weight index out of range
    (3, (4, 0, -1, 2, 2), -4),            # input column out of range
    (3, (4, 0, -1, 0, -1), -4),           # rotation without an angle source
    (3, (0, 0, -1, 1, 0), -4),            # fixed gate with an angle source
    (31, (0, 0, -1, 0, -1), -5),          # W above the limit
    (3, (12, 0, 1, 0, -1, 1), -2),        # CCX with a repeated qubit
    (3, (12, 0, 1, 0, -1, -1), -2),       # CCX without a target
    (3, (13, 0, 1, 0, -1, 3), -2),        # CCZ target out of range
    (3, (10, 2, 2, 1, 0), -2),            # CRY on one qubit
    (3, (14, 0, 1, 0, -1, 2), -4),        # CCRX without an angle source
    (3, (12, 0, 1, 1, 0, 2), -4),         # CCX with an angle source
    (3, (15, 0, -1, 0, -1), -3),          # unknown kind
    (0, (0, 0, -1, 0, -1), -1),
])
def test_plan_rejects(lib, W, gate, code):
    assert _plan_rc(W, [gate]) == code
    assert B.qsv_last_error()


def test_plan_rejects_bad_options(lib):
    for field, val in [("fuse_width", 0), ("fuse_width", 17), ("tile_qubits", 3),
                       ("tile_qubits", 15), ("low_qubits", 12), ("method", 2), ("codegen", 2),
                       ("max_pass_grads", 0), ("pack_beam", -1), ("pack_beam", 257)]:
        o = B.qsv_default_opts()
        setattr(o, field, val)
        assert _plan_rc(4, [(0, 0, -1, 0, -1)], opts=o) == -1, field


def test_c128_amplitudes_only_with_the_plain_method(lib):
    c = I.rx_ry_rz_cz_ladder(6, 2)
    o = B.qsv_default_opts()
    o.amp_dtype = 2
    o.method = 1
    assert _plan_rc(4, [(0, 0, -1, 0, -1)], opts=o) == -1
    with pytest.raises(B.QsvError) as e:
        B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method="fused", amp_dtype="c128")
    assert e.value.code == -1 and "per_gate" in str(e.value)
    with pytest.raises(B.QsvError):
        B.MultiPlan([I.rx_ry_rz_cz_ladder(5, 1), I.rx_ry_rz_cz_ladder(6, 1)], amp_dtype="c128")
    p64 = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method="per_gate")
    p128 = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method="per_gate", amp_dtype="c128")
    batch, S = 8, 8 * (1 << c.n_qubits)  # S: complex64 bytes of the batch
    # backward workspace: matrices, then psi and lambda copies (twice the bytes), then partials
    d = B.qsv_workspace_size(p128.handle, batch, 2) - B.qsv_workspace_size(p64.handle, batch, 2)
    assert d >= 2 * batch * S
    assert B.qsv_workspace_size(p128.handle, batch, 0) > B.qsv_workspace_size(p64.handle, batch, 0)
    # readout partials are float64 either way
    assert B.qsv_workspace_size(p128.handle, batch, 1) == B.qsv_workspace_size(p64.handle, batch, 1)


def test_calls_validate_before_touching_the_device(lib):
    c = I.rx_ry_rz_cz_ladder(5, 1)
    h = B.qsv_plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs)
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    big = 1 << 30
    # batch <= 0
    assert L.qsv_forward(h, fake, fake, 0, fake, fake, big, None) == -1
    # missing workspace / too small
    assert L.qsv_forward(h, fake, fake, 2, fake, None, 0, None) == -1
    assert L.qsv_forward(h, fake, fake, 2, fake, fake, 8, None) == -1
    assert L.qsv_expval(h, fake, 2, fake, fake, 8, None) == -1
    assert L.qsv_backward(h, fake, fake, 2, fake, fake, fake, 8, fake, fake, None) == -1
    # forward + readout: workspace too small, null output, null plan
    assert L.qsv_forward_expval(h, fake, fake, 2, fake, fake, fake, 8, None) == -1
    assert L.qsv_forward_expval(h, fake, fake, 2, fake, None, fake, big, None) == -1
    assert L.qsv_forward_expval(None, fake, fake, 2, fake, fake, fake, big, None) == -8
    assert L.qsv_workspace_size(h, 2, 4) >= L.qsv_workspace_size(h, 2, 0) + L.qsv_workspace_size(h, 2, 1)
    # null pointers
    assert L.qsv_forward(h, None, fake, 2, fake, fake, big, None) == -1
    assert L.qsv_backward(h, fake, fake, 2, None, fake, fake, big, fake, fake, None) == -1
    # null plan
    assert L.qsv_forward(None, fake, fake, 2, fake, fake, big, None) == -8
    assert L.qsv_workspace_size(None, 2, 0) == 0
    info = B.qsv_plan_info()
    assert L.qsv_plan_get_info(None, ctypes.byref(info)) == -8
    B.qsv_plan_destroy(h)


def test_use_after_destroy_is_rejected_without_touching_the_plan(lib):
    """A destroyed handle (and any pointer that was never a handle) is looked
    up in the library's registry of live handles, not read through, so every
    call returns QSV_ERR_HANDLE and a second destroy is ignored (under
    AddressSanitizer this also shows that no freed memory is read)."""
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    big = 1 << 30
    info = B.qsv_plan_info()
    c = I.rx_ry_rz_cz_ladder(5, 1)
    for make in (lambda: B.qsv_plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs),
                 lambda: B.qsv_plan_multi([(c.n_qubits, c.gates, c.n_weights, c.n_inputs)] * 2)):
        h = make()
        assert L.qsv_plan_get_info(h, ctypes.byref(info)) == 0
        B.qsv_plan_destroy(h)
        assert L.qsv_plan_get_info(h, ctypes.byref(info)) == -8
        assert "destroyed" in B.qsv_last_error()
        assert L.qsv_workspace_size(h, 2, 0) == 0
        assert L.qsv_forward(h, fake, fake, 2, fake, fake, big, None) == -8
        assert L.qsv_forward_expval(h, fake, fake, 2, fake, fake, fake, big, None) == -8
        assert L.qsv_forward_expval_noalloc(h, fake, fake, 2, fake, fake, None) == -8
        assert L.qsv_expval(h, fake, 2, fake, fake, big, None) == -8
        assert L.qsv_backward(h, fake, fake, 2, fake, fake, fake, big, fake, fake, None) == -8
        assert L.qsv_state_offset(h, 0) == -8
        assert L.qsv_plan_estimate(h, 2, 1.0, 1.0, 1.0, ctypes.byref(ctypes.c_double())) == -8
        L.qsv_plan_destroy(h)  # second destroy: ignored
    # a pointer that never was a plan or a graph (it points at a ctypes buffer)
    junk = ctypes.create_string_buffer(4096)
    assert L.qsv_plan_get_info(ctypes.addressof(junk), ctypes.byref(info)) == -8
    L.qsv_plan_destroy(ctypes.addressof(junk))
    assert L.qsv_graph_launch(ctypes.addressof(junk), None) == -8
    L.qsv_graph_destroy(ctypes.addressof(junk))
    assert L.qsv_graph_launch(None, None) == -8


def test_launch_shapes_beyond_hip_grid_limits_are_rejected(lib):
    """A tiled pass launches one block per tile; with small tiles on a large
    state the grid would exceed HIP's 2^32 threads per dimension, which must
    be reported before anything is launched."""
    L = B.lib()
    fake = ctypes.c_void_p(0x1000)
    big = 1 << 40
    c = I.rx_ry_rz_cz_ladder(30, 1)
    o = B.qsv_default_opts()
    o.tile_qubits, o.low_qubits = 4, 3  # 64 threads per 16-amplitude tile
    h = B.qsv_plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, o)
    assert L.qsv_forward(h, fake, fake, 1, fake, fake, big, None) == -5
    assert "tile_qubits" in B.qsv_last_error()
    B.qsv_plan_destroy(h)
    o.tile_qubits = 10         # 64 threads per 1024 amplitudes: fits
    h = B.qsv_plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, o)
    assert L.qsv_forward(h, fake, fake, 1, fake, fake, 8, None) == -1  # only the workspace is short
    B.qsv_plan_destroy(h)
    # gradient outputs: one reduction block each
    c = I.rx_ry_rz_cz_ladder(4, 1)
    h = B.qsv_plan(c.n_qubits, c.gates, c.n_weights, 1 << 9, None)
    assert L.qsv_backward(h, fake, fake, 1 << 15, fake, fake, fake, big, fake, fake, None) == -5
    B.qsv_plan_destroy(h)
    # multi-circuit rounds: one 256-thread block per tile of every circuit
    mp = B.MultiPlan([I.rx_ry_rz_cz_ladder(24, 1), I.rx_ry_rz_cz_ladder(24, 1)])
    assert L.qsv_forward(mp.handle, fake, fake, 1 << 10, fake, fake, 8, None) == -1  # fits; workspace short
    assert L.qsv_forward(mp.handle, fake, fake, 1 << 11, fake, fake, 8, None) == -5  # 2^32 threads
    assert "round" in B.qsv_last_error()


def test_strerror(lib):
    for code in range(-8, 1):
        assert B.qsv_strerror(code)


def test_workspace_sizes_grow_with_batch(lib):
    c = I.rx_ry_rz_cz_ladder(10, 2)
    for method in ("fused", "per_gate"):
        p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method=method)
        for op in (0, 1, 2):
            s1 = B.qsv_workspace_size(p.handle, 1, op)
            s8 = B.qsv_workspace_size(p.handle, 8, op)
            assert 0 < s1 <= s8
        # backward holds psi and lambda copies
        assert B.qsv_workspace_size(p.handle, 8, 2) >= 2 * 8 * (1 << 10) * 8


# -- planner invariants ----------------------------------------------------------------

def _qubits(g):
    q = {g[1]}
    if g[0] in I.TWO_QUBIT or g[0] in I.THREE_QUBIT:
        q.add(g[2])
    if g[0] in I.THREE_QUBIT:
        q.add(g[5])
    return q


def _circuits():
    rng = np.random.default_rng(5)
    out = [I.rx_ry_rz_cz_ladder(12, 3), I.ry_rz_cnot_ring(9, 3), I.random_layers(10, 6, rng),
           I.random_mixed(8, 150, rng, n_inputs=3, p_input=0.2), I.random_mixed(3, 60, rng),
           I.random_mixed(6, 80, rng), I.random_mixed(7, 90, rng, kinds=I.ALL_KINDS)]
    return out


@pytest.mark.parametrize("splitter", [0, 1])
@pytest.mark.parametrize("k", [1, 2, 3, 5, 6])
def test_splitter_invariants(lib, k, splitter):
    for c in _circuits():
        p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, fuse_width=k, splitter=splitter)
        blk = p.gate_blocks()
        assert np.all(blk >= 0)
        nb = blk.max() + 1
        assert p.info()["n_blocks"] == nb
        # block qubit sets within k (a single gate may exceed k = 1)
        for b in range(nb):
            members = [c.gates[i] for i in np.nonzero(blk == b)[0]]
            Q = set().union(*[_qubits(g) for g in members])
            assert len(Q) <= k or len(members) == 1, (b, Q)
        # per-qubit program order is preserved by executing blocks in index order
        for q in range(c.n_qubits):
            seq = [blk[i] for i, g in enumerate(c.gates) if q in _qubits(g)]
            assert seq == sorted(seq)


def test_splitter_block_counts_ladder(lib):
    # 20-qubit RX/RY/RZ + CZ-ladder ansatz, 10 layers: blocks at k = 4, 5, 6
    c = I.rx_ry_rz_cz_ladder(20, 10)
    counts = [B.Plan(20, c.gates, c.n_weights, c.n_inputs, fuse_width=k).info()["n_blocks"]
              for k in (4, 5, 6)]
    assert counts == [68, 48, 40]


def test_dag_splitter_needs_no_more_blocks(lib):
    """The dependency-graph splitter against the program-order rule: the
    20-qubit ladder at k = 4, 5, 6 and random-layer circuits at k = 4."""
    c = I.rx_ry_rz_cz_ladder(20, 10)
    counts = [B.Plan(20, c.gates, c.n_weights, c.n_inputs, fuse_width=k, splitter=1).info()["n_blocks"]
              for k in (4, 5, 6)]
    assert counts == [66, 48, 35]
    rng = np.random.default_rng(7)
    tot = [0, 0]
    for _ in range(30):
        c = I.random_layers(int(rng.integers(8, 19)), int(rng.integers(2, 13)), rng)
        for sp in (0, 1):
            tot[sp] += B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, fuse_width=4,
                              splitter=sp).info()["n_blocks"]
    assert tot == [501, 420]


@pytest.mark.parametrize("splitter", [0, 1])
@pytest.mark.parametrize("method", ["fused", "per_gate"])
@pytest.mark.parametrize("k,m,cq", [(5, 12, 5), (3, 8, 2), (2, 6, 0), (6, 10, 4), (4, 4, 1)])
def test_schedule_orders_are_valid(orc, lib, method, k, m, cq, splitter):
    # Applying the gates in the order the kernels use must give the same state.
    for c in _circuits():
        p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method=method, fuse_width=k,
                   tile_qubits=m, low_qubits=cq, splitter=splitter)
        w, x = I.draw_angles(c, 2, 3)
        ref = orc.forward(c.n_qubits, c.gates, w.astype(np.float64), x.astype(np.float64), 2)
        for which in (0, 1):
            order = p.gate_order(which)
            assert sorted(order.tolist()) == list(range(len(c.gates)))
            if which == 1:
                order = order[::-1]
            gates = [c.gates[i] for i in order]
            got = orc.forward(c.n_qubits, gates, w.astype(np.float64), x.astype(np.float64), 2)
            assert np.max(np.abs(got - ref)) < 1e-12, (c.name, which)


def test_pack_beam_never_needs_more_passes(orc, lib):
    """The beam search over tile seeds against the program-order greedy
    (pack_beam = 0): never more passes in either direction, fewer on the
    20-qubit ladder, and the kernels' gate order still gives the circuit's state."""
    rng = np.random.default_rng(11)
    cs = [I.rx_ry_rz_cz_ladder(20, 10), I.ry_rz_cnot_ring(16, 8)]
    cs += [I.random_layers(int(rng.integers(8, 17)), int(rng.integers(2, 9)), rng) for _ in range(6)]
    cs += [I.random_mixed(int(rng.integers(6, 14)), int(rng.integers(20, 120)), rng) for _ in range(6)]
    tot = {0: 0, 16: 0}
    for c in cs:
        for m, cq in ((12, 4), (8, 2)):
            n = {}
            for beam in (0, 16):
                p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, tile_qubits=m, low_qubits=cq,
                           pack_beam=beam)
                i = p.info()
                n[beam] = (i["n_fwd_passes"], i["n_bwd_passes"])
                tot[beam] += sum(n[beam])
            assert n[16][0] <= n[0][0] and n[16][1] <= n[0][1], (c.name, m, cq, n)
    assert tot[16] < tot[0]
    c = I.rx_ry_rz_cz_ladder(20, 10)
    counts = [B.Plan(20, c.gates, c.n_weights, c.n_inputs, pack_beam=b).info() for b in (0, 16)]
    assert [(i["n_fwd_passes"], i["n_bwd_passes"]) for i in counts] == [(5, 6), (4, 5)]
    # schedule validity with the greedy packing (the default packing is covered above)
    for c in cs[2:6]:
        p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, tile_qubits=8, low_qubits=2, pack_beam=0)
        w, x = I.draw_angles(c, 2, 3)
        ref = orc.forward(c.n_qubits, c.gates, w.astype(np.float64), x.astype(np.float64), 2)
        for which in (0, 1):
            order = p.gate_order(which)
            assert sorted(order.tolist()) == list(range(len(c.gates)))
            gates = [c.gates[i] for i in (order[::-1] if which else order)]
            got = orc.forward(c.n_qubits, gates, w.astype(np.float64), x.astype(np.float64), 2)
            assert np.max(np.abs(got - ref)) < 1e-12, (c.name, which)


@pytest.mark.timeout(60)
def test_packing_terminates_on_degenerate_inputs(orc, lib):
    """Inputs with nothing to pack or blocks no pass can hold whole: an empty
    circuit, a circuit that is all product-state prefix (empty forward body),
    and multi-gate blocks with more parametric gates than max_pass_grads
    allows (packed gate by gate)."""
    for W in (5, 13):
        for beam in (0, 16):
            p = B.Plan(W, [], 0, 0, pack_beam=beam)
            i = p.info()
            assert (i["n_fwd_passes"], i["n_bwd_passes"]) == (0, 0)
    gates = [("RX", q, -1, "input", q) for q in range(8)] + [("RY", q, -1, "weight", q) for q in range(8)]
    p = B.Plan(8, gates, 8, 8)
    i = p.info()
    assert i["n_prefix_gates"] == 16 and i["n_fwd_passes"] == 0 and i["n_bwd_passes"] >= 1
    rng = np.random.default_rng(5)
    for _ in range(3):
        c = I.random_layers(int(rng.integers(6, 11)), 4, rng)
        p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, fuse_width=4, max_pass_grads=1,
                   tile_qubits=6, low_qubits=1)
        w, x = I.draw_angles(c, 2, 3)
        ref = orc.forward(c.n_qubits, c.gates, w.astype(np.float64), x.astype(np.float64), 2)
        for which in (0, 1):
            order = p.gate_order(which)
            assert sorted(order.tolist()) == list(range(len(c.gates)))
            gates_o = [c.gates[i] for i in (order[::-1] if which else order)]
            got = orc.forward(c.n_qubits, gates_o, w.astype(np.float64), x.astype(np.float64), 2)
            assert np.max(np.abs(got - ref)) < 1e-12


def test_prefix_covers_embedding_and_first_layer(lib):
    c = I.rx_ry_rz_cz_ladder(20, 10)
    info = B.Plan(20, c.gates, c.n_weights, c.n_inputs).info()
    assert info["n_prefix_gates"] == 20 + 60
    c2 = I.ry_rz_cnot_ring(16, 8)
    assert B.Plan(16, c2.gates, c2.n_weights, c2.n_inputs).info()["n_prefix_gates"] == 16 + 32


@pytest.mark.slow
def test_generated_kernels_compile_for_gfx950(lib):
    # The per-plan kernels compile for gfx950 without a GPU (small plans).
    rng = np.random.default_rng(12)
    for c, opts in [(I.random_mixed(6, 40, rng, n_inputs=2, p_input=0.3), dict(tile_qubits=5, low_qubits=1)),
                    (I.rx_ry_rz_cz_ladder(11, 2), dict(tile_qubits=10, low_qubits=4)),
                    (I.random_layers(9, 3, rng), dict(tile_qubits=8, low_qubits=3)),
                    # 14-qubit tiles with the most gradient slots a pass may hold (LDS bound)
                    (I.rx_ry_rz_cz_ladder(15, 6), dict(tile_qubits=14, low_qubits=6))]:
        p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, **opts)
        src = B.qsv_plan_codegen_source(p.handle)
        assert src.count("__global__") == p.info()["n_fwd_passes"] + p.info()["n_bwd_passes"]
        B.qsv_plan_codegen_check(p.handle, "gfx950")


def test_codegen_source_empty_for_per_gate(lib):
    c = I.rx_ry_rz_cz_ladder(6, 1)
    p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method="per_gate")
    assert B.qsv_plan_codegen_source(p.handle) == ""


def test_parity_plans_cover_every_form_of_control_condition(lib):
    """The generated kernels test a control outside the registers in three ways:
    a swap under a lane-bit control as selects, a wave-uniform control as a
    branch on a value read from the first lane, and any other lane-bit control
    as a per-lane branch. The plans of the GPU parity tests with controlled
    gates on small tiles (tests/test_gpu_parity.py::test_controlled_kinds_small_tiles)
    and of the 16-qubit ring at full size must between them emit all three, so
    that parity covers each."""
    srcs = []
    for W, m, cq in [(9, 4, 1), (11, 6, 2), (13, 8, 3)]:
        rng = np.random.default_rng(100 + W)
        c = I.random_mixed(W, 120, rng, n_inputs=2, p_input=0.3, kinds=I.ALL_KINDS)
        p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method="fused", codegen=1,
                   tile_qubits=m, low_qubits=cq)
        srcs.append(B.qsv_plan_codegen_source(p.handle))
    c, batch, seed = I.workload("w16_b256_ring")
    p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method="fused")
    srcs.append(B.qsv_plan_codegen_source(p.handle))
    src = "\n".join(srcs)
    assert "const bool c_ = ((gT >>" in src                      # lane-bit swap as selects
    assert "if (__builtin_amdgcn_readfirstlane((int)(" in src     # wave-uniform branch
    assert re.search(r"^    if \(\(\(gT >> \d+\) & 1\)", src, re.M)  # lane-bit branch
