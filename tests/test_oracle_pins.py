"""Pins for the CPU oracle: each test ties it to something other than itself.

Sources of truth used here: the paper's worked examples (MSb-0 ordering in
"Symbols", the shape example in "Concept of Shapes", the reshape example in
"Circuit Splitting"), Eq. (1), the dense Kronecker formulation of Eq. (2)
(independent NumPy brute force), textbook states (Bell, GHZ), closed forms,
a classical bit-level simulation of permutation circuits, and exact
shift-rule / finite-difference gradients.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import kron
from paper_2404_09213_amd import inputs as I

TOL = 1e-12


def run(orc, W, gates, weights=(), x=None, batch=1):
    return orc.forward(W, gates, np.asarray(weights, dtype=np.float64), x, batch)


# -- ordering: worked examples -------------------------------------------------------

def test_msb0_last_qubit_is_index_1(orc):
    # "Symbols": |0001> has only the last qubit set.
    st = run(orc, 4, [("X", 3, -1, "none", -1)])
    assert np.argmax(np.abs(st[0])) == 1
    assert abs(st[0, 1] - 1) < TOL


def test_msb0_tensor_position_010(orc):
    # "Concept of Shapes": |010> sits at tensor position (0, 1, 0).
    st = run(orc, 3, [("X", 1, -1, "none", -1)])
    t = st[0].reshape(2, 2, 2)
    assert abs(t[0, 1, 0] - 1) < TOL
    assert np.argmax(np.abs(st[0])) == 2


# -- Eq. (1) and the other gate matrices ----------------------------------------

@pytest.mark.parametrize("theta", [0.0, math.pi / 2, math.pi, 2 * math.pi, 0.7312, -2.1])
def test_eq1_rx_partial_decomposition(orc, theta):
    Ra = np.eye(2)
    Rb = np.array([[0, 1], [1, 0]])
    expected = Ra * math.cos(theta / 2) + Rb * (-1j * math.sin(theta / 2))
    assert np.allclose(orc.gate_matrix("RX", theta), expected, atol=TOL)


def test_rx_special_angles(orc):
    X = np.array([[0, 1], [1, 0]])
    assert np.allclose(orc.gate_matrix("RX", math.pi), -1j * X, atol=TOL)
    assert np.allclose(orc.gate_matrix("RX", 2 * math.pi), -np.eye(2), atol=TOL)


@pytest.mark.parametrize("kind", ["H", "X", "Y", "Z", "RX", "RY", "RZ", "CRX"])
def test_gate_matrices_unitary(orc, kind):
    m = orc.gate_matrix(kind, 1.234)
    assert np.allclose(m @ m.conj().T, np.eye(2), atol=TOL)


@pytest.mark.parametrize("kind,axis", [("RX", "X"), ("RY", "Y"), ("RZ", "Z")])
def test_rotation_is_exponential_of_pauli(orc, kind, axis):
    # exp(-i theta sigma / 2) via an eigen-decomposition of sigma (scipy-free).
    sigma = {"X": kron.X, "Y": kron.Y, "Z": kron.Z}[axis]
    th = 0.913
    vals, vecs = np.linalg.eigh(sigma)
    expm = vecs @ np.diag(np.exp(-0.5j * th * vals)) @ vecs.conj().T
    assert np.allclose(orc.gate_matrix(kind, th), expm, atol=TOL)


# -- Eq. (2): dense Kronecker brute force vs the per-gate oracle -----------------

def _all_single_gates(W):
    gs = []
    for q in range(W):
        for k in ("H", "X", "Y", "Z", "RX", "RY", "RZ"):
            gs.append((k, q, -1, "weight" if k.startswith("R") else "none", 0 if k.startswith("R") else -1))
    for a in range(W):
        for b in range(W):
            if a != b:
                gs.append(("CNOT", a, b, "none", -1))
                gs.append(("CZ", a, b, "none", -1))
                gs.append(("CRX", a, b, "weight", 0))
    return gs


@pytest.mark.parametrize("W", [1, 2, 3, 5])
def test_every_gate_every_qubit_vs_kron(orc, W):
    rng = np.random.default_rng(W)
    # start from a random state: prepare it with a random circuit, then add the gate
    prep = I.random_mixed(W, 12, rng).gates if W > 0 else []
    wprep = rng.uniform(0, 2 * math.pi, size=len(prep))
    prep = [(g[0], g[1], g[2], "weight" if g[3] == "weight" else "none", i if g[3] == "weight" else -1)
            for i, g in enumerate(prep)]
    for g in _all_single_gates(W):
        theta = 0.8123
        w = np.concatenate([wprep, [theta]])
        g2 = (g[0], g[1], g[2], g[3], len(prep) if g[3] == "weight" else -1)
        gates = prep + [g2]
        got = run(orc, W, gates, w)
        ref = kron.states(W, gates, w, None, 1)
        assert np.max(np.abs(got - ref)) < TOL, g


@pytest.mark.parametrize("W,seed", [(4, 1), (6, 2), (8, 3)])
def test_random_circuits_vs_kron(orc, W, seed):
    rng = np.random.default_rng(seed)
    c = I.random_mixed(W, 40, rng, n_inputs=3, p_input=0.3)
    w, x = I.draw_angles(c, 3, seed)
    got = run(orc, W, c.gates, w.astype(np.float64), x.astype(np.float64), 3)
    ref = kron.states(W, c.gates, w.astype(np.float64), x.astype(np.float64), 3)
    assert np.max(np.abs(got - ref)) < 1e-12
    E = orc.expval(W, got)
    assert np.max(np.abs(E - kron.expval(W, ref))) < 1e-12


def test_kron_partials_zero_count():
    # The expanded partial matrices of a single-qubit gate have 2^W non-zeros,
    # i.e. 2^(2W) - 2^W zeros (section "Gate Matrix Caching").
    for W in (1, 3, 5):
        for w in range(W):
            for R in (np.eye(2), np.array([[0, 1], [1, 0]]), np.diag([1, -1]), np.array([[0, -1], [1, 0]])):
                M = kron.expand_1q(W, w, R)
                assert M.shape == (1 << W, 1 << W)
                assert int(np.count_nonzero(M == 0)) == (1 << (2 * W)) - (1 << W)


def test_kron_expansion_msb0():
    # X on the last qubit maps |0000> to |0001> = index 1.
    M = kron.expand_1q(4, 3, kron.X)
    assert M[1, 0] == 1


# -- "Circuit Splitting" worked example: W = 5, sub-circuit on qubits {1, 2} -----

def test_reshape_example_block_on_qubits_1_2(orc):
    rng = np.random.default_rng(11)
    sub = [("RY", 0, -1, "weight", 0), ("CNOT", 0, 1, "none", -1), ("CRX", 1, 0, "weight", 1),
           ("RZ", 1, -1, "weight", 2), ("H", 0, -1, "none", -1), ("CZ", 0, 1, "none", -1)]
    wsub = rng.uniform(0, 2 * math.pi, size=3)
    # the 4x4 block unitary G, column j = the sub-circuit applied to basis state j
    G = np.empty((4, 4), dtype=np.complex128)
    for j in range(4):
        prep = [("X", q, -1, "none", -1) for q in range(2) if (j >> (1 - q)) & 1]
        G[:, j] = run(orc, 2, prep + sub, wsub)[0]
    # a random batched 5-qubit state
    b = 3
    prep5 = I.random_mixed(5, 30, rng)
    w5 = rng.uniform(0, 2 * math.pi, size=prep5.n_weights)
    psi = run(orc, 5, prep5.gates, w5, batch=1)[0]
    batch = np.stack([psi * np.exp(1j * k) for k in range(b)])
    # reshape to (b * d0 * d3 * d4, d1 * d2), multiply the block, reshape back
    t = batch.reshape(b, 2, 2, 2, 2, 2).transpose(0, 1, 4, 5, 2, 3).reshape(b * 8, 4)
    t = t @ G.T
    out = t.reshape(b, 2, 2, 2, 2, 2).transpose(0, 1, 4, 5, 2, 3).reshape(b, 32)
    # the same gates relabelled onto qubits 1, 2 of the 5-qubit circuit
    relabel = [(k, q0 + 1, q1 + 1 if q1 >= 0 else -1, s, i) for (k, q0, q1, s, i) in sub]
    ws = np.concatenate([w5, wsub])
    relabel = [(k, q0, q1, s, i + prep5.n_weights if s == "weight" else -1) for (k, q0, q1, s, i) in relabel]
    full = run(orc, 5, prep5.gates + relabel, ws)[0]
    for k in range(b):
        assert np.max(np.abs(out[k] - full * np.exp(1j * k))) < TOL


# -- textbook states and closed forms ---------------------------------------------

def test_bell_state(orc):
    st = run(orc, 2, [("H", 0, -1, "none", -1), ("CNOT", 0, 1, "none", -1)])[0]
    r = 1 / math.sqrt(2)
    assert np.allclose(st, [r, 0, 0, r], atol=TOL)
    assert np.allclose(orc.expval(2, st[None]), 0, atol=TOL)


@pytest.mark.parametrize("W", [2, 5, 12, 18])
def test_ghz_state(orc, W):
    gates = [("H", 0, -1, "none", -1)] + [("CNOT", q, q + 1, "none", -1) for q in range(W - 1)]
    st = run(orc, W, gates)[0]
    r = 1 / math.sqrt(2)
    assert abs(st[0] - r) < TOL and abs(st[-1] - r) < TOL
    assert np.count_nonzero(np.abs(st) > 1e-14) == 2
    assert np.allclose(orc.expval(W, st[None]), 0, atol=TOL)


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.7, math.pi, 4.0])
def test_ry_expectation_cos(orc, theta):
    st = run(orc, 1, [("RY", 0, -1, "weight", 0)], [theta])
    assert abs(orc.expval(1, st)[0, 0] - math.cos(theta)) < TOL


def test_embedding_closed_form(orc):
    c = I.Circuit(7)
    I.angle_embedding(c)
    w, x = I.draw_angles(c, 4, 5)
    st = run(orc, 7, c.gates, w, x.astype(np.float64), 4)
    E = orc.expval(7, st)
    assert np.max(np.abs(E - np.cos(x.astype(np.float64)))) < 1e-12
    # product state: amplitude = prod_i (cos(x_i/2) if bit_i = 0 else -i sin(x_i/2))
    xb = x[1].astype(np.float64)
    for idx in (0, 5, 77, 127):
        a = 1 + 0j
        for i in range(7):
            a *= math.cos(xb[i] / 2) if not (idx >> (6 - i)) & 1 else -1j * math.sin(xb[i] / 2)
        assert abs(st[1, idx] - a) < TOL


def test_product_state_layer_closed_form(orc):
    # RX(x) RX(a) RY(theta) RZ(phi) on every qubit, no entangler: the two RX
    # add their angles and <Z_i> = cos(x_i + a_i) cos(theta_i).
    W = 6
    c = I.rx_ry_rz_cz_ladder(W, 1)
    c.gates = [g for g in c.gates if g[0] != "CZ"]
    w, x = I.draw_angles(c, 3, 9)
    w64, x64 = w.astype(np.float64), x.astype(np.float64)
    E = orc.expval(W, run(orc, W, c.gates, w64, x64, 3))
    a = w64.reshape(W, 3)[:, 0]
    theta = w64.reshape(W, 3)[:, 1]
    assert np.max(np.abs(E - np.cos(x64 + a[None, :]) * np.cos(theta)[None, :])) < 1e-12


def test_norm_preserved_and_inverse(orc):
    rng = np.random.default_rng(4)
    W = 9
    c = I.random_mixed(W, 120, rng)
    w = rng.uniform(0, 2 * math.pi, size=c.n_weights)
    st = run(orc, W, c.gates, w)[0]
    assert abs(np.vdot(st, st).real - 1) < 1e-12
    # inverse circuit: reversed order, negated angles (fixed gates are self-inverse)
    inv, winv = [], []
    for g in reversed(c.gates):
        if g[3] == "weight":
            inv.append((g[0], g[1], g[2], "weight", len(winv)))
            winv.append(-w[g[4]])
        else:
            inv.append(g if g[0] != "Y" else g)
    back = run(orc, W, c.gates + [(k, a, b, s, (i + c.n_weights) if s == "weight" else -1)
                                  for (k, a, b, s, i) in inv],
               np.concatenate([w, winv]))[0]
    e0 = np.zeros(1 << W)
    e0[0] = 1
    assert np.max(np.abs(back - e0)) < 1e-12


def _classical_sim(W, gates):
    """Track a basis state and a phase through X, CNOT, CZ, RX(pi) (= -i X)."""
    bits, phase = [0] * W, 1 + 0j
    for k, a, b, _, _ in gates:
        if k == "X":
            bits[a] ^= 1
        elif k == "RXPI":
            bits[a] ^= 1
            phase *= -1j
        elif k == "CNOT":
            if bits[a]:
                bits[b] ^= 1
        elif k == "CZ":
            if bits[a] and bits[b]:
                phase = -phase
    idx = 0
    for q in range(W):
        idx = (idx << 1) | bits[q]
    return idx, phase


@pytest.mark.parametrize("W", [3, 10, 20])
def test_permutation_circuits_classical(orc, W):
    rng = np.random.default_rng(W + 100)
    gates, sim = [], []
    for _ in range(60):
        k = ("X", "RXPI", "CNOT", "CZ")[int(rng.integers(4))]
        if k in ("CNOT", "CZ"):
            a, b = (int(v) for v in rng.choice(W, 2, replace=False))
        else:
            a, b = int(rng.integers(W)), -1
        sim.append((k, a, b, "none", -1))
        gates.append(("RX", a, -1, "weight", 0) if k == "RXPI" else (k, a, b, "none", -1))
    st = run(orc, W, gates, [math.pi])[0]
    idx, phase = _classical_sim(W, sim)
    assert abs(st[idx] - phase) < 1e-12
    assert np.count_nonzero(np.abs(st) > 1e-12) == 1


# -- gradients: shift rule, finite differences, adjoint -------------------------

@pytest.mark.parametrize("W,seed", [(3, 21), (5, 22), (7, 23)])
def test_adjoint_vs_shift_rule_vs_fd(orc, W, seed):
    rng = np.random.default_rng(seed)
    c = I.random_mixed(W, 30, rng, n_inputs=2, p_input=0.25)
    B = 2
    w, x = I.draw_angles(c, B, seed)
    w64, x64 = w.astype(np.float64), x.astype(np.float64)
    g = I.draw_grad_out(c, B, seed)
    gw, gx = orc.adjoint(W, c.gates, w64, x64, B, g)
    sw, sx = orc.param_shift(W, c.gates, w64, x64, B, g)
    fw, fx = orc.finite_diff(W, c.gates, w64, x64, B, g)
    for j in range(c.n_weights):
        assert abs(gw[j] - sw[j]) < 1e-10, (j, gw[j], sw[j])
        assert abs(gw[j] - fw[j]) < 1e-6
    for j in range(c.n_inputs):
        assert np.max(np.abs(gx[:, j] - sx[j])) < 1e-10
        assert np.max(np.abs(gx[:, j] - fx[j])) < 1e-6


def test_crx_four_term_rule_needed(orc):
    # Two-term shift is wrong for CRX; the four-term rule matches FD.
    W = 2
    # The H after CRX makes the observable non-diagonal on the control, so the
    # half-frequency term (interference of the two control branches) shows.
    gates = [("H", 0, -1, "none", -1), ("RY", 1, -1, "weight", 0), ("CRX", 0, 1, "weight", 1),
             ("H", 0, -1, "none", -1)]
    w = np.array([0.4, 1.1])
    g = np.array([[0.3, 1.0]])
    fw, _ = orc.finite_diff(W, gates, w, None, 1, g, weight_ids=[1])
    sw, _ = orc.param_shift(W, gates, w, None, 1, g, weight_ids=[1])
    two = 0.5 * (orc.loss(W, gates, w + [0, math.pi / 2], None, 1, g)
                 - orc.loss(W, gates, w - [0, math.pi / 2], None, 1, g)).sum()
    assert abs(sw[1] - fw[1]) < 1e-6
    assert abs(two - fw[1]) > 1e-3


def test_gradient_closed_forms(orc):
    # Product layer RX(x) RX(a) RY(theta) RZ(phi), <Z> = cos(x + a) cos(theta):
    # d/dx = d/da = -sin(x + a) cos(theta), d/dtheta = -cos(x + a) sin(theta),
    # d/dphi = 0. Embedding alone: d cos(x)/dx = -sin(x).
    W = 5
    c = I.rx_ry_rz_cz_ladder(W, 1)
    c.gates = [g for g in c.gates if g[0] != "CZ"]
    B = 3
    w, x = I.draw_angles(c, B, 31)
    w64, x64 = w.astype(np.float64), x.astype(np.float64)
    g = np.ones((B, W))
    gw, gx = orc.adjoint(W, c.gates, w64, x64, B, g)
    a = w64.reshape(W, 3)[:, 0][None, :]
    th = w64.reshape(W, 3)[:, 1][None, :]
    assert np.max(np.abs(gx - (-np.sin(x64 + a) * np.cos(th)))) < 1e-12
    assert np.max(np.abs(gw.reshape(W, 3)[:, 0] - (-np.sin(x64 + a) * np.cos(th)).sum(0))) < 1e-12
    assert np.max(np.abs(gw.reshape(W, 3)[:, 1] - (-np.cos(x64 + a) * np.sin(th)).sum(0))) < 1e-12
    assert np.max(np.abs(gw.reshape(W, 3)[:, 2])) < 1e-12
    emb = I.Circuit(W)
    I.angle_embedding(emb)
    _, gx2 = orc.adjoint(W, emb.gates, np.zeros(0), x64, B, g)
    assert np.max(np.abs(gx2 + np.sin(x64))) < 1e-12


@pytest.mark.slow
def test_adjoint_vs_shift_sampled_w12(orc):
    # A bigger ansatz, a sampled subset of parameters.
    c = I.rx_ry_rz_cz_ladder(12, 3)
    B = 2
    w, x = I.draw_angles(c, B, 1003)
    w64, x64 = w.astype(np.float64), x.astype(np.float64)
    g = np.ones((B, 12))
    gw, gx = orc.adjoint(12, c.gates, w64, x64, B, g)
    wid = [0, 17, 50, 107]
    sw, sx = orc.param_shift(12, c.gates, w64, x64, B, g, weight_ids=wid, input_ids=[3])
    fw, fx = orc.finite_diff(12, c.gates, w64, x64, B, g, weight_ids=wid, input_ids=[3])
    for j in wid:
        assert abs(gw[j] - sw[j]) < 1e-10
        assert abs(gw[j] - fw[j]) < 1e-6
    assert np.max(np.abs(gx[:, 3] - sx[3])) < 1e-10


# -- weight remapping (section "Additional Optimizations") ----------------------

def test_remap_range_and_values(orc):
    w = np.array([0.0, math.atanh(0.5), -math.atanh(0.5), 30.0, -30.0])
    r = orc.remap(w)
    assert r[0] == 0.0
    assert abs(r[1] - math.pi / 2) < 1e-15 and abs(r[2] + math.pi / 2) < 1e-15
    assert abs(r[3] - math.pi) < 1e-12 and abs(r[4] + math.pi) < 1e-12
    x = np.linspace(-5, 5, 101)
    assert np.all(np.abs(orc.remap(x)) < math.pi) and np.all(np.diff(orc.remap(x)) > 0)


def test_remapped_adjoint_vs_fd(orc):
    """Gradients with respect to the raw weights through pi tanh(w), against
    central differences of the loss taken through the remap."""
    W, B = 5, 2
    rng = np.random.default_rng(61)
    c = I.random_mixed(W, 30, rng, n_inputs=2, p_input=0.25)
    w, x = I.draw_angles(c, B, 61)
    w64, x64 = w.astype(np.float64), x.astype(np.float64)
    g = I.draw_grad_out(c, B, 61)
    gw, gx = orc.adjoint_remapped(W, c.gates, w64, x64, B, g)
    h = 1e-4
    for j in range(c.n_weights):
        wp, wm = w64.copy(), w64.copy()
        wp[j] += h
        wm[j] -= h
        fd = (orc.loss(W, c.gates, orc.remap(wp), x64, B, g).sum()
              - orc.loss(W, c.gates, orc.remap(wm), x64, B, g).sum()) / (2 * h)
        assert abs(gw[j] - fd) < 1e-6, (j, gw[j], fd)
    # input gradients are unchanged by the remap (it acts on weights only)
    gw0, gx0 = orc.adjoint(W, c.gates, orc.remap(w64), x64, B, g)
    assert np.array_equal(gx, gx0)


# -- multi-qubit gates: CRY, CRZ, Toffoli (CCX), CCZ, CCRX (section "Conclusion") --

def _x_prep(W, bits):
    """X on every qubit whose bit is 1: prepares the basis state `bits`."""
    return [("X", q, -1, "none", -1) for q in range(W) if (bits >> (W - 1 - q)) & 1]


@pytest.mark.parametrize("order", [(0, 1, 2), (2, 0, 1), (1, 2, 0)])
def test_toffoli_truth_table(orc, order):
    W = 3
    c0, c1, t = order
    for bits in range(8):
        gates = _x_prep(W, bits) + [("CCX", c0, c1, "none", -1, t)]
        st = run(orc, W, gates, np.zeros(0))
        b = [(bits >> (W - 1 - q)) & 1 for q in range(W)]
        if b[c0] and b[c1]:
            b[t] ^= 1
        want = sum(v << (W - 1 - q) for q, v in enumerate(b))
        assert abs(st[0, want] - 1) < 1e-15 and np.count_nonzero(np.abs(st[0]) > 1e-15) == 1


def test_ccz_phase_only_on_all_ones(orc):
    W = 4
    gates = [("H", q, -1, "none", -1) for q in range(W)] + [("CCZ", 3, 0, "none", -1, 2)]
    st = run(orc, W, gates, np.zeros(0))[0]
    for i in range(16):
        sign = -1 if (i >> 3) & 1 and (i >> 0) & 1 and (i >> 1) & 1 else 1  # qubits 0, 2, 3
        assert abs(st[i] - sign * 0.25) < 1e-15


def _controlled_kinds_vs_kron(orc, W, kinds, rng):
    for kind in kinds:
        nq = 3 if kind.startswith("CC") else 2
        for qs in itertools.permutations(range(W), nq):
            prep = I.random_mixed(W, 10, rng)
            w = list(rng.uniform(0, 2 * math.pi, size=prep.n_weights))
            theta = float(rng.uniform(0, 2 * math.pi))
            param = kind in ("CRY", "CRZ", "CCRX")
            if nq == 2:
                g = (kind, qs[0], qs[1], "weight" if param else "none", len(w) if param else -1)
            else:
                g = (kind, qs[0], qs[1], "weight" if param else "none", len(w) if param else -1, qs[2])
            w64 = np.array(w + [theta])
            gates = prep.gates + [g]
            got = run(orc, W, gates, w64)
            ref = kron.states(W, gates, w64, None, 1)
            assert np.max(np.abs(got - ref)) < 1e-12, (kind, qs)


def test_controlled_kinds_every_placement_vs_kron(orc):
    rng = np.random.default_rng(17)
    _controlled_kinds_vs_kron(orc, 3, ("CRY", "CRZ", "CCX", "CCZ", "CCRX"), rng)
    _controlled_kinds_vs_kron(orc, 4, ("CRY", "CRZ", "CCX", "CCZ", "CCRX"), rng)


@pytest.mark.parametrize("W,seed", [(4, 31), (6, 32)])
def test_random_circuits_with_controlled_kinds_vs_kron(orc, W, seed):
    rng = np.random.default_rng(seed)
    c = I.random_mixed(W, 50, rng, n_inputs=2, p_input=0.3, kinds=I.ALL_KINDS)
    w, x = I.draw_angles(c, 2, seed)
    got = run(orc, W, c.gates, w.astype(np.float64), x.astype(np.float64), 2)
    ref = kron.states(W, c.gates, w.astype(np.float64), x.astype(np.float64), 2)
    assert np.max(np.abs(got - ref)) < 1e-12
    assert np.max(np.abs(orc.expval(W, got) - kron.expval(W, ref))) < 1e-12


@pytest.mark.parametrize("W,seed", [(3, 41), (5, 42)])
def test_controlled_rotations_adjoint_vs_four_term_vs_fd(orc, W, seed):
    """Controlled rotations (generator eigenvalues 0, +-1) need the four-term
    rule; the adjoint generator is the target's Pauli where all controls are 1."""
    rng = np.random.default_rng(seed)
    c = I.random_mixed(W, 30, rng, n_inputs=2, p_input=0.25, kinds=I.ALL_KINDS)
    assert any(g[0] in ("CRY", "CRZ", "CCRX") for g in c.gates)
    B = 2
    w, x = I.draw_angles(c, B, seed)
    w64, x64 = w.astype(np.float64), x.astype(np.float64)
    g = I.draw_grad_out(c, B, seed)
    gw, gx = orc.adjoint(W, c.gates, w64, x64, B, g)
    sw, sx = orc.param_shift(W, c.gates, w64, x64, B, g)
    fw, fx = orc.finite_diff(W, c.gates, w64, x64, B, g)
    for j in range(c.n_weights):
        assert abs(gw[j] - sw[j]) < 1e-10, (j, gw[j], sw[j])
        assert abs(gw[j] - fw[j]) < 1e-6
    for j in range(c.n_inputs):
        assert np.max(np.abs(gx[:, j] - sx[j])) < 1e-10
        assert np.max(np.abs(gx[:, j] - fx[j])) < 1e-6
