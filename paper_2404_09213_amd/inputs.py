"""Seeded synthetic workloads: circuits (gate lists) and angle batches.

This module holds no simulation arithmetic. It only writes down gate lists and
draws random angles, so that the oracle and the HIP path can be fed identical
inputs. It imports nothing but numpy.

A gate is a tuple ``(kind, q0, q1, src, idx)``, or ``(kind, q0, q1, src, idx,
q2)`` for the three-qubit kinds:

* ``kind``  one of ``H X Y Z RX RY RZ CNOT CZ CRX CRY CRZ CCX CCZ CCRX``;
* ``q0``    the qubit of a 1-qubit gate, or the first control;
* ``q1``    the target of a 1-control gate, the second control of a 2-control
            gate, ``-1`` for 1-qubit gates;
* ``src``   ``"none"`` (fixed gate), ``"weight"`` (angle = weights[idx]) or
            ``"input"`` (angle = inputs[b, idx], one per batch sample);
* ``idx``   index into the weight vector or the input row, ``-1`` if none;
* ``q2``    the target of a 2-control gate (absent or ``-1`` otherwise).

Qubit 0 is the most significant bit of a basis-state index (the MSb-0
convention of the paper's preliminaries, section "Symbols").

The workload shapes follow the paper's variational-circuit structure
(embedding layer, trainable rotation layers with entanglers, measurement;
section "Hybrid Machine Learning") and its benchmark protocol of random inputs
and optimizer-perturbed weights for every pass (section "Execution Time").
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

KINDS = ("H", "X", "Y", "Z", "RX", "RY", "RZ", "CNOT", "CZ", "CRX")
CONTROLLED_KINDS = ("CRY", "CRZ", "CCX", "CCZ", "CCRX")
ALL_KINDS = KINDS + CONTROLLED_KINDS
PARAMETRIC = ("RX", "RY", "RZ", "CRX", "CRY", "CRZ", "CCRX")
TWO_QUBIT = ("CNOT", "CZ", "CRX", "CRY", "CRZ")
THREE_QUBIT = ("CCX", "CCZ", "CCRX")


def gate_q2(g):
    """Third qubit of a gate tuple (-1 when the gate has fewer qubits)."""
    return g[5] if len(g) > 5 else -1


@dataclass
class Circuit:
    n_qubits: int
    gates: list = field(default_factory=list)
    n_weights: int = 0
    n_inputs: int = 0
    name: str = ""

    # -- construction helpers -------------------------------------------------
    def _add(self, kind, q0, q1, src, idx, q2):
        g = (kind, int(q0), int(q1), src, int(idx))
        self.gates.append(g + (int(q2),) if q2 >= 0 else g)

    def fixed(self, kind, q0, q1=-1, q2=-1):
        self._add(kind, q0, q1, "none", -1, q2)

    def weight(self, kind, q0, q1=-1, q2=-1):
        self._add(kind, q0, q1, "weight", self.n_weights, q2)
        self.n_weights += 1

    def input(self, kind, q0, col, q1=-1, q2=-1):
        self._add(kind, q0, q1, "input", int(col), q2)
        self.n_inputs = max(self.n_inputs, int(col) + 1)

    def arrays(self):
        """Gate list as parallel int arrays plus the kind names (for ctypes)."""
        n = len(self.gates)
        q0 = np.array([g[1] for g in self.gates], dtype=np.int32).reshape(n)
        q1 = np.array([g[2] for g in self.gates], dtype=np.int32).reshape(n)
        src = np.array([{"none": 0, "weight": 1, "input": 2}[g[3]] for g in self.gates],
                       dtype=np.int32).reshape(n)
        idx = np.array([g[4] for g in self.gates], dtype=np.int32).reshape(n)
        q2 = np.array([gate_q2(g) for g in self.gates], dtype=np.int32).reshape(n)
        kinds = [g[0] for g in self.gates]
        return kinds, q0, q1, src, idx, q2


# -- circuit families ----------------------------------------------------------

def angle_embedding(c: Circuit):
    """RX(x_i) on qubit i: the angle-embedding layer (one input column per qubit)."""
    for q in range(c.n_qubits):
        c.input("RX", q, q)


def ry_rz_cnot_ring(n_qubits: int, layers: int, embed: bool = True) -> Circuit:
    """Embedding, then `layers` x [RY(w), RZ(w) on every qubit; CNOT i -> (i+1) mod n]."""
    c = Circuit(n_qubits, name=f"ry_rz_cnot_ring_w{n_qubits}_l{layers}")
    if embed:
        angle_embedding(c)
    for _ in range(layers):
        for q in range(n_qubits):
            c.weight("RY", q)
            c.weight("RZ", q)
        for q in range(n_qubits):
            c.fixed("CNOT", q, (q + 1) % n_qubits)
    return c


def rx_ry_rz_cz_ladder(n_qubits: int, layers: int, embed: bool = True) -> Circuit:
    """Embedding, then `layers` x [RX, RY, RZ (weights) on every qubit; CZ(i, i+1), i < n-1]."""
    c = Circuit(n_qubits, name=f"rx_ry_rz_cz_ladder_w{n_qubits}_l{layers}")
    if embed:
        angle_embedding(c)
    for _ in range(layers):
        for q in range(n_qubits):
            c.weight("RX", q)
            c.weight("RY", q)
            c.weight("RZ", q)
        for q in range(n_qubits - 1):
            c.fixed("CZ", q, q + 1)
    return c


def random_layers(n_qubits: int, layers: int, rng: np.random.Generator) -> Circuit:
    """`layers` layers of random gates, one slot per qubit and layer.

    Slot w draws a kind uniformly from {H, RX, RY, RZ, CNOT, CZ, CRX}; a 2-qubit
    kind takes qubit w as control and a uniformly drawn other qubit as target.
    Every angle is a weight (no embedding).
    """
    kinds = ("H", "RX", "RY", "RZ", "CNOT", "CZ", "CRX")
    c = Circuit(n_qubits, name=f"random_w{n_qubits}_l{layers}")
    for _ in range(layers):
        for w in range(n_qubits):
            k = kinds[int(rng.integers(len(kinds)))]
            if k in TWO_QUBIT:
                if n_qubits < 2:
                    k = "RX"
                else:
                    t = int(rng.integers(n_qubits - 1))
                    t = t + 1 if t >= w else t
                    if k == "CRX":
                        c.weight("CRX", w, t)
                    else:
                        c.fixed(k, w, t)
                    continue
            if k in PARAMETRIC:
                c.weight(k, w)
            else:
                c.fixed(k, w)
    return c


def random_mixed(n_qubits: int, n_gates: int, rng: np.random.Generator,
                 n_inputs: int = 0, p_input: float = 0.0, kinds=KINDS) -> Circuit:
    """A random gate list over the given kinds, every qubit and every ordered
    pair or triple of qubits.

    Used for small-size parity and pin tests. When `n_inputs` > 0, a fraction
    `p_input` of the parametric gates reads a per-sample input column instead
    of a weight (mid-circuit data re-uploading).
    """
    c = Circuit(n_qubits, name=f"random_mixed_w{n_qubits}_g{n_gates}")
    for _ in range(n_gates):
        k = kinds[int(rng.integers(len(kinds)))]
        if (k in TWO_QUBIT and n_qubits < 2) or (k in THREE_QUBIT and n_qubits < 3):
            k = "RY"
        q2 = -1
        if k in THREE_QUBIT:
            a, b, t = rng.choice(n_qubits, size=3, replace=False)
            q0, q1, q2 = int(a), int(b), int(t)
        elif k in TWO_QUBIT:
            a, b = rng.choice(n_qubits, size=2, replace=False)
            q0, q1 = int(a), int(b)
        else:
            q0, q1 = int(rng.integers(n_qubits)), -1
        if k in PARAMETRIC:
            if n_inputs > 0 and rng.random() < p_input:
                c.input(k, q0, int(rng.integers(n_inputs)), q1, q2)
            else:
                c.weight(k, q0, q1, q2)
        else:
            c.fixed(k, q0, q1, q2)
    c.n_inputs = max(c.n_inputs, n_inputs)
    return c


# -- angle batches ---------------------------------------------------------------

def draw_angles(c: Circuit, batch: int, seed: int, run: int = 0):
    """Draw inputs x ~ U(-pi, pi) of shape (batch, n_inputs), then weights
    ~ U(0, 2 pi) in gate order, from numpy's PCG64 with the given seed.

    Values are drawn in float64 and rounded to float32; both the oracle and the
    GPU path consume exactly these float32 values. Timed run `run` > 0 draws a
    fresh x from seed + 100 * run and perturbs the weights by a small seeded
    step, mimicking an optimizer update between passes.
    """
    rng = np.random.default_rng(seed)
    x = rng.uniform(-math.pi, math.pi, size=(batch, c.n_inputs)).astype(np.float32)
    w = rng.uniform(0.0, 2.0 * math.pi, size=(c.n_weights,)).astype(np.float32)
    if run:
        r2 = np.random.default_rng(seed + 100 * run)
        x = r2.uniform(-math.pi, math.pi, size=(batch, c.n_inputs)).astype(np.float32)
        w = (w.astype(np.float64) + r2.normal(0.0, 1e-2, size=w.shape)).astype(np.float32)
    return w, x


def draw_grad_out(c: Circuit, batch: int, seed: int):
    """Upstream gradient dL/dE of shape (batch, n_qubits), float64, ~ U(-1, 1)."""
    rng = np.random.default_rng(seed + 7)
    return rng.uniform(-1.0, 1.0, size=(batch, c.n_qubits))


# -- the five benchmark workloads ---------------------------------------------------

def workload(name: str):
    """Return (circuit, batch, seed) for a named benchmark workload."""
    if name == "w6_b8_ring":
        return ry_rz_cnot_ring(6, 4), 8, 1001
    if name == "w16_b256_ring":
        return ry_rz_cnot_ring(16, 8), 256, 1002
    if name == "w20_b64_ladder":
        return rx_ry_rz_cz_ladder(20, 10), 64, 1003
    if name == "w28_b1_ring":
        return ry_rz_cnot_ring(28, 6), 1, 1005
    raise KeyError(name)


def uneven_set(n_circuits: int = 512, seed: int = 1004, qmin: int = 8, qmax: int = 18,
               lmin: int = 2, lmax: int = 12):
    """Uneven batch: n_circuits circuits with n ~ U{qmin..qmax} qubits and
    depth ~ U{lmin..lmax} layers of `random_layers`; batch 1 each."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_circuits):
        n = int(rng.integers(qmin, qmax + 1))
        L = int(rng.integers(lmin, lmax + 1))
        out.append(random_layers(n, L, rng))
    return out
