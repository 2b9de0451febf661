"""Brute-force Kronecker-product checker (n <= 8 qubits).

TEST INFRASTRUCTURE ONLY.

This follows the paper's dense formulation literally: every gate is expanded
to a full 2^W x 2^W operator by Kronecker products with identities (Eq. (2)),
with the exponent read as I_{2^w} (x) R (x) I_{2^(W-w-1)} for a 0-indexed,
MSb-0 qubit w (the printed I_{2^(W-w)} would give a 2^(W+1) operator). The
circuit unitary is the ordered product of these operators, and <Z_i> is
computed as psi^dagger (I (x) ... (x) Z (x) ... (x) I) psi, with no bit
arithmetic anywhere. Matrices are written here from their definitions,
independently of the C oracle.

Multi-qubit gates are expanded through projectors on the controls:
CU(c, t) = |0><0|_c (x) I + |1><1|_c (x) U_t, and with two controls the sum
over the four control patterns, U_t only on |11>; each term a Kronecker
product of one 2x2 factor per qubit, qubit 0 leftmost.
"""
from __future__ import annotations

import math

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = (X + Z) / math.sqrt(2)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)


def rotation(axis, theta):
    """R_d(theta) = cos(theta/2) I - i sin(theta/2) sigma_d  (Eq. (1) for d = x)."""
    sigma = {"X": X, "Y": Y, "Z": Z}[axis]
    return math.cos(theta / 2) * I2 - 1j * math.sin(theta / 2) * sigma


def kron_all(factors):
    out = np.ones((1, 1), dtype=np.complex128)
    for f in factors:
        out = np.kron(out, f)
    return out


def expand_1q(W, w, R):
    """I_{2^w} (x) R (x) I_{2^(W-w-1)}."""
    return np.kron(np.kron(np.eye(1 << w), R), np.eye(1 << (W - w - 1)))


def expand_controlled(W, c, t, U):
    return expand_multi_controlled(W, [c], t, U)


def expand_multi_controlled(W, controls, t, U):
    """sum over control patterns p of (x)_c |p_c><p_c| (x) (U_t if all ones else I):
    every term a Kronecker product of one 2x2 factor per qubit."""
    out = np.zeros((1 << W, 1 << W), dtype=np.complex128)
    for pattern in range(1 << len(controls)):
        f = [I2] * W
        for j, c in enumerate(controls):
            f[c] = P1 if (pattern >> j) & 1 else P0
        if pattern == (1 << len(controls)) - 1:
            f[t] = U
        out += kron_all(f)
    return out


def gate_operator(W, gate, theta):
    kind, q0, q1 = gate[0], gate[1], gate[2]
    q2 = gate[5] if len(gate) > 5 else -1
    if kind in ("RX", "RY", "RZ"):
        return expand_1q(W, q0, rotation(kind[1], theta))
    if kind in ("H", "X", "Y", "Z"):
        return expand_1q(W, q0, {"H": H, "X": X, "Y": Y, "Z": Z}[kind])
    if kind == "CNOT":
        return expand_controlled(W, q0, q1, X)
    if kind == "CZ":
        return expand_controlled(W, q0, q1, Z)
    if kind in ("CRX", "CRY", "CRZ"):
        return expand_controlled(W, q0, q1, rotation(kind[2], theta))
    if kind == "CCX":
        return expand_multi_controlled(W, [q0, q1], q2, X)
    if kind == "CCZ":
        return expand_multi_controlled(W, [q0, q1], q2, Z)
    if kind == "CCRX":
        return expand_multi_controlled(W, [q0, q1], q2, rotation("X", theta))
    raise KeyError(kind)


def gate_angle(gate, weights, inputs_row):
    if gate[3] == "weight":
        return float(weights[gate[4]])
    if gate[3] == "input":
        return float(inputs_row[gate[4]])
    return 0.0


def circuit_unitary(W, gates, weights, inputs_row):
    """Ordered product U_N ... U_1 of the expanded gate operators."""
    assert W <= 8, "brute force is for small circuits only"
    U = np.eye(1 << W, dtype=np.complex128)
    for g in gates:
        U = gate_operator(W, g, gate_angle(g, weights, inputs_row)) @ U
    return U


def states(W, gates, weights, inputs, batch):
    """(batch, 2^W) final states: the first column of each sample's unitary."""
    out = np.empty((batch, 1 << W), dtype=np.complex128)
    for b in range(batch):
        row = None if inputs is None else np.asarray(inputs, dtype=np.float64).reshape(batch, -1)[b]
        out[b] = circuit_unitary(W, gates, weights, row)[:, 0]
    return out


def expval(W, psi_batch):
    """<Z_i> = psi^dagger Z_i psi with Z_i expanded by Kronecker products."""
    out = np.empty((psi_batch.shape[0], W))
    for i in range(W):
        Zi = expand_1q(W, i, Z)
        out[:, i] = np.einsum("bj,jk,bk->b", psi_batch.conj(), Zi, psi_batch).real
    return out
