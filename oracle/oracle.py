"""ctypes wrapper over the C oracle, plus shift-rule and finite-difference gradients.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).

Everything here is float64 / complex128. The angles handed in are whatever the
caller passes; to compare with the float32 GPU path, pass the same float32
values (they are upcast exactly).

Gradient conventions:

* Loss L = sum_{b,i} g[b,i] <Z_i>_b, with g the upstream gradient.
* Weight gradients are summed over samples and over every gate that reads the
  weight; input gradients are per sample.
* Parameter shift (section "Hybrid Machine Learning" names the rule; the paper
  calls it a finite-difference approximation, but for gates exp(-i theta P/2)
  with P^2 = 1 it is exact): df/dtheta = [f(theta + pi/2) - f(theta - pi/2)] / 2.
  The generator of CRX, |1><1| (x) X, has eigenvalues {0, +-1}, so its angle
  enters with two frequencies (1/2 and 1) and needs the four-term rule (as do
  CRY, CRZ and the doubly controlled CCRX)
  df = c+ [f(+pi/2) - f(-pi/2)] - c- [f(+3pi/2) - f(-3pi/2)],
  c+- = (sqrt(2) +- 1) / (4 sqrt(2)).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
_CLANG = "/opt/rocm/llvm/bin/clang"

# oracle-private gate numbering (must match the enum in qsv_oracle.c)
KIND_CODE = {"H": 0, "X": 1, "Y": 2, "Z": 3, "RX": 4, "RY": 5, "RZ": 6,
             "CNOT": 7, "CZ": 8, "CRX": 9, "CRY": 10, "CRZ": 11, "CCX": 12, "CCZ": 13,
             "CCRX": 14}
# kinds whose angle enters with two frequencies (a controlled rotation's
# generator has eigenvalues 0 and +-1): four-term shift rule
CONTROLLED_ROTATIONS = ("CRX", "CRY", "CRZ", "CCRX")
SRC_CODE = {"none": 0, "weight": 1, "input": 2}

_lib = None


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile qsv_oracle.c with gcc into liboracle.so next to it.

    sanitize: build liboracle_san.so instead, with clang's AddressSanitizer and
    UndefinedBehaviorSanitizer (the runtime of the sanitized libqsv build, so
    both can be loaded into one CPU test process; select it with
    QSV_ORACLE_LIB=<path>)."""
    if sanitize:
        tmp = _LIB_SAN + ".tmp"
        llvm_lib = os.path.join(os.path.dirname(os.path.dirname(_CLANG)), "lib")
        subprocess.check_call([_CLANG, "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                               "-fno-omit-frame-pointer", "-Wl,-rpath," + llvm_lib,
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_SAN)
        return _LIB_SAN
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("QSV_ORACLE_LIB") or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(path)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.orc_forward.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, ip, ip, ip, ip, dp, ctypes.c_int,
                                  dp, ctypes.c_int, ctypes.c_int, dp, vp]
        L.orc_expval.argtypes = [ctypes.c_int, ctypes.c_int, vp, dp]
        L.orc_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, ip, ip, ip, ip, dp, ctypes.c_int,
                                  dp, ctypes.c_int, ctypes.c_int, dp, dp, dp, vp]
        L.orc_gate_matrix.argtypes = [ctypes.c_int, ctypes.c_double, vp]
        for f in (L.orc_forward, L.orc_expval, L.orc_adjoint, L.orc_gate_matrix):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None else None


class _Gates:
    """Gate list of an inputs.Circuit (or any list of 5-tuples) as int arrays."""

    def __init__(self, gates):
        self.n = len(gates)
        self.kind = np.array([KIND_CODE[g[0]] for g in gates], dtype=np.intc).reshape(self.n)
        self.q0 = np.array([g[1] for g in gates], dtype=np.intc).reshape(self.n)
        self.q1 = np.array([g[2] for g in gates], dtype=np.intc).reshape(self.n)
        self.src = np.array([SRC_CODE[g[3]] for g in gates], dtype=np.intc).reshape(self.n)
        self.idx = np.array([g[4] for g in gates], dtype=np.intc).reshape(self.n)
        self.q2 = np.array([g[5] if len(g) > 5 else -1 for g in gates], dtype=np.intc).reshape(self.n)

    def args(self):
        ip = ctypes.c_int
        return (self.n, _ptr(self.kind, ip), _ptr(self.q0, ip), _ptr(self.q1, ip),
                _ptr(self.src, ip), _ptr(self.idx, ip), _ptr(self.q2, ip))


def _prep(weights, inputs, batch, n_inputs):
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
    if w.size == 0:
        w = np.zeros(1)
    if inputs is None or n_inputs == 0:
        x = np.zeros((batch, max(n_inputs, 1)))
    else:
        x = np.ascontiguousarray(np.asarray(inputs, dtype=np.float64).reshape(batch, n_inputs))
    return w, x


def forward(n_qubits, gates, weights, inputs, batch, shift=None):
    """States (batch, 2^n) complex128 after the gate list, from |0...0>."""
    G = _Gates(gates)
    n_w = int(np.asarray(weights).size)
    n_in = 0 if inputs is None else int(np.asarray(inputs).reshape(batch, -1).shape[1])
    w, x = _prep(weights, inputs, batch, n_in)
    st = np.empty((batch, 1 << n_qubits), dtype=np.complex128)
    sh = None if shift is None else np.ascontiguousarray(np.asarray(shift, dtype=np.float64))
    rc = lib().orc_forward(n_qubits, *G.args(), _ptr(w, ctypes.c_double), n_w,
                           _ptr(x, ctypes.c_double), n_in, batch,
                           _ptr(sh, ctypes.c_double), st.ctypes.data)
    if rc:
        raise ValueError(f"oracle forward rejected the circuit (code {rc})")
    return st


def expval(n_qubits, states):
    """<Z_i> for every sample and qubit: (batch, n) float64."""
    states = np.ascontiguousarray(states, dtype=np.complex128)
    batch = states.shape[0]
    out = np.empty((batch, n_qubits))
    lib().orc_expval(n_qubits, batch, states.ctypes.data, _ptr(out, ctypes.c_double))
    return out


def adjoint(n_qubits, gates, weights, inputs, batch, grad_out, want_state=False):
    """Adjoint gradients: (grad_weights (P,), grad_inputs (batch, n_inputs)[, states])."""
    G = _Gates(gates)
    n_w = int(np.asarray(weights).size)
    n_in = 0 if inputs is None else int(np.asarray(inputs).reshape(batch, -1).shape[1])
    w, x = _prep(weights, inputs, batch, n_in)
    g = np.ascontiguousarray(np.asarray(grad_out, dtype=np.float64).reshape(batch, n_qubits))
    gw = np.zeros(max(n_w, 1))
    gx = np.zeros((batch, max(n_in, 1)))
    st = np.empty((batch, 1 << n_qubits), dtype=np.complex128) if want_state else None
    rc = lib().orc_adjoint(n_qubits, *G.args(), _ptr(w, ctypes.c_double), n_w,
                           _ptr(x, ctypes.c_double), n_in, batch, _ptr(g, ctypes.c_double),
                           _ptr(gw, ctypes.c_double), _ptr(gx, ctypes.c_double),
                           st.ctypes.data if st is not None else None)
    if rc:
        raise ValueError(f"oracle adjoint rejected the circuit (code {rc})")
    out = (gw[:n_w], gx[:, :n_in])
    return out + (st,) if want_state else out


def gate_matrix(kind, theta=0.0):
    """The oracle's own 2x2 matrix for a gate kind (the target part of a controlled kind)."""
    out = np.empty(4, dtype=np.complex128)
    if lib().orc_gate_matrix(KIND_CODE[kind], float(theta), out.ctypes.data):
        raise ValueError(kind)
    return out.reshape(2, 2)


def remap(weights):
    """Quantum weight remapping (section "Additional Optimizations"): weights
    are mapped into (-pi, pi) by a smooth function; the paper names tanh and
    the range [-pi, pi], read here as w -> pi tanh(w)."""
    return math.pi * np.tanh(np.asarray(weights, dtype=np.float64))


def adjoint_remapped(n_qubits, gates, weights, inputs, batch, grad_out, want_state=False):
    """`adjoint` of the circuit whose gates take pi tanh(w) for every weight w;
    weight gradients with respect to w (chain rule: pi (1 - tanh(w)^2))."""
    w = np.asarray(weights, dtype=np.float64).reshape(-1)
    out = adjoint(n_qubits, gates, remap(w), inputs, batch, grad_out, want_state)
    gw = out[0] * (math.pi * (1.0 - np.tanh(w) ** 2))
    return (gw,) + tuple(out[1:])


def loss(n_qubits, gates, weights, inputs, batch, grad_out, shift=None):
    """Per-sample L_b = sum_i g[b,i] <Z_i>_b (float64, shape (batch,))."""
    E = expval(n_qubits, forward(n_qubits, gates, weights, inputs, batch, shift))
    return (E * np.asarray(grad_out).reshape(batch, n_qubits)).sum(axis=1)


_CP = (math.sqrt(2) + 1) / (4 * math.sqrt(2))
_CM = (math.sqrt(2) - 1) / (4 * math.sqrt(2))


def _gate_shift_derivative(n_qubits, gates, weights, inputs, batch, grad_out, k):
    """d L_b / d(angle of gate k) by the exact shift rule, per sample."""
    n = len(gates)

    def L(delta):
        sh = np.zeros(n)
        sh[k] = delta
        return loss(n_qubits, gates, weights, inputs, batch, grad_out, sh)

    if gates[k][0] in CONTROLLED_ROTATIONS:
        h1, h3 = math.pi / 2, 3 * math.pi / 2
        return _CP * (L(h1) - L(-h1)) - _CM * (L(h3) - L(-h3))
    return 0.5 * (L(math.pi / 2) - L(-math.pi / 2))


def param_shift(n_qubits, gates, weights, inputs, batch, grad_out, weight_ids=None,
                input_ids=None):
    """Shift-rule gradients for chosen weights / input columns (all by default)."""
    n_w = int(np.asarray(weights).size)
    n_in = 0 if inputs is None else int(np.asarray(inputs).reshape(batch, -1).shape[1])
    weight_ids = range(n_w) if weight_ids is None else weight_ids
    input_ids = range(n_in) if input_ids is None else input_ids
    gw = {j: 0.0 for j in weight_ids}
    gx = {j: np.zeros(batch) for j in input_ids}
    for k, g in enumerate(gates):
        if g[3] == "weight" and g[4] in gw:
            gw[g[4]] += _gate_shift_derivative(n_qubits, gates, weights, inputs, batch,
                                               grad_out, k).sum()
        elif g[3] == "input" and g[4] in gx:
            gx[g[4]] += _gate_shift_derivative(n_qubits, gates, weights, inputs, batch,
                                               grad_out, k)
    return gw, gx


def finite_diff(n_qubits, gates, weights, inputs, batch, grad_out, weight_ids=None,
                input_ids=None, h=1e-3):
    """Central differences in float64 with step h on the weights / input columns."""
    w0 = np.asarray(weights, dtype=np.float64).reshape(-1).copy()
    n_in = 0 if inputs is None else int(np.asarray(inputs).reshape(batch, -1).shape[1])
    x0 = None if inputs is None else np.asarray(inputs, dtype=np.float64).reshape(batch, n_in).copy()
    weight_ids = range(w0.size) if weight_ids is None else weight_ids
    input_ids = range(n_in) if input_ids is None else input_ids
    gw, gx = {}, {}
    for j in weight_ids:
        wp, wm = w0.copy(), w0.copy()
        wp[j] += h
        wm[j] -= h
        gw[j] = (loss(n_qubits, gates, wp, x0, batch, grad_out).sum()
                 - loss(n_qubits, gates, wm, x0, batch, grad_out).sum()) / (2 * h)
    for j in input_ids:
        xp, xm = x0.copy(), x0.copy()
        xp[:, j] += h
        xm[:, j] -= h
        gx[j] = (loss(n_qubits, gates, w0, xp, batch, grad_out)
                 - loss(n_qubits, gates, w0, xm, batch, grad_out)) / (2 * h)
    return gw, gx
