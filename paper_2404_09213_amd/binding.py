"""ctypes binding of libqsv (the C ABI declared in include/qsv.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of libqsv. The functions keep the C names (qsv_plan, qsv_forward,
qsv_expval, qsv_backward, ...); :class:`Plan` is a small owner object around a
plan handle that allocates workspaces with torch and passes device pointers
and the current HIP stream.

If the shared library has not been built, importing works but every call
raises -- there is no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# QSV_LIB selects another build of the same library (the sanitizer build of
# build_lib --sanitize, for CPU test runs)
LIB_PATH = os.environ.get("QSV_LIB") or os.path.join(_HERE, "libqsv.so")

KIND = {"H": 0, "X": 1, "Y": 2, "Z": 3, "RX": 4, "RY": 5, "RZ": 6, "CNOT": 7, "CZ": 8, "CRX": 9,
        "CRY": 10, "CRZ": 11, "CCX": 12, "CCZ": 13, "CCRX": 14}
SRC = {"none": 0, "weight": 1, "input": 2}
METHOD = {"fused": 0, "per_gate": 1}
OP_FORWARD, OP_EXPVAL, OP_BACKWARD, OP_STEP, OP_FORWARD_EXPVAL = 0, 1, 2, 3, 4
AMP = {"c64": 0, "c128": 1}

ERR_NAMES = {0: "QSV_OK", -1: "QSV_ERR_ARG", -2: "QSV_ERR_QUBIT", -3: "QSV_ERR_GATE",
             -4: "QSV_ERR_PARAM", -5: "QSV_ERR_TOO_BIG", -6: "QSV_ERR_OOM", -7: "QSV_ERR_HIP",
             -8: "QSV_ERR_HANDLE"}


class QsvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class qsv_gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("src", ctypes.c_int32), ("idx", ctypes.c_int32), ("q2", ctypes.c_int32)]


class qsv_opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("fuse_width", ctypes.c_int32),
                ("tile_qubits", ctypes.c_int32), ("low_qubits", ctypes.c_int32),
                ("max_pass_grads", ctypes.c_int32), ("codegen", ctypes.c_int32),
                ("bwd_gate_by_gate", ctypes.c_int32), ("mfma", ctypes.c_int32),
                ("weight_remap", ctypes.c_int32), ("splitter", ctypes.c_int32),
                ("amp_dtype", ctypes.c_int32), ("pack_beam", ctypes.c_int32)]


class qsv_plan_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "n_qubits", "n_gates", "n_weights", "n_inputs", "method", "fuse_width", "tile_qubits",
        "low_qubits", "n_prefix_gates", "n_blocks", "n_fwd_passes", "n_bwd_passes",
        "n_fwd_stages", "n_bwd_stages", "n_param_gates", "n_recipes", "n_circuits")]


class qsv_circuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32),
                ("gates", ctypes.POINTER(qsv_gate)), ("n_weights", ctypes.c_int32),
                ("n_inputs", ctypes.c_int32)]


class qsv_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]


EXPORTS = ("qsv_default_opts", "qsv_plan", "qsv_plan_multi", "qsv_plan_multi_each", "qsv_plan_circuit_offsets",
           "qsv_state_offset",
           "qsv_plan_multi_items", "qsv_plan_destroy", "qsv_workspace_size",
           "qsv_forward", "qsv_expval", "qsv_forward_expval", "qsv_forward_expval_noalloc",
           "qsv_backward", "qsv_plan_get_info",
           "qsv_plan_gate_order", "qsv_plan_gate_blocks", "qsv_plan_codegen_source",
           "qsv_plan_codegen_check", "qsv_plan_estimate", "qsv_pass_copy", "qsv_graph_create", "qsv_graph_launch",
           "qsv_graph_destroy", "qsv_profile_enable",
           "qsv_profile_read", "qsv_strerror", "qsv_last_error")

_lib = None


def lib():
    """Load libqsv.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"libqsv.so not found at {LIB_PATH}; run __graft_entry__.build()")
        # PyTorch bundles its own HIP runtime under the same library name as
        # the system one that libqsv.so was linked against. Loading torch first
        # makes libqsv.so bind to that runtime, so the process has one HIP
        # runtime; two separate runtimes in one process would each try to own
        # the GPU, and the one initialised second finds no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.qsv_default_opts.argtypes = [ctypes.POINTER(qsv_opts)]
        L.qsv_default_opts.restype = None
        L.qsv_plan.argtypes = [i32, ctypes.POINTER(qsv_gate), i32, i32, i32,
                               ctypes.POINTER(qsv_opts), ctypes.POINTER(vp)]
        L.qsv_plan.restype = ctypes.c_int
        L.qsv_plan_multi.argtypes = [ctypes.POINTER(qsv_circuit), i32, ctypes.POINTER(qsv_opts),
                                     ctypes.POINTER(vp)]
        L.qsv_plan_multi.restype = ctypes.c_int
        L.qsv_plan_multi_each.argtypes = [ctypes.POINTER(qsv_circuit), i32, ctypes.POINTER(qsv_opts),
                                          ctypes.POINTER(vp)]
        L.qsv_plan_multi_each.restype = ctypes.c_int
        L.qsv_plan_circuit_offsets.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                               ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.qsv_plan_circuit_offsets.restype = ctypes.c_int
        L.qsv_state_offset.argtypes = [vp, i32]
        L.qsv_state_offset.restype = i64
        L.qsv_plan_multi_items.argtypes = [vp, i64, i32, vp, i64, ctypes.POINTER(i64)]
        L.qsv_plan_multi_items.restype = ctypes.c_int
        L.qsv_plan_destroy.argtypes = [vp]
        L.qsv_plan_destroy.restype = None
        L.qsv_workspace_size.argtypes = [vp, i64, i32]
        L.qsv_workspace_size.restype = sz
        L.qsv_forward.argtypes = [vp, vp, vp, i64, vp, vp, sz, vp]
        L.qsv_forward.restype = ctypes.c_int
        L.qsv_expval.argtypes = [vp, vp, i64, vp, vp, sz, vp]
        L.qsv_expval.restype = ctypes.c_int
        L.qsv_forward_expval.argtypes = [vp, vp, vp, i64, vp, vp, vp, sz, vp]
        L.qsv_forward_expval.restype = ctypes.c_int
        L.qsv_forward_expval_noalloc.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.qsv_forward_expval_noalloc.restype = ctypes.c_int
        L.qsv_backward.argtypes = [vp, vp, vp, i64, vp, vp, vp, sz, vp, vp, vp]
        L.qsv_backward.restype = ctypes.c_int
        L.qsv_plan_get_info.argtypes = [vp, ctypes.POINTER(qsv_plan_info)]
        L.qsv_plan_get_info.restype = ctypes.c_int
        L.qsv_plan_gate_order.argtypes = [vp, i32, vp]
        L.qsv_plan_gate_order.restype = ctypes.c_int
        L.qsv_plan_gate_blocks.argtypes = [vp, vp]
        L.qsv_plan_gate_blocks.restype = ctypes.c_int
        L.qsv_plan_codegen_source.argtypes = [vp, ctypes.c_char_p, sz, ctypes.POINTER(sz)]
        L.qsv_plan_codegen_source.restype = ctypes.c_int
        L.qsv_plan_codegen_check.argtypes = [vp, ctypes.c_char_p]
        L.qsv_plan_codegen_check.restype = ctypes.c_int
        L.qsv_plan_estimate.argtypes = [vp, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_double)]
        L.qsv_plan_estimate.restype = ctypes.c_int
        L.qsv_pass_copy.argtypes = [vp, i32, i32, i64, vp, vp, sz, i32, vp]
        L.qsv_pass_copy.restype = ctypes.c_int
        L.qsv_graph_create.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp,
                                       ctypes.POINTER(vp)]
        L.qsv_graph_create.restype = ctypes.c_int
        L.qsv_graph_launch.argtypes = [vp, vp]
        L.qsv_graph_launch.restype = ctypes.c_int
        L.qsv_graph_destroy.argtypes = [vp]
        L.qsv_graph_destroy.restype = None
        L.qsv_profile_enable.argtypes = [vp, i32]
        L.qsv_profile_enable.restype = ctypes.c_int
        L.qsv_profile_read.argtypes = [vp, ctypes.POINTER(qsv_kernel_stat), i32,
                                       ctypes.POINTER(i32)]
        L.qsv_profile_read.restype = ctypes.c_int
        L.qsv_strerror.argtypes = [ctypes.c_int]
        L.qsv_strerror.restype = ctypes.c_char_p
        L.qsv_last_error.argtypes = []
        L.qsv_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise QsvError(rc, lib().qsv_last_error().decode())
    return rc


# -- thin wrappers with the C names ------------------------------------------------

def qsv_default_opts():
    o = qsv_opts()
    lib().qsv_default_opts(ctypes.byref(o))
    return o


def qsv_plan(n_qubits, gates, n_weights, n_inputs, opts=None):
    """gates: sequence of (kind, q0, q1, src, idx[, q2]) with kind/src as names or codes."""
    n = len(gates)
    arr = _gate_array(gates)
    h = ctypes.c_void_p()
    _check(lib().qsv_plan(int(n_qubits), arr, n, int(n_weights), int(n_inputs),
                          ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)))
    return h


def _gate_array(gates):
    n = len(gates)
    arr = (qsv_gate * max(n, 1))()
    for i, g in enumerate(gates):
        k, q0, q1, s, idx = g[:5]
        q2 = g[5] if len(g) > 5 else -1
        arr[i] = qsv_gate(KIND[k] if isinstance(k, str) else int(k), int(q0), int(q1),
                          SRC[s] if isinstance(s, str) else int(s), int(idx), int(q2))
    return arr


def _circuit_array(circuits):
    keep = [_gate_array(g) for (_, g, _, _) in circuits]
    arr = (qsv_circuit * len(circuits))()
    for i, (n, g, nw, ni) in enumerate(circuits):
        arr[i] = qsv_circuit(int(n), len(g), ctypes.cast(keep[i], ctypes.POINTER(qsv_gate)),
                             int(nw), int(ni))
    return arr, keep


def qsv_plan_multi(circuits, opts=None):
    """circuits: sequence of (n_qubits, gates, n_weights, n_inputs)."""
    arr, keep = _circuit_array(circuits)
    h = ctypes.c_void_p()
    _check(lib().qsv_plan_multi(arr, len(circuits), ctypes.byref(opts) if opts is not None else None,
                                ctypes.byref(h)))
    return h


def qsv_plan_multi_each(circuits, per_circuit):
    """circuits as for qsv_plan_multi; per_circuit: one qsv_opts per circuit."""
    arr, keep = _circuit_array(circuits)
    opts = (qsv_opts * len(circuits))(*per_circuit)
    h = ctypes.c_void_p()
    _check(lib().qsv_plan_multi_each(arr, len(circuits), opts, ctypes.byref(h)))
    return h


def qsv_plan_circuit_offsets(h, circuit):
    a, q, w, x = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().qsv_plan_circuit_offsets(h, int(circuit), ctypes.byref(a), ctypes.byref(q),
                                          ctypes.byref(w), ctypes.byref(x)))
    return {"amp": a.value, "qubit": q.value, "weight": w.value, "input": x.value}


def qsv_state_offset(h, circuit):
    """Byte offset of a circuit's amplitudes within one sample's state row."""
    v = int(lib().qsv_state_offset(h, int(circuit)))
    if v < 0:
        raise QsvError(v, lib().qsv_last_error().decode())
    return v


def qsv_plan_multi_items(h, batch, which):
    """Work list of a multi-circuit plan: int32 array (n_items, 3) of (circuit, pass, tile)."""
    n = ctypes.c_int64()
    _check(lib().qsv_plan_multi_items(h, int(batch), int(which), None, 0, ctypes.byref(n)))
    out = np.zeros((n.value, 3), dtype=np.int32)
    if n.value:
        _check(lib().qsv_plan_multi_items(h, int(batch), int(which), out.ctypes.data_as(ctypes.c_void_p), n.value,
                                          ctypes.byref(n)))
    return out


def qsv_plan_destroy(h):
    lib().qsv_plan_destroy(h)


def qsv_workspace_size(h, batch, op):
    return int(lib().qsv_workspace_size(h, int(batch), int(op)))


def qsv_forward(h, d_weights, d_inputs, batch, d_state, d_ws, ws_bytes, stream):
    return _check(lib().qsv_forward(h, d_weights, d_inputs, int(batch), d_state, d_ws,
                                    int(ws_bytes), stream))


def qsv_expval(h, d_state, batch, d_out, d_ws, ws_bytes, stream):
    return _check(lib().qsv_expval(h, d_state, int(batch), d_out, d_ws, int(ws_bytes), stream))


def qsv_forward_expval(h, d_weights, d_inputs, batch, d_state, d_out, d_ws, ws_bytes, stream):
    return _check(lib().qsv_forward_expval(h, d_weights, d_inputs, int(batch), d_state, d_out, d_ws,
                                           int(ws_bytes), stream))


def qsv_forward_expval_noalloc(h, d_weights, d_inputs, batch, d_state, d_out, stream):
    return _check(lib().qsv_forward_expval_noalloc(h, d_weights, d_inputs, int(batch), d_state, d_out,
                                                   stream))


def qsv_backward(h, d_weights, d_inputs, batch, d_state, d_grad_out, d_ws, ws_bytes,
                 d_grad_weights, d_grad_inputs, stream):
    return _check(lib().qsv_backward(h, d_weights, d_inputs, int(batch), d_state, d_grad_out,
                                     d_ws, int(ws_bytes), d_grad_weights, d_grad_inputs, stream))


def qsv_plan_get_info(h):
    info = qsv_plan_info()
    _check(lib().qsv_plan_get_info(h, ctypes.byref(info)))
    return {n: getattr(info, n) for n, _ in qsv_plan_info._fields_}


def qsv_plan_estimate(h, batch, hbm_gbs, alu_tflops, launch_us):
    us = ctypes.c_double()
    _check(lib().qsv_plan_estimate(h, int(batch), float(hbm_gbs), float(alu_tflops), float(launch_us),
                                   ctypes.byref(us)))
    return us.value


def qsv_pass_copy(h, which, pass_index, batch, d_state, d_ws, ws_bytes, lds_bytes, stream):
    _check(lib().qsv_pass_copy(h, which, pass_index, batch, d_state, d_ws, ws_bytes, lds_bytes, stream))


def qsv_plan_gate_order(h, which, n_gates):
    out = np.zeros(max(n_gates, 1), dtype=np.int32)
    _check(lib().qsv_plan_gate_order(h, int(which), out.ctypes.data))
    return out[:n_gates]


def qsv_plan_gate_blocks(h, n_gates):
    out = np.zeros(max(n_gates, 1), dtype=np.int32)
    _check(lib().qsv_plan_gate_blocks(h, out.ctypes.data))
    return out[:n_gates]


def qsv_plan_codegen_source(h):
    need = ctypes.c_size_t()
    _check(lib().qsv_plan_codegen_source(h, None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib().qsv_plan_codegen_source(h, buf, need.value, ctypes.byref(need)))
    return buf.value.decode()


def qsv_plan_codegen_check(h, arch):
    return _check(lib().qsv_plan_codegen_check(h, arch.encode()))


class StepGraph:
    """A captured step (forward + readout + backward) replayed with one call.

    The buffers passed at capture are fixed: write new angles / upstream
    gradients into them between replays. Owns its workspace.
    """

    def __init__(self, plan, weights, inputs, batch, state, expval, grad_out, gw, gx, stream):
        import torch
        self.plan = plan
        n = qsv_workspace_size(plan.handle, batch, OP_STEP)
        self.ws = torch.empty(max(n, 256), dtype=torch.uint8, device=state.device)
        self.stream = stream
        h = ctypes.c_void_p()
        P = Plan._ptr
        _check(lib().qsv_graph_create(plan.handle, int(batch), P(_f32(weights)), P(_f32(inputs)),
                                      P(state), P(expval), P(grad_out), P(gw), P(gx), P(self.ws),
                                      self.ws.numel(), ctypes.c_void_p(stream.cuda_stream),
                                      ctypes.byref(h)))
        self.handle = h
        self._keep = (weights, inputs, state, expval, grad_out, gw, gx)

    def launch(self):
        _check(lib().qsv_graph_launch(self.handle, ctypes.c_void_p(self.stream.cuda_stream)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            lib().qsv_graph_destroy(h)
            self.handle = None


def qsv_profile_enable(h, on):
    """on: False / 0 off, True / 1 per-kernel totals, 2 one record per launch."""
    return _check(lib().qsv_profile_enable(h, 2 if on == 2 else int(bool(on))))


def qsv_profile_read(h, max_out=512):
    """Per-kernel totals since the last read: {name: {launches, total_ms, bytes, flops}}."""
    arr = (qsv_kernel_stat * max_out)()
    n = ctypes.c_int32()
    _check(lib().qsv_profile_read(h, arr, max_out, ctypes.byref(n)))
    return {arr[i].name.decode(): {"launches": arr[i].launches, "total_ms": arr[i].total_ms,
                                   "bytes": arr[i].bytes, "flops": arr[i].flops}
            for i in range(n.value)}


def qsv_profile_read_launches(h, max_out=1 << 16):
    """Records of the per-launch mode (profile enabled with 2), in launch order:
    [{name, ms, bytes, flops}]."""
    arr = (qsv_kernel_stat * max_out)()
    n = ctypes.c_int32()
    _check(lib().qsv_profile_read(h, arr, max_out, ctypes.byref(n)))
    if n.value >= max_out:
        raise RuntimeError(f"more than {max_out - 1} launches recorded: read more often or raise max_out")
    return [{"name": arr[i].name.decode(), "ms": arr[i].total_ms, "bytes": arr[i].bytes,
             "flops": arr[i].flops} for i in range(n.value)]


def qsv_strerror(code):
    return lib().qsv_strerror(int(code)).decode()


def qsv_last_error():
    return lib().qsv_last_error().decode()


# -- plan owner with torch-allocated workspaces -------------------------------------

def make_opts(method="fused", fuse_width=None, tile_qubits=None, low_qubits=None,
              max_pass_grads=None, codegen=None, bwd_gate_by_gate=None, mfma=None,
              weight_remap=None, splitter=None, amp_dtype=None, pack_beam=None):
    o = qsv_default_opts()
    if pack_beam is not None:
        o.pack_beam = int(pack_beam)
    if amp_dtype is not None:
        o.amp_dtype = AMP[amp_dtype] if isinstance(amp_dtype, str) else int(amp_dtype)
    if splitter is not None:
        o.splitter = int(splitter)
    if weight_remap is not None:
        o.weight_remap = int(weight_remap)
    if mfma is not None:
        o.mfma = int(mfma)
    if bwd_gate_by_gate is not None:
        o.bwd_gate_by_gate = int(bwd_gate_by_gate)
    if codegen is not None:
        o.codegen = int(codegen)
    o.method = METHOD[method] if isinstance(method, str) else int(method)
    if fuse_width is not None:
        o.fuse_width = fuse_width
    if tile_qubits is not None:
        o.tile_qubits = tile_qubits
    if low_qubits is not None:
        o.low_qubits = low_qubits
    if max_pass_grads is not None:
        o.max_pass_grads = max_pass_grads
    return o


class Plan:
    """Owns a qsv plan; calls run on torch's current HIP stream."""

    def __init__(self, n_qubits, gates, n_weights, n_inputs, **opts):
        self.n_qubits = int(n_qubits)
        self.n_gates = len(gates)
        self.n_weights = int(n_weights)
        self.n_inputs = int(n_inputs)
        self.opts = make_opts(**opts)
        self.handle = qsv_plan(n_qubits, gates, n_weights, n_inputs, self.opts)
        self.state_len = 1 << self.n_qubits   # amplitudes per sample
        self.n_out = self.n_qubits            # expectation columns per sample
        self._ws = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            qsv_plan_destroy(h)
            self.handle = None

    def info(self):
        return qsv_plan_get_info(self.handle)

    def state_dtype(self):
        """torch dtype of the plan's states: complex64, or complex128 (amp_dtype c128)."""
        import torch
        return torch.complex128 if self.opts.amp_dtype == AMP["c128"] else torch.complex64

    def gate_order(self, which):
        return qsv_plan_gate_order(self.handle, which, self.n_gates)

    def gate_blocks(self):
        return qsv_plan_gate_blocks(self.handle, self.n_gates)

    def profile(self, on=True):
        qsv_profile_enable(self.handle, on)

    def profile_read(self):
        return qsv_profile_read(self.handle)

    def profile_launches(self):
        return qsv_profile_read_launches(self.handle)

    def workspace(self, batch, op, device):
        """Workspace of kind `op` for the current stream on `device`: calls on
        different streams get different buffers (the library requires distinct
        workspaces for calls that may run concurrently); calls on one stream
        reuse theirs in stream order."""
        import torch
        n = qsv_workspace_size(self.handle, batch, op)
        key = (op, str(device), torch.cuda.current_stream(device).cuda_stream)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < n:
            ws = torch.empty(max(n, 256), dtype=torch.uint8, device=device)
            self._ws[key] = ws
        return ws

    @staticmethod
    def _ptr(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    @staticmethod
    def _stream(device):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)

    def forward(self, weights, inputs, batch, state=None):
        """weights (P,) f32, inputs (B, n_inputs) f32 on the GPU -> state (B, 2^W) complex64."""
        import torch
        dev = weights.device if weights is not None and weights.numel() else inputs.device
        if state is None:
            state = torch.empty((batch, self.state_len), dtype=self.state_dtype(), device=dev)
        ws = self.workspace(batch, OP_FORWARD, dev)
        qsv_forward(self.handle, self._ptr(_f32(weights)), self._ptr(_f32(inputs)), batch,
                    self._ptr(state), self._ptr(ws), ws.numel(), self._stream(dev))
        return state

    def expval(self, state, out=None):
        import torch
        batch = state.shape[0]
        if out is None:
            out = torch.empty((batch, self.n_out), dtype=torch.float64, device=state.device)
        ws = self.workspace(batch, OP_EXPVAL, state.device)
        qsv_expval(self.handle, self._ptr(state), batch, self._ptr(out), self._ptr(ws), ws.numel(),
                   self._stream(state.device))
        return out

    def forward_expval(self, weights, inputs, batch, state=None, out=None):
        """forward() and expval() in one call -> (state, E)."""
        import torch
        dev = weights.device if weights is not None and weights.numel() else inputs.device
        if state is None:
            state = torch.empty((batch, self.state_len), dtype=self.state_dtype(), device=dev)
        if out is None:
            out = torch.empty((batch, self.n_out), dtype=torch.float64, device=dev)
        ws = self.workspace(batch, OP_FORWARD_EXPVAL, dev)
        qsv_forward_expval(self.handle, self._ptr(_f32(weights)), self._ptr(_f32(inputs)), batch,
                           self._ptr(state), self._ptr(out), self._ptr(ws), ws.numel(), self._stream(dev))
        return state, out

    def forward_expval_noalloc(self, weights, inputs, batch, state, out):
        """forward_expval() on the library's own scratch array: no workspace is
        allocated, so state and out must be given (and the plan must have run
        once on this device, which creates its tables)."""
        dev = state.device
        qsv_forward_expval_noalloc(self.handle, self._ptr(_f32(weights)), self._ptr(_f32(inputs)), batch,
                                   self._ptr(state), self._ptr(out), self._stream(dev))
        return state, out

    def pass_copy(self, which, pass_index, batch, state, lds_bytes=0):
        """qsv_pass_copy on a torch complex64 state; a backward pass runs on the
        backward workspace this plan uses for the current stream."""
        ws = self.workspace(batch, OP_BACKWARD, state.device) if which == 1 else None
        qsv_pass_copy(self.handle, which, pass_index, batch, self._ptr(state), self._ptr(ws),
                      0 if ws is None else ws.numel(), lds_bytes, self._stream(state.device))

    def backward(self, weights, inputs, state, grad_out, want_inputs=True, gw=None, gx=None):
        import torch
        batch = state.shape[0]
        dev = state.device
        if gw is None:
            gw = torch.empty((max(self.n_weights, 1),), dtype=torch.float64, device=dev)
        if gx is None and want_inputs and self.n_inputs:
            gx = torch.empty((batch, self.n_inputs), dtype=torch.float64, device=dev)
        ws = self.workspace(batch, OP_BACKWARD, dev)
        go = grad_out.to(torch.float64).contiguous()
        qsv_backward(self.handle, self._ptr(_f32(weights)), self._ptr(_f32(inputs)), batch,
                     self._ptr(state), self._ptr(go), self._ptr(ws), ws.numel(), self._ptr(gw),
                     self._ptr(gx) if want_inputs else None, self._stream(dev))
        return gw[: self.n_weights], gx


def _f32(t):
    if t is None or t.numel() == 0:
        return None
    import torch
    assert t.dtype == torch.float32 and t.is_contiguous(), "angles must be contiguous float32"
    return t


class MultiPlan(Plan):
    """Many circuits simulated together (one launch per round of passes).

    circuits: sequence of inputs.Circuit (or objects with n_qubits, gates,
    n_weights, n_inputs). Layouts are documented with qsv_plan_multi.
    """

    def __init__(self, circuits, per_circuit=None, **opts):
        """per_circuit: optional list of option dicts, one per circuit (each
        completed by `opts` and the defaults): qsv_plan_multi_each."""
        self.opts = make_opts(**opts)
        spec = [(c.n_qubits, c.gates, c.n_weights, c.n_inputs) for c in circuits]
        if per_circuit is None:
            self.handle = qsv_plan_multi(spec, self.opts)
        else:
            if len(per_circuit) != len(spec):
                raise ValueError("per_circuit needs one option set per circuit")
            self.handle = qsv_plan_multi_each(spec, [make_opts(**{**opts, **o}) for o in per_circuit])
        self.n_circuits = len(spec)
        self.n_gates = sum(len(c[1]) for c in spec)
        self.n_weights = sum(c[2] for c in spec)
        self.n_inputs = sum(c[3] for c in spec)
        self.n_qubits = sum(c[0] for c in spec)
        self.offsets = [qsv_plan_circuit_offsets(self.handle, i) for i in range(len(spec))]
        self.sizes = [c[0] for c in spec]
        self.state_len = self.offsets[-1]["amp"] + (1 << spec[-1][0])
        self.n_out = self.n_qubits
        self._ws = {}
