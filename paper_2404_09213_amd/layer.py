"""torch.nn integration: an autograd Function over the C ABI and a Module
holding the quantum weights as Parameters (section "API": circuits behave like
ordinary torch.nn.Modules, weights reachable through .parameters()).

Forward: qsv_forward_expval -> (B, W) float64 expectations (and psi_N).
Backward: qsv_backward (adjoint method; psi_N saved from the forward).
"""
from __future__ import annotations

import math

import torch

from . import binding
from . import inputs as _inputs


class QsvFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, weights, x, plan):
        w32 = weights.detach().to(torch.float32).contiguous()
        x32 = x.detach().to(torch.float32).contiguous()
        state, E = plan.forward_expval(w32, x32, x32.shape[0])
        ctx.plan = plan
        ctx.save_for_backward(w32, x32, state)
        ctx.dtypes = (weights.dtype, x.dtype)
        return E

    @staticmethod
    def backward(ctx, grad_E):
        w32, x32, state = ctx.saved_tensors
        plan = ctx.plan
        need_x = ctx.needs_input_grad[1]
        gw, gx = plan.backward(w32, x32, state, grad_E.detach(), want_inputs=need_x)
        gw = gw.to(ctx.dtypes[0]) if ctx.needs_input_grad[0] else None
        gx = gx.to(ctx.dtypes[1]) if (need_x and gx is not None) else None
        return gw, gx, None


class QuantumLayer(torch.nn.Module):
    """A parameterised circuit as a layer: forward(x (B, n_inputs)) -> <Z_i> (B, W)."""

    def __init__(self, circuit: "_inputs.Circuit", method: str = "fused", seed: int = 0, **opts):
        super().__init__()
        self.circuit = circuit
        self.plan = binding.Plan(circuit.n_qubits, circuit.gates, circuit.n_weights,
                                 circuit.n_inputs, method=method, **opts)
        g = torch.Generator().manual_seed(seed)
        self.weights = torch.nn.Parameter(
            torch.rand(circuit.n_weights, generator=g, dtype=torch.float32) * 2 * math.pi)

    def forward(self, x):
        return QsvFunction.apply(self.weights, x, self.plan)
