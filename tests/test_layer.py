"""torch.nn integration (section "API"): QuantumLayer / QsvFunction over the C ABI."""
import numpy as np
import pytest

from paper_2404_09213_amd import inputs as I

from .helpers import EXP_TOL, grad_close


def test_layer_holds_weights_as_parameters():
    import torch
    from paper_2404_09213_amd.layer import QuantumLayer
    c = I.rx_ry_rz_cz_ladder(6, 2)
    layer = QuantumLayer(c, seed=3)
    params = list(layer.parameters())
    assert len(params) == 1 and params[0].shape == (c.n_weights,)
    assert params[0].requires_grad and params[0].dtype == torch.float32


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["fused", "per_gate"])
def test_layer_forward_backward_vs_oracle(orc, method):
    import torch
    from paper_2404_09213_amd.layer import QuantumLayer
    print(f"[layer] {method}", flush=True)
    c = I.rx_ry_rz_cz_ladder(8, 3)
    B = 5
    dev = torch.device("cuda:0")
    layer = QuantumLayer(c, method=method, seed=4).to(dev)
    _, x = I.draw_angles(c, B, 4)
    xt = torch.from_numpy(np.ascontiguousarray(x.reshape(B, c.n_inputs))).to(dev).requires_grad_(True)
    g = I.draw_grad_out(c, B, 4)
    E = layer(xt)
    loss = (E * torch.from_numpy(g).to(dev)).sum()
    loss.backward()
    w = layer.weights.detach().cpu().numpy().astype(np.float64)
    gw, gx, st = orc.adjoint(c.n_qubits, c.gates, w, x.astype(np.float64), B, g, want_state=True)
    assert np.abs(E.detach().cpu().numpy() - orc.expval(c.n_qubits, st)).max() <= EXP_TOL
    ok, rel = grad_close(layer.weights.grad.cpu().numpy(), gw)
    assert ok, rel
    ok, rel = grad_close(xt.grad.cpu().numpy(), gx)
    assert ok, rel


@pytest.mark.gpu
def test_layer_trains():
    """A few Adam steps on a fixed target lower the loss (the optimizer loop the
    paper's benchmark times, section "Execution Time")."""
    import torch
    from paper_2404_09213_amd.layer import QuantumLayer
    print("[layer] train", flush=True)
    torch.manual_seed(0)
    c = I.ry_rz_cnot_ring(6, 2)
    dev = torch.device("cuda:0")
    layer = QuantumLayer(c, seed=1).to(dev)
    x = (torch.rand(16, c.n_inputs) * 2 - 1).to(dev)
    target = torch.linspace(-0.5, 0.5, c.n_qubits, dtype=torch.float64, device=dev).expand(16, -1)
    opt = torch.optim.Adam(layer.parameters(), lr=0.05)
    losses = []
    for _ in range(30):
        opt.zero_grad()
        loss = ((layer(x) - target) ** 2).mean()
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
    assert losses[-1] < 0.5 * losses[0], losses
