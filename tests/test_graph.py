"""One captured step (forward + readout + backward) replayed as a HIP graph.

Every replay must give what the eager calls give on the same angles, with
other eager work and synchronisations between replays, and new angles written
into the captured buffers before each replay.
"""
import numpy as np
import pytest

from paper_2404_09213_amd import binding as B
from paper_2404_09213_amd import inputs as I

from .helpers import AMP_TOL, EXP_TOL, grad_close


def test_step_workspace_covers_parts():
    c = I.rx_ry_rz_cz_ladder(6, 2)
    p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs)
    step = B.qsv_workspace_size(p.handle, 8, B.OP_STEP)
    bwd = B.qsv_workspace_size(p.handle, 8, B.OP_BACKWARD)
    ev = B.qsv_workspace_size(p.handle, 8, B.OP_EXPVAL)
    fwd = B.qsv_workspace_size(p.handle, 8, B.OP_FORWARD)
    fx = B.qsv_workspace_size(p.handle, 8, B.OP_FORWARD_EXPVAL)
    # forward + readout runs first, then the backward over the same bytes
    assert step >= max(bwd, fx)
    # forward_expval: forward matrices, then the readout's partials
    assert fx >= fwd + ev


def _plans():
    rng = np.random.default_rng(77)
    c1 = I.random_mixed(11, 150, rng, n_inputs=4, p_input=0.2)
    c2 = I.rx_ry_rz_cz_ladder(9, 3)
    return [
        ("fused", [c1], lambda: B.Plan(c1.n_qubits, c1.gates, c1.n_weights, c1.n_inputs)),
        ("fused_tables", [c1], lambda: B.Plan(c1.n_qubits, c1.gates, c1.n_weights, c1.n_inputs,
                                              codegen=0)),
        ("per_gate", [c1], lambda: B.Plan(c1.n_qubits, c1.gates, c1.n_weights, c1.n_inputs,
                                          method="per_gate")),
        ("multi", [c1, c2], lambda: B.MultiPlan([c1, c2])),
    ]


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["fused", "fused_tables", "per_gate", "multi"])
def test_graph_replays_match_eager(name):
    import torch
    _, circs, make = [p for p in _plans() if p[0] == name][0]
    print(f"graph replay case={name}", flush=True)
    dev = torch.device("cuda:0")
    plan = make()
    batch = 5
    nw, nx = plan.n_weights, plan.n_inputs
    wbuf = torch.zeros(max(nw, 1), dtype=torch.float32, device=dev)
    xbuf = torch.zeros((batch, nx), dtype=torch.float32, device=dev)
    state = torch.empty((batch, plan.state_len), dtype=torch.complex64, device=dev)
    E = torch.empty((batch, plan.n_out), dtype=torch.float64, device=dev)
    gout = torch.zeros((batch, plan.n_out), dtype=torch.float64, device=dev)
    gw = torch.empty(max(nw, 1), dtype=torch.float64, device=dev)
    gx = torch.empty((batch, max(nx, 1)), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    s = torch.cuda.Stream(device=dev)
    graph = B.StepGraph(plan, wbuf[:nw], xbuf, batch, state, E, gout, gw, gx, s)
    rng = np.random.default_rng(5)
    for rep in range(4):
        w = rng.uniform(0, 2 * np.pi, nw).astype(np.float32)
        x = rng.uniform(-np.pi, np.pi, (batch, nx)).astype(np.float32)
        g = rng.normal(size=(batch, plan.n_out))
        wt = torch.from_numpy(w).to(dev)
        xt = torch.from_numpy(x).to(dev)
        gt = torch.from_numpy(g).to(dev)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            wbuf[:nw].copy_(wt)
            xbuf.copy_(xt)
            gout.copy_(gt)
            graph.launch()
        s.synchronize()
        # eager on the default stream
        st_e, E_e = plan.forward_expval(wt, xt, batch)
        gw_e, gx_e = plan.backward(wt, xt, st_e, gt)
        torch.cuda.synchronize()
        assert torch.equal(state, st_e), f"replay {rep}: state differs from eager"
        assert torch.equal(E, E_e), f"replay {rep}: expval differs from eager"
        ok, rel = grad_close(gw[:nw].cpu().numpy(), gw_e.cpu().numpy(), tol=1e-6)
        assert ok, f"replay {rep}: weight gradient rel err {rel}"
        if nx:
            ok, rel = grad_close(gx[:, :nx].cpu().numpy(), gx_e.cpu().numpy(), tol=1e-6)
            assert ok, f"replay {rep}: input gradient rel err {rel}"
    del graph
    torch.cuda.synchronize()


@pytest.mark.gpu
def test_graph_replay_matches_oracle(orc):
    """First replay against the oracle (not only against the eager path)."""
    import torch
    from .helpers import oracle_run
    print("graph replay vs oracle w6_b8_ring", flush=True)
    c, batch, seed = I.workload("w6_b8_ring")
    w, x = I.draw_angles(c, batch, seed)
    g = I.draw_grad_out(c, batch, seed)
    dev = torch.device("cuda:0")
    plan = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs)
    wt = torch.from_numpy(w).to(dev)
    xt = torch.from_numpy(np.ascontiguousarray(x.reshape(batch, c.n_inputs))).to(dev)
    state = torch.empty((batch, plan.state_len), dtype=torch.complex64, device=dev)
    E = torch.empty((batch, plan.n_out), dtype=torch.float64, device=dev)
    gt = torch.from_numpy(np.ascontiguousarray(g)).to(dev)
    gw = torch.empty(max(c.n_weights, 1), dtype=torch.float64, device=dev)
    gx = torch.empty((batch, c.n_inputs), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    s = torch.cuda.Stream(device=dev)
    graph = B.StepGraph(plan, wt, xt, batch, state, E, gt, gw, gx, s)
    for _ in range(2):
        graph.launch()
        s.synchronize()
    ref = oracle_run(orc, c, w, x, batch, g)
    assert np.abs(state.cpu().numpy() - ref["state"]).max() <= AMP_TOL
    assert np.abs(E.cpu().numpy() - ref["E"]).max() <= EXP_TOL
    ok, rel = grad_close(gw[: c.n_weights].cpu().numpy(), ref["gw"])
    assert ok, rel
    ok, rel = grad_close(gx.cpu().numpy(), ref["gx"])
    assert ok, rel


def test_graph_rejects_default_stream_and_small_workspace():
    """Argument checks happen before any device work (runs without a GPU)."""
    import ctypes
    c = I.rx_ry_rz_cz_ladder(4, 1)
    p = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs)
    L = B.lib()
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(256)
    rc = L.qsv_graph_create(p.handle, 2, dummy, dummy, dummy, dummy, None, dummy, dummy, dummy,
                            1 << 30, None, ctypes.byref(h))
    assert rc == -1 and h.value is None
    rc = L.qsv_graph_create(p.handle, 2, dummy, dummy, dummy, dummy, None, dummy, dummy, dummy,
                            16, dummy, ctypes.byref(h))
    assert rc == -1 and h.value is None
    assert L.qsv_graph_launch(None, None) == -8
    L.qsv_graph_destroy(None)


@pytest.mark.gpu
@pytest.mark.parametrize("method", ["fused", "per_gate"])
def test_one_plan_on_two_streams(method):
    """Two streams share a plan and run forward + readout + backward
    concurrently on different inputs; each stream gets its own workspace and
    the results equal the sequential ones bit for bit."""
    import torch
    print(f"[graph] two streams {method}", flush=True)
    dev = torch.device("cuda:0")
    c = I.rx_ry_rz_cz_ladder(14, 3)
    plan = B.Plan(c.n_qubits, c.gates, c.n_weights, c.n_inputs, method=method)
    batch = 6
    runs = []
    for seed in (11, 12):
        w, x = I.draw_angles(c, batch, seed)
        g = I.draw_grad_out(c, batch, seed)
        runs.append((torch.from_numpy(w).to(dev), torch.from_numpy(x).to(dev), torch.from_numpy(g).to(dev)))
    ref = []
    for w, x, g in runs:  # sequential, default stream
        st, E = plan.forward_expval(w, x, batch)
        gw, gx = plan.backward(w, x, st, g)
        ref.append((st, E, gw, gx))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    out = [None, None]
    for r in range(3):  # several rounds, both streams in flight together
        for i, (w, x, g) in enumerate(runs):
            with torch.cuda.stream(streams[i]):
                st, E = plan.forward_expval(w, x, batch)
                gw, gx = plan.backward(w, x, st, g)
                out[i] = (st, E, gw, gx)
        torch.cuda.synchronize()
        for i in range(2):
            for got, want in zip(out[i], ref[i]):
                assert torch.equal(got, want), (r, i)
