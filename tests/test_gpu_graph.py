"""A whole step (model build + forward + adjoint) recorded into a HIP graph and
replayed: every replay, with eager work and synchronisations in between and
with new inputs copied in, must reproduce the eager results (the forward
bit for bit; the adjoint, which sums with atomics, to 1e-12, and bit for bit
with deterministic gradients on)."""
import numpy as np
import pytest

from workloads import make_workload

pytestmark = pytest.mark.gpu


def eager(model, r, eta, dl):
    import torch
    logp = model.forward_raw(r, eta)
    gr, ge = model.backward_raw(r, eta, dl)
    torch.cuda.synchronize()
    return logp.cpu().numpy(), gr.cpu().numpy(), ge.cpu().numpy()


@pytest.mark.parametrize("cfg,P,order", [(2, 512, 3), (4, 64, 3), (5, 48, 2)])
def test_graph_replays_match_eager(cfg, P, order):
    """20 modes (rows up to 14 clicks), and the first rows of the 100-mode
    (25-60 clicks, order 3) and 144-mode (40-110 clicks, order 2) batches, whose
    rows above 40 clicks take the large-row kernels."""
    import torch
    from paper_2106_01445_amd.torch_api import ClickModel, StepGraph
    wl = make_workload(cfg, P=P)
    model = ClickModel(wl.U, wl.offsets, wl.modes, order)
    dev = torch.device("cuda")
    r0 = torch.tensor(wl.r, device=dev)
    eta0 = torch.tensor(wl.eta, device=dev)
    dl = torch.linspace(0.5, 1.5, wl.P, dtype=torch.float64, device=dev)
    ref = eager(model, r0, eta0, dl)           # also freezes the plan
    g = StepGraph(model, r0, eta0, dl)
    rng = np.random.default_rng(3)
    for k in range(4):
        a = torch.randn(256, 256, device=dev)   # unrelated eager work between replays
        (a @ a).sum().item()
        if k == 2:
            r1 = r0 * 1.01
            eta1 = eta0 * 0.99
            g.r.copy_(r1)
            g.eta.copy_(eta1)
            ref = eager(model, r1, eta1, dl)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(g.logp.cpu().numpy(), ref[0]), k
        assert np.all(g.status.cpu().numpy() == 0)
        for got, want in ((g.grad_r, ref[1]), (g.grad_eta, ref[2])):
            got = got.cpu().numpy()
            assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.max(np.abs(want))), k
        rng.random()


@pytest.mark.parametrize("cfg,P", [(2, 512), (4, 64)])
def test_graph_replays_deterministic(cfg, P):
    """With deterministic gradients on, every replay of the recorded step
    (eager work between replays, new inputs copied in at the third) gives the
    eager gradients bit for bit, at 20 modes and on the first rows of the
    100-mode batch (rows above 40 clicks in the large-row kernel), order 3."""
    import torch
    from paper_2106_01445_amd.torch_api import ClickModel, StepGraph
    wl = make_workload(cfg, P=P)
    model = ClickModel(wl.U, wl.offsets, wl.modes, 3)
    model.ctx.gbs_set_deterministic(True)
    dev = torch.device("cuda")
    r0 = torch.tensor(wl.r, device=dev)
    eta0 = torch.tensor(wl.eta, device=dev)
    dl = torch.linspace(0.5, 1.5, wl.P, dtype=torch.float64, device=dev)
    ref = eager(model, r0, eta0, dl)
    g = StepGraph(model, r0, eta0, dl)
    for k in range(4):
        a = torch.randn(256, 256, device=dev)
        (a @ a).sum().item()
        if k == 2:
            r1 = r0 * 1.01
            eta1 = eta0 * 0.99
            g.r.copy_(r1)
            g.eta.copy_(eta1)
            ref = eager(model, r1, eta1, dl)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(g.logp.cpu().numpy(), ref[0]), k
        assert np.array_equal(g.grad_r.cpu().numpy(), ref[1]), k
        assert np.array_equal(g.grad_eta.cpu().numpy(), ref[2]), k
