"""torch.autograd wrapper: log p_hat of a batch of click patterns as a
differentiable function of the squeezing parameters r and the transmissions
eta (the interferometer U is held fixed).

Forward = gbs_set_model_dev + gbs_prob_approx_dev; backward = gbs_grad_dev
(hand-written adjoint in libgbs.so).  The library runs on its own stream,
ordered against torch's current stream with events; PyTorch only provides the
device memory.  The contour plan is frozen after the first forward so that
repeated evaluations (fit loops, finite differences) see a smooth function.
"""
from __future__ import annotations

import numpy as np
import torch

from .gbs import Context


class ClickModel:
    """A fixed interferometer U and a fixed batch of click patterns."""

    def __init__(self, U: np.ndarray, offsets, modes, order: int, device: int = 0,
                 freeze_plan: bool = True):
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(self.device)   # default priority
        self.ctx = Context(device, stream=self.stream.cuda_stream)
        M = U.shape[0]
        self.M = M
        self.ure = torch.tensor(np.ascontiguousarray(U.real), dtype=torch.float64, device=self.device)
        self.uim = torch.tensor(np.ascontiguousarray(U.imag), dtype=torch.float64, device=self.device)
        # a first model is needed to validate the patterns against M
        self.ctx.gbs_set_model(U, np.zeros(M), np.ones(M))
        self.plan = self.ctx.gbs_plan_create(offsets, modes, order)
        self.P = len(offsets) - 1
        self.freeze_plan = freeze_plan
        self._ran = False

    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self, *tensors):
        cur = torch.cuda.current_stream(self.device)
        cur.wait_stream(self.stream)
        for t in tensors:
            t.record_stream(self.stream)

    def _param(self, x: torch.Tensor, name: str) -> torch.Tensor:
        """r or eta as a contiguous float64 tensor of length M on the model's device."""
        x = x.detach().to(self.device, torch.float64).contiguous()
        if x.numel() != self.M:
            raise ValueError(f"{name} must have M = {self.M} elements, got {x.numel()}")
        return x

    def forward_raw(self, r: torch.Tensor, eta: torch.Tensor) -> torch.Tensor:
        logp = torch.empty(self.P, dtype=torch.float64, device=self.device)
        status = torch.empty(self.P, dtype=torch.int32, device=self.device)
        r = self._param(r, "r")
        eta = self._param(eta, "eta")
        self._enter()
        self.ctx.gbs_set_model_dev(self.ure, self.uim, r, eta)
        self.ctx.gbs_prob_approx_dev(self.plan, logp, status)
        self._leave(logp, status, r, eta)
        if not self._ran and self.freeze_plan:
            self.stream.synchronize()
            self.plan.freeze(True)
        self._ran = True
        return logp

    def backward_raw(self, r, eta, dl):
        gr = torch.empty(self.M, dtype=torch.float64, device=self.device)
        ge = torch.empty(self.M, dtype=torch.float64, device=self.device)
        logp = torch.empty(self.P, dtype=torch.float64, device=self.device)
        status = torch.empty(self.P, dtype=torch.int32, device=self.device)
        r = self._param(r, "r")
        eta = self._param(eta, "eta")
        dl = dl.detach().to(self.device, torch.float64).contiguous()
        self._enter()
        self.ctx.gbs_set_model_dev(self.ure, self.uim, r, eta)
        self.ctx.gbs_grad_dev(self.plan, dl, logp, gr, ge, status)
        self._leave(gr, ge, logp, status, r, eta, dl)
        return gr, ge

    def __call__(self, r: torch.Tensor, eta: torch.Tensor) -> torch.Tensor:
        return ClickLogProb.apply(r, eta, self)


class ClickLogProb(torch.autograd.Function):
    @staticmethod
    def forward(ctx, r, eta, model: ClickModel):
        ctx.model = model
        ctx.save_for_backward(r, eta)
        return model.forward_raw(r, eta)

    @staticmethod
    def backward(ctx, grad_logp):
        r, eta = ctx.saved_tensors
        gr, ge = ctx.model.backward_raw(r, eta, grad_logp)
        return gr, ge, None


class StepGraph:
    """One model build + forward (+ adjoint when dl is given) of a ClickModel,
    recorded once into a HIP graph on the model's stream.  The inputs live in
    the tensors self.r, self.eta (and self.dl): copy new values into them and
    call replay(); results land in self.logp, self.status, self.grad_r,
    self.grad_eta.  The first, eager run allocates every workspace, so the
    recorded launches make no allocation or host synchronisation."""

    def __init__(self, model: ClickModel, r: torch.Tensor, eta: torch.Tensor,
                 dl: torch.Tensor = None):
        dev = model.device
        self.model = model
        self.r = r.detach().to(dev, torch.float64).clone()
        self.eta = eta.detach().to(dev, torch.float64).clone()
        self.dl = None if dl is None else dl.detach().to(dev, torch.float64).clone()
        self.logp = torch.empty(model.P, dtype=torch.float64, device=dev)
        self.status = torch.empty(model.P, dtype=torch.int32, device=dev)
        self.grad_r = torch.zeros(model.M, dtype=torch.float64, device=dev)
        self.grad_eta = torch.zeros(model.M, dtype=torch.float64, device=dev)
        model._enter()
        self._launch()
        model.stream.synchronize()
        if model.freeze_plan:
            model.plan.freeze(True)
            model._ran = True
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=model.stream):
            self._launch()
        model.stream.synchronize()

    def _launch(self):
        m = self.model
        m.ctx.gbs_set_model_dev(m.ure, m.uim, self.r, self.eta)
        if self.dl is None:
            m.ctx.gbs_prob_approx_dev(m.plan, self.logp, self.status)
        else:
            m.ctx.gbs_grad_dev(m.plan, self.dl, self.logp, self.grad_r, self.grad_eta, self.status)

    def replay(self):
        """Re-run the recorded step on the model's stream (ordered after the
        current stream's work; the current stream waits for it)."""
        self.model._enter()
        self.graph.replay()
        torch.cuda.current_stream(self.model.device).wait_stream(self.model.stream)
