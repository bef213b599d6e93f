"""torch.autograd over branch lengths: forward = post-order pass, backward =
pre-order pass (Sections 2.3-2.6).

    lik = PhyloLikelihood(workload)          # tree, patterns, model on the GPU
    t = torch.exp(log_r) * tau               # any differentiable map to lengths
    logL = lik(t)                            # 0-dim FP64 CUDA tensor
    logL.backward()                          # pre-order gradient, chain rule by torch

The forward call runs the transition matrices, the post-order pass and the
logL reduction through ``pg_logL_and_grad_device`` with no gradient output;
the partial vectors stay resident and the backward runs only the pre-order
pass (``pg_grad_device``).  Both run on torch's current stream.  If another
forward of the same object ran in between, the backward first re-runs the
forward on the saved lengths so it always differentiates its own inputs.
"""
from __future__ import annotations

import torch

from .binding import PG_FP64, Context


class PhyloLikelihood:
    """A GPU log-likelihood bound to one tree, alignment and model."""

    def __init__(self, workload=None, *, parent=None, tip_masks=None, weights=None, Q=None, pi=None,
                 rates=None, cat_weights=None, device=0, precision=PG_FP64):
        self.ctx = Context(device, precision)
        self.device = torch.device("cuda", device)
        if workload is not None:
            self.ctx.set_workload(workload)
        else:
            self.ctx.set_tree(parent)
            Qa = torch.as_tensor(Q).cpu().numpy()
            self.ctx.set_patterns(tip_masks, weights, Qa.shape[0])
            self.ctx.set_model(Qa, pi, rates, cat_weights)
        self.n_branches = self.ctx.n_branches
        self.generation = 0
        self._stream = None

    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            self.ctx.set_stream(s)
            self._stream = s

    def _forward(self, t64):
        self._bind_stream()
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        self.ctx.logL_and_grad_device(t64.data_ptr(), out.data_ptr(), 0)
        self.generation += 1
        return out

    def __call__(self, t):
        return _PhyloLogL.apply(t, self)

    def close(self):
        self.ctx.close()


class _PhyloLogL(torch.autograd.Function):
    @staticmethod
    def forward(fctx, t, lik):
        if t.shape != (lik.n_branches,):
            raise ValueError(f"expected {lik.n_branches} branch lengths, got shape {tuple(t.shape)}")
        t64 = t.detach().to(device=lik.device, dtype=torch.float64).contiguous()
        out = lik._forward(t64)
        fctx.lik = lik
        fctx.gen = lik.generation
        fctx.in_dtype = t.dtype
        fctx.save_for_backward(t64)
        return out[0]

    @staticmethod
    def backward(fctx, grad_out):
        lik = fctx.lik
        (t64,) = fctx.saved_tensors
        if lik.generation != fctx.gen:
            lik._forward(t64)
        lik._bind_stream()
        g = torch.empty_like(t64)
        lik.ctx.grad_device(g.data_ptr())
        return (grad_out * g).to(fctx.in_dtype), None
