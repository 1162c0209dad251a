"""Fitting probe radiance to images through the probe trace.

The trace is linear in the stored radiance once the hit test is fixed, so an image loss
can be minimised over the radiance texels with its exact gradient (ProbeTraceFn ->
probe_trace_backward_hits from the forward's stored hits, or probe_trace_backward).  The
master radiance is FP32; the trace reads its FP16 rounding.  Adam updates the master: by
default pt_adam_step, which writes the FP16 storage for the next forward in the same pass,
or torch's Adam (the storage is then rounded from the master on every forward).
"""
from __future__ import annotations

import torch

from . import PT_FLAG_PERSISTENT, ProbeTraceFn, adam_step, make_views, trace_opts


class RadianceFit:
    """Adam on FP32 master radiance [P,N,N,3] against target images of the given views.

    keep_hits: the adjoint from the forward's hits (12 bytes per ray: probe and texel as
    int32, t as FP32) instead of a second
    trace.  optimizer: "fused" (pt_adam_step: moments, master and FP16 storage in one pass)
    or "torch" (torch.optim.Adam, its fused kernel where available)."""

    def __init__(self, grid, views, target_rgb, init=0.5, lr=1e-2, opts=None, keep_hits=True,
                 optimizer="fused", betas=(0.9, 0.999), eps=1e-8):
        if optimizer not in ("fused", "torch"):
            raise ValueError(f"optimizer must be 'fused' or 'torch', got {optimizer!r}")
        self.grid = grid
        self.views = make_views(views)
        if opts is None and len(self.views) > 1:
            # many views: one persistent launch over all their tiles, forward and adjoint
            opts = trace_opts(flags=PT_FLAG_PERSISTENT)
        self.target = target_rgb
        shape = (grid.P_total, grid.N, grid.N, 3)
        self.master = torch.full(shape, float(init), dtype=torch.float32, device=target_rgb.device,
                                 requires_grad=True)
        self.opts = opts
        self.keep_hits = keep_hits
        self.optimizer = optimizer
        self.lr, self.betas, self.eps = lr, betas, eps
        if optimizer == "fused":
            self.exp_avg = torch.zeros_like(self.master, requires_grad=False)
            self.exp_avg_sq = torch.zeros_like(self.master, requires_grad=False)
            self.storage = self.master.detach().to(torch.float16)
            self.steps = 0
        else:
            self.storage = None
            try:
                self.optim = torch.optim.Adam([self.master], lr=lr, betas=betas, eps=eps, fused=True)
            except (RuntimeError, TypeError, ValueError):
                self.optim = torch.optim.Adam([self.master], lr=lr, betas=betas, eps=eps)

    def loss(self):
        rgb = ProbeTraceFn.apply(self.master, self.grid, self.views, self.opts, self.keep_hits, self.storage)
        return ((rgb - self.target) ** 2).mean()

    def step(self) -> torch.Tensor:
        """One Adam step; returns the loss before the update (device scalar)."""
        # no gradient held between steps: the adjoint's fresh buffer becomes the gradient
        # itself (zeroing a held one and adding into it would move 6.4 GB more per step)
        self.master.grad = None
        loss = self.loss()
        loss.backward()
        if self.optimizer == "fused":
            self.steps += 1
            adam_step(self.master.detach(), self.master.grad, self.exp_avg, self.exp_avg_sq, self.storage,
                      self.steps, self.lr, self.betas, self.eps)
        else:
            self.optim.step()
        return loss.detach()
