"""Fitting probe radiance to images through the probe trace.

The trace is linear in the stored radiance once the hit test is fixed, so an image loss
can be minimised over the radiance texels with its exact gradient (ProbeTraceFn ->
probe_trace_backward_hits from the forward's stored hits, or probe_trace_backward).  The master radiance is FP32 and is rounded to the FP16 storage
the trace reads on every forward; Adam (torch) updates the master.
"""
from __future__ import annotations

import torch

from . import PT_FLAG_PERSISTENT, ProbeTraceFn, make_views, trace_opts


class RadianceFit:
    """Adam on FP32 master radiance [P,N,N,3] against target images of the given views."""

    def __init__(self, grid, views, target_rgb, init=0.5, lr=1e-2, opts=None, keep_hits=True):
        self.grid = grid
        self.views = make_views(views)
        if opts is None and len(self.views) > 1:
            # many views: one persistent launch over all their tiles, forward and adjoint
            opts = trace_opts(flags=PT_FLAG_PERSISTENT)
        self.target = target_rgb
        shape = (grid.P_total, grid.N, grid.N, 3)
        self.master = torch.full(shape, float(init), dtype=torch.float32, device=target_rgb.device,
                                 requires_grad=True)
        # one fused kernel per step over the 400M-texel master where torch offers it
        try:
            self.optim = torch.optim.Adam([self.master], lr=lr, fused=True)
        except (RuntimeError, TypeError, ValueError):
            self.optim = torch.optim.Adam([self.master], lr=lr)
        self.opts = opts
        # adjoint from the forward's hits (8 bytes per ray) instead of a recomputed trace
        self.keep_hits = keep_hits

    def loss(self):
        rgb = ProbeTraceFn.apply(self.master, self.grid, self.views, self.opts, self.keep_hits)
        return ((rgb - self.target) ** 2).mean()

    def step(self) -> torch.Tensor:
        """One Adam step; returns the loss before the update (device scalar)."""
        # no gradient held between steps: the adjoint's fresh buffer becomes the gradient
        # itself (zeroing a held one and adding into it would move 6.4 GB more per step)
        self.optim.zero_grad(set_to_none=True)
        loss = self.loss()
        loss.backward()
        self.optim.step()
        return loss.detach()
