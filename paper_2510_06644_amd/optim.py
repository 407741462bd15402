"""Map update (Sec. 3.1: in mapping, the Gaussian gradients of Step 5 update
the 3D Gaussian parameters) with the library's Adam kernel.

A MapAdam keeps one session's parameter tensors and their two Adam moments
resident in device memory.  `step_many` updates any number of sessions with
one kernel launch per 64 tensors (`adam_step` in the C ABI)."""
from __future__ import annotations

import torch

from . import rtgs

# per-parameter learning rates of the map (means, log_scales, quats,
# opacity_logits, colors), the 3DGS-style schedule without decay
MAP_LRS = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3)


class MapAdam:
    def __init__(self, params, lrs=MAP_LRS, betas=(0.9, 0.999), eps=1e-15):
        self.params = [p.detach() for p in params]
        for p in self.params:
            if p.dtype != torch.float32 or not p.is_contiguous():
                raise ValueError("MapAdam takes contiguous float32 tensors")
        if len(lrs) != len(self.params):
            raise ValueError("one learning rate per tensor")
        self.lrs = [float(x) for x in lrs]
        self.betas = (float(betas[0]), float(betas[1]))
        self.eps = float(eps)
        self.exp_avg = [torch.zeros_like(p) for p in self.params]
        self.exp_avg_sq = [torch.zeros_like(p) for p in self.params]
        self.t = 0

    def groups(self, grads):
        grads = list(grads)
        if len(grads) != len(self.params):
            raise ValueError("one gradient per tensor")
        return [(p, g, m, v, lr, self.t + 1) for p, g, m, v, lr in
                zip(self.params, grads, self.exp_avg, self.exp_avg_sq, self.lrs)]

    def step(self, handle, grads, stream=None):
        step_many(handle, [(self, grads)], stream)

    def fused(self):
        """The C state of the next update (step t + 1) for a backward that
        applies it in the same pass (RTGS_GRAD_ADAM); the caller advances t
        once that backward is enqueued."""
        a = rtgs.CMapAdam()
        for k in range(5):
            a.exp_avg[k] = self.exp_avg[k].data_ptr()
            a.exp_avg_sq[k] = self.exp_avg_sq[k].data_ptr()
            a.lr[k] = self.lrs[k]
        a.step = self.t + 1
        a.beta1, a.beta2 = self.betas
        a.eps = self.eps
        return a

    def to(self, device):
        """Move the moments (the parameters are the caller's) to `device`."""
        self.exp_avg = [m.to(device) for m in self.exp_avg]
        self.exp_avg_sq = [v.to(device) for v in self.exp_avg_sq]
        return self

    def rebind(self, params):
        """Point at new parameter tensors (e.g. after moving them)."""
        self.params = [p.detach() for p in params]


def step_many(handle, items, stream=None):
    """items: [(MapAdam, grads)]; one update of every session's map."""
    items = list(items)
    if not items:
        return
    betas, eps = items[0][0].betas, items[0][0].eps
    groups = []
    for opt, grads in items:
        if opt.betas != betas or opt.eps != eps:
            raise ValueError("step_many: sessions must share betas and eps")
        groups += opt.groups(grads)
    rtgs.adam_step(handle, groups, betas[0], betas[1], eps, stream)
    for opt, _ in items:
        opt.t += 1
