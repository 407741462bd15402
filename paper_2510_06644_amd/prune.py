"""Adaptive Gaussian pruning as a mask-prune schedule over tracking
iterations (Sec. 4.1), with the tile lists of each window reused (Sec. 3,
Observation 6).

Readings of the paper (it fixes lambda = 0.8, K0 = 5, the 5% rule and a
50% cap on the pruned fraction, Sec. 6.1-6.2; the rest is ours):

* A window is one full iteration followed by K masked iterations.  The full
  iteration bins and sorts afresh, scores every Gaussian by Eq. 7 from its
  gradients to mean and covariance, and masks the lowest.  The K masked
  iterations leave the masked Gaussians out of rendering and reuse the full
  iteration's tile lists and depth order (projection only).  The next full
  iteration first removes the masked Gaussians for good (stable compaction
  of the map), which is the paper's "(K+1)-th iteration".
* K is K0 for the first window; after each window the next K is K0 // 2 if
  the change ratio of tile-Gaussian intersections over the window exceeds
  5%, otherwise 2 K0 (both relative to K0, as the text states them).
* The change ratio compares, over the Gaussians that survive the removal,
  the pairs of the window's full iteration with those of the next full
  iteration: pairs in exactly one of the two, divided by the former (a
  Gaussian's pairs are the tiles of its rectangle).  Masked Gaussians are
  kept until then, so removal itself does not count as change.
* Each window masks window_ratio of the visible unmasked Gaussians, and the
  removed total never exceeds cap (50%) of the initial map.
"""
from __future__ import annotations

import dataclasses

import torch

from . import rtgs


class MaskPruneSchedule:
    """The interval logic alone (no GPU): which iterations are full, and K."""

    def __init__(self, k0=5, threshold=0.05):
        if k0 < 1:
            raise ValueError("k0 >= 1")
        self.k0 = int(k0)
        self.threshold = float(threshold)
        self.k = 0
        self.left = 0
        self.windows = []          # (K, change ratio or None) per window

    def next_is_full(self):
        return self.left == 0

    def start_window(self, ratio=None):
        """A full iteration ran; ratio is the change over the last window
        (None for the first).  Returns the new window's K."""
        if ratio is None:
            k = self.k0
        else:
            k = max(1, self.k0 // 2) if ratio > self.threshold else 2 * self.k0
        self.k = k
        self.left = k
        self.windows.append((k, ratio))
        return k

    def step_masked(self):
        if self.left <= 0:
            raise RuntimeError("no masked iteration left in this window")
        self.left -= 1


@dataclasses.dataclass
class PruneConfig:
    k0: int = 5
    lam: float = 0.8
    window_ratio: float = 0.1
    cap: float = 0.5
    threshold: float = 0.05


class MaskPruneTracker:
    """Tracking iterations of one map under the schedule, on the GPU.

    scene: the five map tensors (means, log_scales, quats, opacity_logits,
    colors); the tracker replaces them by compacted copies when it removes
    Gaussians (read .scene after each iteration).  grads_fn(state) returns
    (dL/dcolor, dL/ddepth) for a forward state.

    No iteration waits for the GPU: the masked count and the change ratio
    are copied to pinned host memory behind an event and read when they are
    needed (the ratio at the window's first masked iteration, which then
    fixes K; the count at the next full iteration, to size the compacted
    map)."""

    def __init__(self, renderer, scene, cam, cfg: PruneConfig | None = None):
        self.R = renderer
        self.scene = tuple(scene)
        self.cam = cam
        self.cfg = cfg or PruneConfig()
        self.sched = MaskPruneSchedule(self.cfg.k0, self.cfg.threshold)
        self.n0 = self.scene[0].shape[0]
        self.removed = 0
        self.mask = None           # device uint8 [n]: masked in the current window
        self.ref = None            # forward state of the window's full iteration
        self.rect_ref = None       # its tile rectangles, device int32 [n, 4]
        self.full_iters = 0
        self.masked_iters = 0
        self._pending = False      # a full iteration ran; K not fixed yet
        dev = self.scene[0].device
        self._count = torch.zeros(1, dtype=torch.int32, device=dev)
        self._kept = torch.zeros(1, dtype=torch.int32, device=dev)
        self._change = torch.zeros(2, dtype=torch.int64, device=dev)
        self._h_count = torch.zeros(1, dtype=torch.int32).pin_memory()
        self._h_change = torch.zeros(2, dtype=torch.int64).pin_memory()
        self._ev_count = torch.cuda.Event()
        self._ev_change = torch.cuda.Event()
        self._has_change = False

    @property
    def n(self):
        return self.scene[0].shape[0]

    def iteration(self, view, grads_fn):
        """One tracking iteration; returns dL/dxi (device float [6])."""
        if self._pending:
            ratio = None
            if self._has_change:
                self._ev_change.synchronize()
                d, r = (int(x) for x in self._h_change.tolist())
                ratio = d / r if r > 0 else 0.0
            self.sched.start_window(ratio)
            self._pending = False
        if self.sched.next_is_full():
            return self._full(view, grads_fn)
        return self._masked(view, grads_fn)

    def _remove_masked(self):
        n = self.n
        self._ev_count.synchronize()                 # recorded a window ago
        k = n - int(self._h_count.item())
        outs = [torch.empty((k,) + tuple(t.shape[1:]), dtype=t.dtype, device=t.device)
                for t in self.scene]
        rect = torch.empty(k, 4, dtype=torch.int32, device=self.rect_ref.device)
        if k < n:
            rtgs.compact_by_mask(self.mask, list(zip(self.scene, outs)) +
                                 [(self.rect_ref, rect)], self._kept)
            self.scene = tuple(outs)
            self.rect_ref = rect
            self.removed += n - k

    def _full(self, view, grads_fn):
        if self.mask is not None:
            self._remove_masked()
        R, cam = self.R, self.cam
        st = R.forward(self.scene, view, cam)
        rects = torch.empty(self.n, 4, dtype=torch.int32, device=view.device)
        rtgs.rtgs_tile_rects(st, rects)
        self._has_change = self.rect_ref is not None
        if self._has_change:
            rtgs.tile_pair_change(self.rect_ref, rects, None, self._change)
            self._h_change.copy_(self._change, non_blocking=True)
            self._ev_change.record()
        gc, gd = grads_fn(st)
        g = R.backward(self.scene, view, cam, st, gc, gd, pose=True, map_grads=False, score=True)
        budget = max(0.0, self.cfg.cap * self.n0 - self.removed)
        ratio_w = min(self.cfg.window_ratio, budget / max(self.n, 1), 0.5)
        mask = torch.zeros(self.n, dtype=torch.uint8, device=view.device)
        rtgs.prune_by_grad(R.handle, g["means"], g["cov3d"], st.visible, None, self.cfg.lam,
                           ratio_w, mask, self._count)
        self._h_count.copy_(self._count, non_blocking=True)
        self._ev_count.record()
        self.mask, self.ref, self.rect_ref = mask, st, rects
        self._pending = True
        self.full_iters += 1
        return g["pose"]

    def _masked(self, view, grads_fn):
        R, cam = self.R, self.cam
        st = R.forward(self.scene, view, cam, gauss_mask=self.mask, reuse_lists_of=self.ref)
        gc, gd = grads_fn(st)
        g = R.backward(self.scene, view, cam, st, gc, gd, pose=True, map_grads=False,
                       gauss_mask=self.mask)
        self.sched.step_masked()
        self.masked_iters += 1
        return g["pose"]
