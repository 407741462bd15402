"""Tracking / mapping loss (oracle; test infrastructure).

Eq. (6) weighs a photometric and a geometric residual.  Reading used here
(the design doc): L1 colour plus 0.5 times L1 depth, each a mean over the active
pixels Omega:  L = sum|C - C^| / (3|Omega|) + 0.5 sum|D - D^| / |Omega|,
with sign(0) = 0 in the gradient.
"""
import torch


def l1_loss_grads(color, depth, target_color, target_depth, pixel_mask=None):
    """(L, dL/dC [3,H,W], dL/dD [H,W]) in float64."""
    c = torch.as_tensor(color, dtype=torch.float64)
    d = torch.as_tensor(depth, dtype=torch.float64)
    tc = torch.as_tensor(target_color, dtype=torch.float64)
    td = torch.as_tensor(target_depth, dtype=torch.float64)
    m = (torch.ones_like(d) if pixel_mask is None
         else torch.as_tensor(pixel_mask).to(torch.float64))
    n = m.sum().clamp(min=1.0)
    loss = ((c - tc).abs() * m).sum() / (3 * n) + 0.5 * ((d - td).abs() * m).sum() / n
    gc = torch.sign(c - tc) * m / (3 * n)
    gd = 0.5 * torch.sign(d - td) * m / n
    return loss, gc, gd
