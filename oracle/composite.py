"""Steps 3-1 and 3-2: alpha computing and front-to-back blending, brute force
(oracle; test infrastructure).

For every pixel P (sample point (i + 0.5, j + 0.5)) and every Gaussian k,
with d = P - mu*_k and conic M_k = Sigma*_k^-1 (Eq. 2):

    alpha~_{P,k} = o_k exp(-1/2 d^T M_k d)

Fragments are visited in ascending view-space depth, ties by Gaussian index
(Step 2; one order serves every pixel because depth is per Gaussian).  The
blending rule (Eq. 3 with the constants read from the problem statement):

* alpha = min(0.99, alpha~); a fragment with alpha~ < 1/255 is skipped;
* T' = T (1 - alpha); if T' < 1e-4 the pixel stops and this fragment is
  not blended (the early termination of Sec. 2.1);
* otherwise w = alpha T, C += w c_k, D += w z_k, T = T'.

Outputs per pixel: colour C, depth D (expected depth, not normalised),
alpha A = 1 - T_final, T_final, the id of the last blended Gaussian and the
blended count.  Background is 0.

The sequential rule is written in closed form: T_{P,k} is the product of
(1 - alpha) over earlier fragments (Eq. 3), and since T never increases, the
fragments before the stop are exactly those whose inclusive product stays at or
above 1e-4.  No tiling, no culling by bounding boxes.

``ambiguity_flags`` marks pixels whose result float32 arithmetic could
legitimately decide differently: a fragment within a relative band of the
1/255 floor, of the 0.99 clamp or of the 1e-4 stop, or two fragments whose
depths are nearly equal.

Pins: tests/test_oracle_pins.py (single Gaussian closed form, two-Gaussian
order, five-of-K early stop, clamp and skip, invariants, colour linearity).
"""
import dataclasses

import torch

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4


@dataclasses.dataclass
class Composite:
    color: torch.Tensor      # [P,3]
    depth: torch.Tensor      # [P]
    alpha: torch.Tensor      # [P]
    final_t: torch.Tensor    # [P]
    last_id: torch.Tensor    # [P] int64, -1 if nothing blended
    n_blended: torch.Tensor  # [P] int64
    flags: torch.Tensor      # [P] bool, near a float32 decision boundary


def depth_order(z: torch.Tensor) -> torch.Tensor:
    """Indices sorted by (z, index): a stable sort on z."""
    return torch.sort(z.detach(), stable=True).indices


def composite_pixels(px, py, u, v, a, b, c, opacity, z, colors, valid, order,
                     band_alpha=1e-4, band_t=1e-4, band_z=1e-6) -> Composite:
    """Blend all Gaussians (in `order`) at sample points (px, py) [P]."""
    if order.numel() == 0:                 # nothing visible: background
        zero = px * 0.0
        none = torch.full(px.shape, -1, dtype=torch.long)
        return Composite(torch.stack([zero] * 3, 1) + 0.0 * colors.sum(), zero, zero,
                         zero + 1.0, none, none + 1, torch.zeros(px.shape, dtype=torch.bool))
    u, v, a, b, c = (t[order] for t in (u, v, a, b, c))
    o, zz, col, ok = opacity[order], z[order], colors[order], valid[order]
    dx = u[None, :] - px[:, None]
    dy = v[None, :] - py[:, None]
    quad = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy
    alpha_raw = o * torch.exp(-0.5 * quad)                        # Eq. (2)
    keep = ok[None, :] & (alpha_raw >= ALPHA_MIN)
    alpha = torch.where(keep, torch.clamp(alpha_raw, max=ALPHA_MAX),
                        torch.zeros_like(alpha_raw))
    t_incl = torch.cumprod(1.0 - alpha, dim=1)
    blended = keep & (t_incl >= T_MIN)
    alpha_b = torch.where(blended, alpha, torch.zeros_like(alpha))
    t_after = torch.cumprod(1.0 - alpha_b, dim=1)
    t_before = torch.cat([torch.ones_like(t_after[:, :1]), t_after[:, :-1]], 1)
    w = alpha_b * t_before                                         # Eq. (3)
    color = w @ col
    depth = w @ zz
    final_t = t_after[:, -1]
    n_blend = blended.sum(1)
    pos = torch.arange(blended.shape[1]).expand_as(blended)
    last_pos = torch.where(blended, pos, torch.full_like(pos, -1)).max(1).values
    last_id = torch.where(last_pos >= 0, order[last_pos.clamp(min=0)],
                          torch.full_like(last_pos, -1))
    with torch.no_grad():
        flags = _flags(alpha_raw, keep, t_incl, zz, ok, band_alpha, band_t, band_z)
    return Composite(color, depth, 1.0 - final_t, final_t, last_id, n_blend, flags)


def _flags(alpha_raw, keep, t_incl, z, ok, band_alpha, band_t, band_z):
    """Pixels where a float32 evaluation may take another discrete decision."""
    t_before = torch.cat([torch.ones_like(t_incl[:, :1]), t_incl[:, :-1]], 1)
    live = ok[None, :] & (t_before >= T_MIN * (1 - band_t))   # reached by the loop
    near_floor = live & ((alpha_raw * 255.0 - 1.0).abs() < band_alpha)
    near_clamp = live & keep & ((alpha_raw / ALPHA_MAX - 1.0).abs() < band_alpha)
    near_stop = live & keep & ((t_incl / T_MIN - 1.0).abs() < band_t)
    # depth near-ties between consecutive kept fragments before the stop
    rel = keep & live
    pos = torch.arange(rel.shape[1]).expand_as(rel)
    marked = torch.where(rel, pos, torch.full_like(pos, -1))
    prev = torch.cummax(marked, dim=1).values
    prev = torch.cat([torch.full_like(prev[:, :1], -1), prev[:, :-1]], 1)
    zprev = z[prev.clamp(min=0)]
    near_z = rel & (prev >= 0) & ((z[None, :] - zprev).abs() <= band_z * z[None, :])
    return (near_floor | near_clamp | near_stop | near_z).any(1)
