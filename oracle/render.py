"""The whole forward pass and its exact derivative (oracle; test infrastructure).

Forward: activation (Eq. 1) -> projection (Step 1-1) -> brute-force
compositing (Eqs. 2-3) for a set of pixels.

Backward (Steps 4 and 5, Rendering BP and Preprocessing BP): the paper's
Eq. (4) and Eq. (5) sketch the derivative of the blend with respect to each
alpha and the reverse transmittance recurrence; as printed they omit the T and
1/(1 - alpha) factors, so the reading used here is the exact derivative of the
forward above.  It is obtained by automatic differentiation of that forward in
float64 (the library routine is the derivative, no hand derivation), which is
then pinned against central finite differences.

Pose gradient: the forward is evaluated at T = (I + xi^) T0 with xi = 0, whose
derivative equals that of Exp(xi) T0 at xi = 0 (left perturbation, xi = (rho,
phi)); the tests pin it by finite differences of the true exponential.

`render_with_grads` also returns the gradients with respect to the 2D stage
values (u, v, a, b, c, o, colour, z) that Rendering BP hands to
Preprocessing BP, for stage-level comparisons.

Pins: tests/test_oracle_pins.py and tests/test_oracle_fd.py.
"""
import dataclasses

import torch

from .camera import apply_left_linear
from .composite import composite_pixels, depth_order
from .gaussians import activate
from .projection import project

F64 = torch.float64


def _t(x):
    return torch.as_tensor(x).to(F64)


@dataclasses.dataclass
class RenderOut:
    color: torch.Tensor    # [3,H,W] (or [3,P] for pixel lists)
    depth: torch.Tensor
    alpha: torch.Tensor
    final_t: torch.Tensor
    last_id: torch.Tensor
    n_blended: torch.Tensor
    flags: torch.Tensor
    proj: object = None


@dataclasses.dataclass
class Grads:
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    colors: torch.Tensor
    pose: torch.Tensor          # [6] (rho, phi)
    cov3d: torch.Tensor         # [N,3,3] dL/dSigma (world frame)
    viewmat: torch.Tensor       # [3,4] dL/d(view-matrix entries)
    stage2d: dict               # u, v, a, b, c, o, z: [N]; rgb: [N,3]


def _pixel_grid(w, h, pixels=None):
    if pixels is None:
        idx = torch.arange(w * h)
    else:
        idx = torch.as_tensor(pixels, dtype=torch.long)
    return idx, (idx % w).to(F64) + 0.5, (idx // w).to(F64) + 0.5


def _stage(params, viewmat, cam, gauss_mask, xi):
    means, log_scales, quats, opacity_logits, colors = params
    cov3d, opac = activate(log_scales, quats, opacity_logits)
    vm = apply_left_linear(xi, viewmat) if xi is not None else viewmat
    proj = project(means, cov3d, opac, vm, cam, gauss_mask)
    return cov3d, opac, proj


def _groups(idx, w, order, chunk, tile_lists):
    """Pixel groups and the fragment order each is composited in: chunks of
    `chunk` pixels in the global depth order, or, with tile_lists =
    (tile_w, tile_h, ranges [T, 2], ids), the pixels of each tile in that
    tile's list order (lists frozen at an earlier pose: the reuse of tile
    intersection and sorting across the iterations of a frame, Sec. 3,
    Observation 6)."""
    if tile_lists is None:
        for s in range(0, idx.numel(), chunk):
            yield torch.arange(s, min(s + chunk, idx.numel())), order
        return
    tw, th, ranges, ids = tile_lists
    ranges = torch.as_tensor(ranges, dtype=torch.long)
    ids = torch.as_tensor(ids, dtype=torch.long)
    tiles_x = (w + tw - 1) // tw
    tile = (idx // w) // th * tiles_x + (idx % w) // tw
    for t in torch.unique(tile).tolist():
        sel = torch.nonzero(tile == t).flatten()
        yield sel, ids[ranges[t, 0]:ranges[t, 1]]


def _active_pixels(idx, pixel_mask):
    if pixel_mask is None:
        return torch.ones_like(idx, dtype=torch.bool)
    return torch.as_tensor(pixel_mask).reshape(-1)[idx].bool()


def render(scene, viewmat, cam, gauss_mask=None, pixel_mask=None, pixels=None,
           chunk=2048, tile_lists=None, **band) -> RenderOut:
    """Forward only, in float64.  `scene` holds the five parameter arrays
    (float32 values are promoted exactly).  `pixels` optionally restricts the
    evaluation to a list of raster indices (j*W + i); masked pixels render as
    background with T_final = 1.  tile_lists: see _groups."""
    params = tuple(_t(x) for x in scene)
    vm = _t(viewmat)
    w, h = cam[0], cam[1]
    gm = None if gauss_mask is None else torch.as_tensor(gauss_mask)
    with torch.no_grad():
        _, opac, proj = _stage(params, vm, cam, gm, None)
        keep = torch.nonzero(proj.valid).flatten()
        order_local = depth_order(proj.z[keep])
        order = keep[order_local]
        idx, pxs, pys = _pixel_grid(w, h, pixels)
        act = _active_pixels(idx, pixel_mask)
        outs, sels = [], []
        for sel, order_g in _groups(idx, w, order, chunk, tile_lists):
            cp = composite_pixels(pxs[sel], pys[sel], proj.u, proj.v, proj.a, proj.b,
                                  proj.c, opac, proj.z, params[4], proj.valid,
                                  order_g, **band)
            outs.append(cp)
            sels.append(sel)
    color, depth, final_t, last_id, n_bl, flags = _scatter(outs, sels, idx.numel())
    a = act
    color = torch.where(a[:, None], color, torch.zeros_like(color))
    depth = torch.where(a, depth, torch.zeros_like(depth))
    final_t = torch.where(a, final_t, torch.ones_like(final_t))
    last_id = torch.where(a, last_id, torch.full_like(last_id, -1))
    n_bl = torch.where(a, n_bl, torch.zeros_like(n_bl))
    flags = flags & a
    shape = (h, w) if pixels is None else (idx.numel(),)
    return RenderOut(color.T.reshape((3,) + shape), depth.reshape(shape),
                     (1 - final_t).reshape(shape), final_t.reshape(shape),
                     last_id.reshape(shape), n_bl.reshape(shape),
                     flags.reshape(shape), proj)


def render_with_grads(scene, viewmat, cam, g_color, g_depth, g_alpha=None,
                      gauss_mask=None, pixel_mask=None, pixels=None, chunk=1024,
                      tile_lists=None, **band):
    """Forward plus the gradient of  L = sum(g_color C) + sum(g_depth D)
    + sum(g_alpha A)  with respect to every parameter and the pose.

    g_* have the shape of the outputs ([3,H,W] / [H,W], or [3,P] / [P] when
    `pixels` is given).  Returns (RenderOut, Grads)."""
    params = [_t(x).clone().requires_grad_(True) for x in scene]
    xi = torch.zeros(6, dtype=F64, requires_grad=True)
    vm = _t(viewmat).clone().requires_grad_(True)
    w, h = cam[0], cam[1]
    gm = None if gauss_mask is None else torch.as_tensor(gauss_mask)
    cov3d, opac, proj = _stage(params, vm, cam, gm, xi)
    cov3d.retain_grad()
    # 2D stage values become leaves for the compositing part
    leaves = {k: getattr(proj, k).detach().clone().requires_grad_(True)
              for k in ("u", "v", "a", "b", "c", "z")}
    leaves["o"] = opac.detach().clone().requires_grad_(True)
    leaves["rgb"] = params[4].detach().clone().requires_grad_(True)
    keep = torch.nonzero(proj.valid).flatten()
    order = keep[depth_order(proj.z.detach()[keep])]
    idx, pxs, pys = _pixel_grid(w, h, pixels)
    act = _active_pixels(idx, pixel_mask)
    gc = _t(g_color).reshape(3, -1).T
    gd = _t(g_depth).reshape(-1)
    ga = None if g_alpha is None else _t(g_alpha).reshape(-1)
    outs, sels = [], []
    for sl, order_g in _groups(idx, w, order, chunk, tile_lists):
        cp = composite_pixels(pxs[sl], pys[sl], leaves["u"], leaves["v"], leaves["a"],
                              leaves["b"], leaves["c"], leaves["o"], leaves["z"],
                              leaves["rgb"], proj.valid, order_g, **band)
        m = act[sl].to(F64)
        loss = ((cp.color * gc[sl]).sum(1) * m).sum() + (cp.depth * gd[sl] * m).sum()
        if ga is not None:
            loss = loss + (cp.alpha * ga[sl] * m).sum()
        if loss.requires_grad:
            loss.backward()
        outs.append(Composite_detached(cp))
        sels.append(sl)
    stage_grads = {k: (t.grad if t.grad is not None else torch.zeros_like(t))
                   for k, t in leaves.items()}
    # Preprocessing BP: push the 2D gradients back through the stage
    tensors = [proj.u, proj.v, proj.a, proj.b, proj.c, proj.z, opac, params[4]]
    grads = [stage_grads[k] for k in ("u", "v", "a", "b", "c", "z", "o", "rgb")]
    torch.autograd.backward(tensors, grads)
    color, depth, final_t, last_id, n_bl, flags = _scatter(outs, sels, idx.numel())
    color = torch.where(act[:, None], color, torch.zeros_like(color))
    depth = torch.where(act, depth, torch.zeros_like(depth))
    final_t = torch.where(act, final_t, torch.ones_like(final_t))
    last_id = torch.where(act, last_id, torch.full_like(last_id, -1))
    n_bl = torch.where(act, n_bl, torch.zeros_like(n_bl))
    flags = flags & act
    shape = (h, w) if pixels is None else (idx.numel(),)
    out = RenderOut(color.T.reshape((3,) + shape), depth.reshape(shape),
                    (1 - final_t).reshape(shape), final_t.reshape(shape),
                    last_id.reshape(shape), n_bl.reshape(shape),
                    flags.reshape(shape), proj)
    g = Grads(params[0].grad, params[1].grad, params[2].grad, params[3].grad,
              params[4].grad, xi.grad, cov3d.grad, vm.grad, stage_grads)
    return out, g


@dataclasses.dataclass
class Composite_detached:
    color: torch.Tensor
    depth: torch.Tensor
    final_t: torch.Tensor
    last_id: torch.Tensor
    n_blended: torch.Tensor
    flags: torch.Tensor

    def __init__(self, cp):
        self.color = cp.color.detach()
        self.depth = cp.depth.detach()
        self.final_t = cp.final_t.detach()
        self.last_id = cp.last_id
        self.n_blended = cp.n_blended
        self.flags = cp.flags


def _scatter(outs, sels, n):
    """Per-group composite outputs back to pixel order."""
    color = torch.zeros(n, 3, dtype=F64)
    depth = torch.zeros(n, dtype=F64)
    final_t = torch.ones(n, dtype=F64)
    last_id = torch.full((n,), -1, dtype=torch.long)
    n_bl = torch.zeros(n, dtype=torch.long)
    flags = torch.zeros(n, dtype=torch.bool)
    for o, sel in zip(outs, sels):
        color[sel] = o.color.detach()
        depth[sel] = o.depth.detach()
        final_t[sel] = o.final_t.detach()
        last_id[sel] = o.last_id
        n_bl[sel] = o.n_blended
        flags[sel] = o.flags
    return color, depth, final_t, last_id, n_bl, flags
