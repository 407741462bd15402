"""torch.autograd.Function around render_fwd / render_bwd.

``render(means, log_scales, quats, opacity_logits, colors, viewmat, cam, ...)``
returns (color [3,H,W], depth [H,W], alpha [H,W]) and differentiates to the
five Gaussian parameter tensors and to the 12 entries of ``viewmat`` (3x4
world->camera).  The view-matrix gradient treats the entries as independent,
so any SE(3) parametrisation built in torch (e.g. ``pose.apply_left(xi, T0)``)
receives its exact gradient through autograd.

State between the passes, three policies (the paper's R&B buffer keeps
per-fragment results for the backward, Sec. 5.2):

* ``state="save"``: per pixel the final transmittance and the last blended
  list position (8 bytes per pixel); the backward recovers each fragment's
  transmittance and re-evaluates its alpha (Eq. 2);
* ``"fragments"``: that, and every blended fragment's alpha as the forward
  computed it (workspace proportional to the pairs: 2 KB per pair of
  capacity); the backward reads it instead of re-evaluating, with bitwise the
  same gradients;
* ``"recompute"``: nothing per pixel; the backward re-runs the forward
  compositing to rebuild the per-pixel state;
* ``"auto"``: save unless 8 B/pixel would exceed ``auto_budget`` of the free
  device memory.
"""
import torch

from . import rtgs

_renderers = {}


def default_renderer(device=None):
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _renderers:
        _renderers[dev] = rtgs.Renderer(dev, check="every")
    return _renderers[dev]


class RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, colors, viewmat, cam, renderer,
                gauss_mask, pixel_mask, state, need_cov3d):
        scene = tuple(t.detach().contiguous() for t in
                      (means, log_scales, quats, opacity_logits, colors))
        vm = viewmat.detach().contiguous()
        st = renderer.forward(scene, vm, cam, gauss_mask=gauss_mask, pixel_mask=pixel_mask,
                              save_state=state != "recompute",
                              save_fragments=state == "fragments")
        ctx.scene = scene
        ctx.vm = vm
        ctx.cam = cam
        ctx.renderer = renderer
        ctx.st = st
        ctx.gauss_mask = gauss_mask
        ctx.pixel_mask = pixel_mask
        ctx.need_cov3d = need_cov3d
        ctx.needs = (any(ctx.needs_input_grad[:5]), ctx.needs_input_grad[5])
        ctx.mark_non_differentiable(st.visible)
        return st.color, st.depth, st.alpha, st.visible

    @staticmethod
    def backward(ctx, g_color, g_depth, g_alpha, _g_visible):
        need_map, need_pose = ctx.needs
        st = ctx.st
        h, w = st.depth.shape
        dev = st.depth.device
        g_color = torch.zeros(3, h, w, device=dev) if g_color is None else g_color.contiguous()
        g_depth = torch.zeros(h, w, device=dev) if g_depth is None else g_depth.contiguous()
        if not (need_map or need_pose):
            return (None,) * 12
        g = ctx.renderer.backward(ctx.scene, ctx.vm, ctx.cam, st, g_color, g_depth,
                                  None if g_alpha is None else g_alpha.contiguous(),
                                  pose=need_pose, map_grads=need_map,
                                  cov3d=need_map and ctx.need_cov3d,
                                  gauss_mask=ctx.gauss_mask, pixel_mask=ctx.pixel_mask)
        ctx.renderer.last_grads = g
        out = [g.get("means"), g.get("log_scales"), g.get("quats"), g.get("opacity_logits"),
               g.get("colors"), g.get("viewmat")]
        return tuple(out) + (None,) * 6


def render(means, log_scales, quats, opacity_logits, colors, viewmat, cam, renderer=None,
           gauss_mask=None, pixel_mask=None, state="auto", auto_budget=0.05, need_cov3d=False):
    """Differentiable render; see the module docstring.  Returns
    (color, depth, alpha, visible).  With need_cov3d, the world-frame
    covariance gradient of the last backward is kept in
    ``renderer.last_grads["cov3d"]`` for prune_by_grad."""
    renderer = renderer or default_renderer(means.device.index)
    if state == "auto":
        free, _total = torch.cuda.mem_get_info(means.device)
        state = "save" if 8 * cam.width * cam.height <= auto_budget * free else "recompute"
    elif state not in ("save", "fragments", "recompute"):
        raise ValueError("state must be 'save', 'fragments', 'recompute' or 'auto'")
    vm = viewmat.reshape(3, 4)
    c, d, a, vis = RenderFn.apply(means, log_scales, quats, opacity_logits, colors, vm, cam,
                                  renderer, gauss_mask, pixel_mask, state, need_cov3d)
    return c, d, a, vis
