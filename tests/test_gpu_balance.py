"""Lanes assigned by previous work (RTGS_FWD_BALANCE_LANES, the GPU form of
the paper's workload scheduling unit, Sec. 5.2): a balanced forward renders
each pixel with exactly the arithmetic of the quadrant form (images bitwise
equal), writes the entries each sample walked, and the balanced backward's
gradients match the oracle and the quadrant form."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_06644_amd import rtgs, synth
from tests.gpu_util import (GRAD_TOL, MAP_GRADS, cam_tuple, dev_scene, eye_view, grad_err,
                            rcam, rel_err, say, view_from)

pytestmark = pytest.mark.gpu


def _walked_reference(r, dsc, dview, cam):
    """Entries walked per pixel from the statistics plane of a plain forward."""
    h, w = cam.height, cam.width
    ws = torch.empty(rtgs.rtgs_workspace_size(dsc[0].shape[0], w, h, r.cap), dtype=torch.uint8,
                     device="cuda")
    out = dict(scene=dsc, viewmat=dview, cam=rcam(cam), color=torch.empty(3, h, w, device="cuda"),
               depth=torch.empty(h, w, device="cuda"), alpha=torch.empty(h, w, device="cuda"),
               stats=torch.zeros(3, h, w, dtype=torch.int32, device="cuda"))
    rtgs.render_fwd_batched(r.handle, [out], ws, r.cap, flags=rtgs.RTGS_FWD_STATS)
    torch.cuda.synchronize()
    return out["stats"][1].cpu().numpy()


@pytest.mark.parametrize("name,xi", [("c0", None), ("c0", (37, 0.03, 2.0))])
def test_balanced_lanes_render_and_differentiate_like_the_quadrants(name, xi):
    say(f"test_balanced_lanes {name} posed={xi is not None}")
    spec = synth.CONFIGS[name]
    cam = synth.make_camera(spec.width, spec.height)
    sc = synth.make_scene(spec, cam)
    view = eye_view() if xi is None else view_from(synth.pose_offset(*xi))
    r = rtgs.Renderer(0, check="every")
    dsc = dev_scene(sc)
    dview = torch.from_numpy(view).cuda()
    h, w = cam.height, cam.width
    work0 = torch.zeros(h, w, dtype=torch.uint16, device="cuda")
    work1 = torch.zeros(h, w, dtype=torch.uint16, device="cuda")
    r.forward(dsc, dview, rcam(cam), balance=True, lane_work=None, lane_work_out=work0)
    bal = r.forward(dsc, dview, rcam(cam), balance=True, lane_work=work0, lane_work_out=work1)
    quad = r.forward(dsc, dview, rcam(cam))
    torch.cuda.synchronize()
    for k in ("color", "depth", "alpha", "final_T", "last_idx"):
        assert torch.equal(getattr(bal, k), getattr(quad, k)), k
    walked = _walked_reference(r, dsc, dview, cam)
    assert np.array_equal(work1.cpu().numpy().astype(np.int64), walked)
    assert np.array_equal(work0.cpu().numpy().astype(np.int64), walked)
    ref_f = oracle.render(sc.arrays(), view, cam_tuple(cam))
    keep = ~ref_f.flags.numpy()
    gc, gd, ga = synth.upstream_grads(w, h, 12)
    gc, gd, ga = gc * keep[None], gd * keep, ga * keep
    args = [torch.from_numpy(x).cuda() for x in (gc, gd, ga)]
    gb = r.backward(dsc, dview, rcam(cam), bal, *args)
    gq = r.backward(dsc, dview, rcam(cam), quad, *args)
    torch.cuda.synchronize()
    _, ref = oracle.render_with_grads(sc.arrays(), view, cam_tuple(cam), gc, gd, ga)
    for nm in MAP_GRADS:
        x, q, rr = gb[nm].cpu().numpy(), gq[nm].cpu().numpy(), getattr(ref, nm).numpy()
        e1, e2 = grad_err(x, rr), grad_err(x, q)
        say(f"  {nm}: vs oracle {e1:.2e}, vs quadrant lanes {e2:.2e}")
        assert e1 < GRAD_TOL and e2 < GRAD_TOL, nm
    assert rel_err(gb["pose"].cpu().numpy(), ref.pose.numpy()) < GRAD_TOL


def test_balanced_lanes_on_a_downsampled_frame():
    say("test_balanced_lanes_on_a_downsampled_frame")
    cam = synth.Camera(200, 120, 160.0, 160.0, 100.0, 60.0)
    sc = synth.make_scene(synth.SceneSpec("ds", 200, 120, 3000, 91), cam)
    view = view_from(synth.pose_offset(72, 0.02, 1.0))
    r = rtgs.Renderer(0, check="every")
    dsc = dev_scene(sc)
    dview = torch.from_numpy(view).cuda()
    full = r.forward(dsc, dview, rcam(cam))
    mask = torch.empty(120, 200, dtype=torch.uint8, device="cuda")
    rtgs.downsample_mask(full.final_T, 2, mask)
    work = torch.zeros(120, 200, dtype=torch.uint16, device="cuda")
    r.forward(dsc, dview, rcam(cam), pixel_mask=mask, sample_log2=2, balance=True,
              lane_work_out=work)
    bal = r.forward(dsc, dview, rcam(cam), pixel_mask=mask, sample_log2=2, balance=True,
                    lane_work=work)
    quad = r.forward(dsc, dview, rcam(cam), pixel_mask=mask, sample_log2=2)
    torch.cuda.synchronize()
    for k in ("color", "depth", "alpha", "final_T", "last_idx"):
        assert torch.equal(getattr(bal, k), getattr(quad, k)), k
    pm = mask.cpu().numpy()
    ref_f = oracle.render(sc.arrays(), view, cam_tuple(cam), pixel_mask=pm)
    keep = ~ref_f.flags.numpy()
    gc, gd, ga = synth.upstream_grads(200, 120, 13)
    gc, gd, ga = gc * keep[None], gd * keep, ga * keep
    g = r.backward(dsc, dview, rcam(cam), bal, *[torch.from_numpy(x).cuda() for x in (gc, gd, ga)],
                   pixel_mask=mask)
    torch.cuda.synchronize()
    _, ref = oracle.render_with_grads(sc.arrays(), view, cam_tuple(cam), gc, gd, ga, pixel_mask=pm)
    for nm in MAP_GRADS:
        assert grad_err(g[nm].cpu().numpy(), getattr(ref, nm).numpy()) < GRAD_TOL, nm
