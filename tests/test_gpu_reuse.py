"""Reuse of tile intersection and sorting across the iterations of a frame
(RTGS_FWD_REUSE_LISTS; Sec. 3, Observation 6) on the GPU.

Parity notion: the lists are frozen at the reference iteration.  The oracle
composites each pixel through its tile's reference list, in the reference
order, with the Gaussians projected at the current pose (oracle render with
`tile_lists`); images and gradients are compared at 1e-4 as elsewhere.  The
reference lists are the oracle's float32 replay of the reference forward's
stage values, checked bit for bit against the kernel's."""
import numpy as np
import pytest
import torch

import oracle
from oracle import binning
from paper_2510_06644_amd import rtgs, synth
from tests.gpu_util import (GRAD_TOL, IMG_TOL, cam_tuple, dev_scene, eye_view, grad_err, rcam, rel_err,
                            say, view_from)

pytestmark = pytest.mark.gpu


def _setup():
    spec = synth.CONFIGS["c0"]
    cam = synth.make_camera(spec.width, spec.height)
    sc = synth.make_scene(spec, cam)
    return sc, cam


@pytest.mark.parametrize("move", [(0.0, 0.0), (0.004, 0.3)])
def test_reuse_lists_matches_frozen_list_oracle(move):
    say(f"test_reuse_lists_matches_frozen_list_oracle move={move}")
    sc, cam = _setup()
    r = rtgs.Renderer(0, check="every")
    dsc = dev_scene(sc)
    ref_view = eye_view()
    st0 = r.forward(dsc, torch.from_numpy(ref_view).cuda(), rcam(cam))
    torch.cuda.synchronize()
    dbg = st0.stage()
    stg = dbg["stage"]
    proj0 = oracle.render(sc.arrays(), ref_view, cam_tuple(cam), pixels=[0]).proj
    ranges, ids = binning.tile_lists(stg[:, 0], stg[:, 1], stg[:, 7], stg[:, 8], stg[:, 6],
                                     proj0.valid.numpy(), cam.width, cam.height)
    assert np.array_equal(dbg["ranges"], ranges) and np.array_equal(dbg["ids"], ids)
    color0 = st0.color.clone()
    # the next iteration of the frame: the pose has moved a little
    view = view_from(synth.pose_offset(77, *move)) if move[0] > 0 else ref_view
    dview = torch.from_numpy(np.ascontiguousarray(view, dtype=np.float32)).cuda()
    st = r.forward(dsc, dview, rcam(cam), reuse_lists_of=st0)
    torch.cuda.synchronize()
    if move[0] == 0:
        assert torch.equal(st.color, color0)   # same pose: the same lists, the same image
    lists = (16, 16, ranges, ids)
    ref = oracle.render(sc.arrays(), view, cam_tuple(cam), tile_lists=lists)
    keep = ~ref.flags.numpy()
    say(f"  flagged {int((~keep).sum())}")
    assert keep.mean() > 0.995
    assert rel_err(st.color.cpu().numpy(), ref.color.numpy(), keep) < IMG_TOL
    assert rel_err(st.depth.cpu().numpy(), ref.depth.numpy(), keep) < IMG_TOL
    assert rel_err(st.final_T.cpu().numpy(), ref.final_t.numpy(), keep) < IMG_TOL
    # backward through the frozen lists
    gc, gd, ga = synth.upstream_grads(cam.width, cam.height, 3)
    gc, gd, ga = gc * keep[None], gd * keep, ga * keep
    g = r.backward(dsc, dview, rcam(cam), st, torch.from_numpy(gc).cuda(),
                   torch.from_numpy(gd).cuda(), torch.from_numpy(ga).cuda())
    torch.cuda.synchronize()
    _, rg = oracle.render_with_grads(sc.arrays(), view, cam_tuple(cam), gc, gd, ga,
                                     tile_lists=lists)
    for name in ("means", "log_scales", "quats", "opacity_logits", "colors", "pose"):
        e = grad_err(g[name].cpu().numpy(), getattr(rg, name).numpy())
        say(f"  {name}: {e:.2e}")
        assert e < GRAD_TOL, name


def test_reuse_lists_rejects_other_geometry():
    say("test_reuse_lists_rejects_other_geometry")
    sc, cam = _setup()
    r = rtgs.Renderer(0)
    dsc = dev_scene(sc)
    st0 = r.forward(dsc, torch.from_numpy(eye_view()).cuda(), rcam(cam))
    small = rtgs.Cam(cam.width // 2, cam.height // 2, cam.fx, cam.fy, cam.cx, cam.cy)
    with pytest.raises(ValueError):
        r.forward(dsc, torch.from_numpy(eye_view()).cuda(), small, reuse_lists_of=st0)
