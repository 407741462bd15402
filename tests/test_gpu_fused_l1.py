"""The loss gradient formed by the forward (rtgs_session.l1): for every pixel
the values loss_l1_grad computes from the forward's colour and depth, bit for
bit, and the float64 oracle of the loss to one rounding of its scale; the
image and saved state are those of a forward without it.  Full frames, a
pixel mask, a downsampled frame (sample blocks, background pixels), a batch
of three mixed sessions, a mapping loop whose parameters follow the unfused
loop exactly, and the argument checks."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_06644_amd import optim, pose, rtgs, synth
from tests.gpu_util import dev_scene, eye_view, rcam, say

pytestmark = pytest.mark.gpu


def _targets(h, w, seed, color=None, depth=None):
    g = torch.Generator(device="cuda").manual_seed(seed)
    tc = torch.rand(3, h, w, generator=g, device="cuda")
    td = 4 * torch.rand(h, w, generator=g, device="cuda")
    if color is not None:
        # some exact ties, where the gradient is sign(0) = 0
        tc[:, :4, :6] = color[:, :4, :6]
        td[:3, :5] = depth[:3, :5]
    return tc, td


def _mask(h, w, j, seed):
    ft = torch.rand(h, w, generator=torch.Generator().manual_seed(seed)).cuda()
    mask = torch.empty(h, w, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    rtgs.downsample_mask(ft, j, mask, cnt)
    return mask, cnt


def _check_session(color, depth, tc, td, gc, gd, mask, cnt, wc=1.0, wd=0.5):
    """gc, gd (from the forward) against loss_l1_grad on the same image
    (bitwise, signed zeros included) and against the oracle."""
    rc = torch.full_like(gc, float("nan"))
    rd = torch.full_like(gd, float("nan"))
    rtgs.loss_l1_grad(color, depth, tc, td, rc, rd, pixel_mask=mask, n_active=cnt,
                      w_color=wc, w_depth=wd)
    torch.cuda.synchronize()
    a = np.concatenate([gc.cpu().numpy().ravel(), gd.cpu().numpy().ravel()])
    b = np.concatenate([rc.cpu().numpy().ravel(), rd.cpu().numpy().ravel()])
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), "not bitwise the loss pass"
    m = None if mask is None else mask.cpu().numpy()
    # the oracle's loss weighs colour 1 and depth 0.5
    _, oc, od = oracle.l1_loss_grads(color.cpu().numpy(), depth.cpu().numpy(), tc.cpu().numpy(),
                                     td.cpu().numpy(), m)
    np.testing.assert_allclose(gc.cpu().numpy(), wc * oc.numpy(), rtol=2e-7, atol=0)
    np.testing.assert_allclose(gd.cpu().numpy(), (wd / 0.5) * od.numpy(), rtol=2e-7, atol=0)


@pytest.mark.parametrize("case", ["full", "masked", "downsampled"])
def test_forward_loss_gradient_equals_loss_pass(case):
    say(f"test_forward_loss_gradient_equals_loss_pass case={case}")
    spec = synth.CONFIGS["c0"]
    cam = synth.make_camera(spec.width, spec.height)
    scene = dev_scene(synth.make_scene(spec, cam))
    view = torch.from_numpy(eye_view()).cuda()
    h, w = cam.height, cam.width
    mask = cnt = None
    j = 0
    if case == "masked":
        mask = torch.from_numpy(
            (np.random.default_rng(8).random((h, w)) < 0.6).astype(np.uint8)).cuda()
        cnt = torch.tensor([int(mask.sum().item())], dtype=torch.int32, device="cuda")
    elif case == "downsampled":
        j = 2
        mask, cnt = _mask(h, w, j, 9)
    R = rtgs.Renderer(0)
    ref = R.forward(scene, view, rcam(cam), pixel_mask=mask, sample_log2=j)
    tc, td = _targets(h, w, 4, ref.color, ref.depth)
    st = R.forward(scene, view, rcam(cam), pixel_mask=mask, sample_log2=j, l1=(tc, td, cnt))
    torch.cuda.synchronize()
    for k in ("color", "depth", "alpha", "final_T", "last_idx"):
        assert torch.equal(getattr(st, k), getattr(ref, k)), k
    _check_session(st.color, st.depth, tc, td, st.dL_dcolor, st.dL_ddepth, mask, cnt)


def test_batched_sessions_each_get_their_loss_gradient():
    """Three sessions of one launch (two sizes, one downsampled, one with
    weights of its own), each against its own loss pass."""
    say("test_batched_sessions_each_get_their_loss_gradient")
    items, checks = [], []
    for k, (wd_, ht, n, j, wts) in enumerate([(200, 152, 3000, 0, (1.0, 0.5)),
                                               (160, 120, 2000, 2, (1.0, 0.5)),
                                               (200, 152, 2500, 0, (0.7, 1.3))]):
        spec = synth.SceneSpec(f"s{k}", wd_, ht, n, 40 + k)
        cam = synth.make_camera(wd_, ht)
        scene = dev_scene(synth.make_scene(spec, cam))
        mask = cnt = None
        if j:
            mask, cnt = _mask(ht, wd_, j, 50 + k)
        tc, td = _targets(ht, wd_, 60 + k)
        out = dict(scene=scene, viewmat=torch.from_numpy(eye_view()).cuda(), cam=rcam(cam),
                   pixel_mask=mask, sample_log2=j,
                   color=torch.empty(3, ht, wd_, device="cuda"),
                   depth=torch.empty(ht, wd_, device="cuda"),
                   alpha=torch.empty(ht, wd_, device="cuda"),
                   final_T=torch.empty(ht, wd_, device="cuda"),
                   last_idx=torch.empty(ht, wd_, dtype=torch.int32, device="cuda"))
        gc = torch.full((3, ht, wd_), float("nan"), device="cuda")
        gd = torch.full((ht, wd_), float("nan"), device="cuda")
        out["l1"] = rtgs.l1_loss(tc, td, gc, gd, cnt, *wts)
        items.append(out)
        checks.append((out, tc, td, gc, gd, mask, cnt, wts))
    ns = [it["scene"][0].shape[0] for it in items]
    cap = 1 << 18
    ws = torch.empty(rtgs.rtgs_workspace_size_batched(
        ns, [it["cam"].width for it in items], [it["cam"].height for it in items], cap),
        dtype=torch.uint8, device="cuda")
    rtgs.render_fwd_batched(rtgs.Renderer(0).handle, items, ws, cap)
    torch.cuda.synchronize()
    for out, tc, td, gc, gd, mask, cnt, wts in checks:
        _check_session(out["color"], out["depth"], tc, td, gc, gd, mask, cnt, *wts)


def test_mapping_loop_with_fused_loss_follows_the_unfused_loop():
    """Forward with the loss gradient + backward with the fused Adam update,
    against forward, loss pass, backward and adam_step: the same parameters
    and moments, bitwise, over three iterations."""
    say("test_mapping_loop_with_fused_loss_follows_the_unfused_loop")
    spec = synth.CONFIGS["c0"]
    cam = synth.make_camera(spec.width, spec.height)
    sc = synth.make_scene(spec, cam)
    view = torch.from_numpy(eye_view()).cuda()
    rc = rcam(cam)
    R = rtgs.Renderer(0)
    tgt = R.forward(dev_scene(synth.perturb_scene(sc, 31)), view, rc)
    tc, td = tgt.color.clone(), tgt.depth.clone()
    sep = [p.clone() for p in dev_scene(sc)]
    fus = [p.clone() for p in dev_scene(sc)]
    opt_s, opt_f = optim.MapAdam(sep), optim.MapAdam(fus)
    for it in range(3):
        st = R.forward(tuple(sep), view, rc)
        gc = torch.empty_like(st.color)
        gd = torch.empty_like(st.depth)
        rtgs.loss_l1_grad(st.color, st.depth, tc, td, gc, gd)
        gs = R.backward(tuple(sep), view, rc, st, gc, gd, pose=False)
        opt_s.step(R.handle, [gs[k] for k in ("means", "log_scales", "quats", "opacity_logits",
                                             "colors")])
        sf = R.forward(tuple(fus), view, rc, l1=(tc, td, None))
        R.backward(tuple(fus), view, rc, sf, sf.dL_dcolor, sf.dL_ddepth, pose=False, adam=opt_f)
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(sep, fus)):
            assert torch.equal(a, b), f"iteration {it}: parameter {k}"
            assert torch.equal(opt_s.exp_avg[k], opt_f.exp_avg[k]), f"iteration {it}: m {k}"
        say(f"  iteration {it}: bitwise equal")


def test_forward_loss_gradient_argument_checks():
    say("test_forward_loss_gradient_argument_checks")
    spec = synth.CONFIGS["c0"]
    cam = synth.make_camera(spec.width, spec.height)
    scene = dev_scene(synth.make_scene(spec, cam))
    view = torch.from_numpy(eye_view()).cuda()
    h, w = cam.height, cam.width
    R = rtgs.Renderer(0)
    tc, td = _targets(h, w, 5)
    mask = torch.ones(h, w, dtype=torch.uint8, device="cuda")
    with pytest.raises(rtgs.RtgsError) as e:        # a mask needs the device count
        R.forward(scene, view, rcam(cam), pixel_mask=mask, l1=(tc, td, None))
    assert e.value.code == rtgs.RTGS_ERR_INVALID_ARG
    with pytest.raises(rtgs.RtgsError) as e:        # weights must be finite
        R.forward(scene, view, rcam(cam), l1=(tc, td, None, float("inf"), 0.5))
    assert e.value.code == rtgs.RTGS_ERR_INVALID_ARG
    gc, gd = torch.empty(3, h, w, device="cuda"), torch.empty(h, w, device="cuda")
    bad = rtgs.l1_loss(tc, td, gc, gd)
    bad.dL_ddepth = None                              # a null output array
    out = dict(scene=scene, viewmat=view, cam=rcam(cam), color=torch.empty(3, h, w, device="cuda"),
               depth=torch.empty(h, w, device="cuda"), alpha=torch.empty(h, w, device="cuda"),
               l1=bad)
    cap = 1 << 16
    ws = torch.empty(rtgs.rtgs_workspace_size(scene[0].shape[0], w, h, cap), dtype=torch.uint8,
                     device="cuda")
    with pytest.raises(rtgs.RtgsError) as e:
        rtgs.render_fwd_batched(R.handle, [out], ws, cap, flags=0)
    assert e.value.code == rtgs.RTGS_ERR_INVALID_ARG


def test_forward_loss_gradient_on_reused_lists():
    """A forward on the tile lists of an earlier one (another pose) also
    writes the loss gradient of its own image."""
    say("test_forward_loss_gradient_on_reused_lists")
    spec = synth.CONFIGS["c0"]
    cam = synth.make_camera(spec.width, spec.height)
    scene = dev_scene(synth.make_scene(spec, cam))
    R = rtgs.Renderer(0)
    ref = R.forward(scene, torch.from_numpy(eye_view()).cuda(), rcam(cam))
    xi = torch.tensor(synth.pose_offset(3, 0.01, 0.5), dtype=torch.float32, device="cuda")
    view = pose.apply_left(xi, torch.from_numpy(eye_view()).cuda()).contiguous()
    plain = R.forward(scene, view, rcam(cam), reuse_lists_of=ref)
    tc, td = _targets(cam.height, cam.width, 7, plain.color, plain.depth)
    st = R.forward(scene, view, rcam(cam), reuse_lists_of=ref, l1=(tc, td, None))
    torch.cuda.synchronize()
    for k in ("color", "depth", "final_T", "last_idx"):
        assert torch.equal(getattr(st, k), getattr(plain, k)), k
    _check_session(st.color, st.depth, tc, td, st.dL_dcolor, st.dL_ddepth, None, None)
