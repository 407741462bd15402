"""GPU parity of render_fwd / render_bwd against the float64 oracle at the small
configuration (128x128, 2,000 Gaussians) and on hand-built edge cases.

Stage values within tolerance; tile lists and depth order bit-exact (oracle
replay on the kernel's float32 stage values); images and gradients within
1e-4 relative.  Pixels the oracle flags as near a float32 decision boundary
are left out of element-wise image comparisons, and their upstream gradient
is zeroed on both sides for the gradient comparisons (the backward is linear
in it)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import binning
from paper_2510_06644_amd import rtgs, synth
from tests.gpu_util import (GRAD_TOL, IMG_TOL, cam_tuple, dev_scene, eye_view, grad_err,
                            norm_err, rcam, rel_err, say, view_from)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def renderer():
    return rtgs.Renderer(0, check="every")


def _case(name="c0", xi=None, n=None, cam=None, seed=None):
    spec = synth.CONFIGS[name]
    cam = cam or synth.make_camera(spec.width, spec.height)
    sc = synth.make_scene(spec, cam, n=n, seed=seed)
    view = eye_view() if xi is None else view_from(xi)
    return sc, cam, view


def test_wave_sum_selftest():
    say("test_wave_sum_selftest")
    g = torch.Generator().manual_seed(0)
    # distinct magnitudes per value so that a value landing in another
    # value's slot cannot pass
    scale = 10.0 ** torch.arange(10, dtype=torch.float32)[None, :, None] / 1e5
    x = (torch.randn(37, 10, 64, generator=g) + 3.0) * scale
    out = torch.full((37 * 10,), float("nan")).cuda()
    rtgs.rtgs_selftest_wave_sum(x.reshape(-1).cuda(), out)
    torch.cuda.synchronize()
    want = x.double().sum(2).reshape(-1)
    assert torch.allclose(out.double().cpu(), want, rtol=1e-5, atol=0)


@pytest.mark.parametrize("posed", [False, True])
def test_forward_stages_lists_and_images_c0(renderer, posed):
    say(f"test_forward c0 posed={posed}")
    xi = synth.pose_offset(31, 0.05, 3.0) if posed else None
    sc, cam, view = _case("c0", xi)
    dsc = dev_scene(sc)
    st = renderer.forward(dsc, torch.from_numpy(view).cuda(), rcam(cam))
    torch.cuda.synchronize()
    dbg = st.stage()
    stg = dbg["stage"]
    # stage values against the float64 projection
    ref = oracle.render(sc.arrays(), view, cam_tuple(cam))
    p = ref.proj
    valid = p.valid.numpy()
    o = 1 / (1 + np.exp(-sc.opacity_logits.astype(np.float64)))
    t = 2 * np.log(np.maximum(255 * o, 1.0))
    ex = np.sqrt(t * p.cov2d[:, 0, 0].numpy())
    assert valid.sum() > 0.9 * len(valid)
    v = valid
    assert np.abs(stg[v, 0] - p.u.numpy()[v]).max() < 1e-4 * max(cam.width, 1)
    assert rel_err(stg[v, 2], p.a.numpy()[v]) < 1e-6
    assert rel_err(stg[v, 3], p.b.numpy()[v]) < 1e-5
    assert rel_err(stg[v, 4], p.c.numpy()[v]) < 1e-6
    assert rel_err(stg[v, 6], p.z.numpy()[v]) < 1e-6
    assert rel_err(stg[v, 7], ex[v]) < 1e-6
    # tile lists: bit-exact against the replay on the kernel's float32 values
    ranges, ids = binning.tile_lists(stg[:, 0], stg[:, 1], stg[:, 7], stg[:, 8], stg[:, 6],
                                     valid, cam.width, cam.height)
    assert np.array_equal(dbg["ranges"], ranges)
    assert np.array_equal(dbg["ids"], ids)
    assert np.array_equal(st.visible.cpu().numpy().astype(bool),
                          binning.tile_rects(stg[:, 0], stg[:, 1], stg[:, 7], stg[:, 8], valid,
                                             cam.width, cam.height)[2] >=
                          binning.tile_rects(stg[:, 0], stg[:, 1], stg[:, 7], stg[:, 8], valid,
                                             cam.width, cam.height)[0])
    # images
    flags = ref.flags.numpy()
    keep = ~flags
    say(f"  flagged pixels {flags.sum()} of {flags.size}")
    assert flags.mean() < 0.002
    col = st.color.cpu().numpy()
    assert rel_err(col, ref.color.numpy(), keep) < IMG_TOL
    assert rel_err(st.depth.cpu().numpy(), ref.depth.numpy(), keep) < IMG_TOL
    assert rel_err(st.alpha.cpu().numpy(), ref.alpha.numpy(), keep) < IMG_TOL
    assert rel_err(st.final_T.cpu().numpy(), ref.final_t.numpy(), keep) < IMG_TOL
    assert norm_err(col, ref.color.numpy()) < IMG_TOL
    # last contributor: position in the sorted list -> Gaussian id
    last = st.last_idx.cpu().numpy()
    gid = np.where(last >= 0, dbg["ids"][np.maximum(last, 0)], -1)
    assert np.array_equal(gid[keep], ref.last_id.numpy()[keep])


def _grad_case(renderer, sc, cam, view, seed=7, pixel_mask=None, gauss_mask=None, pose=True,
               map_grads=True, alpha_grad=True):
    dsc = dev_scene(sc)
    dview = torch.from_numpy(view).cuda()
    pm = None if pixel_mask is None else torch.from_numpy(pixel_mask).cuda()
    gm = None if gauss_mask is None else torch.from_numpy(gauss_mask).cuda()
    st = renderer.forward(dsc, dview, rcam(cam), gauss_mask=gm, pixel_mask=pm)
    ref_f = oracle.render(sc.arrays(), view, cam_tuple(cam), gauss_mask=gauss_mask,
                          pixel_mask=pixel_mask)
    keep = ~ref_f.flags.numpy()
    gc, gd, ga = synth.upstream_grads(cam.width, cam.height, seed)
    gc, gd, ga = gc * keep[None], gd * keep, ga * keep
    if not alpha_grad:
        ga = None
    grads = renderer.backward(dsc, dview, rcam(cam), st, torch.from_numpy(gc).cuda(),
                              torch.from_numpy(gd).cuda(),
                              None if ga is None else torch.from_numpy(ga).cuda(),
                              pose=pose, map_grads=map_grads, cov3d=map_grads, gauss_mask=gm,
                              pixel_mask=pm)
    torch.cuda.synchronize()
    _, ref = oracle.render_with_grads(sc.arrays(), view, cam_tuple(cam), gc, gd, ga,
                                      gauss_mask=gauss_mask, pixel_mask=pixel_mask)
    return {k: v.cpu().numpy() for k, v in grads.items()}, ref, keep


def _cov6(m):
    m = m.numpy()
    return np.stack([m[:, 0, 0], m[:, 0, 1], m[:, 0, 2], m[:, 1, 1], m[:, 1, 2], m[:, 2, 2]], 1)


@pytest.mark.parametrize("posed,alpha_grad,with_pose", [(False, True, True), (True, True, True),
                                                        (True, False, True), (False, True, False),
                                                        (True, True, False)])
def test_backward_all_gradients_c0(renderer, posed, alpha_grad, with_pose):
    # alpha_grad: with and without an alpha-image gradient (the kernel
    # leaves that term out when no session passes one); with_pose: the map
    # gradients with the pose gradient or alone
    say(f"test_backward c0 posed={posed} alpha_grad={alpha_grad} with_pose={with_pose}")
    xi = synth.pose_offset(32, 0.05, 3.0) if posed else None
    sc, cam, view = _case("c0", xi)
    g, ref, keep = _grad_case(renderer, sc, cam, view, alpha_grad=alpha_grad, pose=with_pose)
    pairs = [("means", ref.means), ("log_scales", ref.log_scales), ("quats", ref.quats),
             ("opacity_logits", ref.opacity_logits), ("colors", ref.colors)]
    for name, r in pairs:
        e1, e2 = grad_err(g[name], r.numpy()), norm_err(g[name], r.numpy())
        say(f"  {name}: rel {e1:.2e} norm {e2:.2e}")
        assert e1 < GRAD_TOL and e2 < GRAD_TOL, name
    e1 = rel_err(g["cov3d"], _cov6(ref.cov3d))
    say(f"  cov3d: rel {e1:.2e}")
    assert e1 < GRAD_TOL
    if not with_pose:
        return
    e1, e2 = rel_err(g["pose"], ref.pose.numpy()), norm_err(g["pose"], ref.pose.numpy())
    say(f"  pose: rel {e1:.2e} norm {e2:.2e}  {g['pose']}  {ref.pose.numpy()}")
    assert e1 < GRAD_TOL and e2 < GRAD_TOL
    e1 = rel_err(g["viewmat"], ref.viewmat.numpy())
    say(f"  viewmat: rel {e1:.2e}")
    assert e1 < GRAD_TOL


def test_backward_pose_only_matches_full(renderer):
    say("test_backward_pose_only")
    sc, cam, view = _case("c0", synth.pose_offset(33, 0.02, 1.0))
    g, ref, _ = _grad_case(renderer, sc, cam, view, map_grads=False, alpha_grad=False)
    assert set(g) == {"pose", "viewmat"}
    assert rel_err(g["pose"], ref.pose.numpy()) < GRAD_TOL


def test_ragged_image_masks_and_recompute(renderer):
    say("test_ragged_image_masks_and_recompute")
    cam = synth.Camera(100, 70, 80.0, 80.0, 50.0, 35.0)
    spec = synth.SceneSpec("ragged", 100, 70, 900, 4321)
    sc = synth.make_scene(spec, cam)
    view = view_from(synth.pose_offset(34, 0.03, 2.0))
    rng = np.random.default_rng(5)
    pm = (rng.random((70, 100)) < 0.6).astype(np.uint8)
    gm = (rng.random(900) < 0.2).astype(np.uint8)
    g, ref, keep = _grad_case(renderer, sc, cam, view, pixel_mask=pm, gauss_mask=gm)
    for name in ("means", "log_scales", "quats", "opacity_logits", "colors"):
        assert grad_err(g[name], getattr(ref, name).numpy()) < GRAD_TOL, name
    assert np.all(g["means"][gm.astype(bool)] == 0)
    assert rel_err(g["pose"], ref.pose.numpy()) < GRAD_TOL
    # forward without saved state, backward recomputes it
    dsc = dev_scene(sc)
    dview = torch.from_numpy(view).cuda()
    st = renderer.forward(dsc, dview, rcam(cam), pixel_mask=torch.from_numpy(pm).cuda(),
                          gauss_mask=torch.from_numpy(gm).cuda(), save_state=False)
    ref_f = oracle.render(sc.arrays(), view, cam_tuple(cam), gauss_mask=gm, pixel_mask=pm)
    k = ~ref_f.flags.numpy()
    assert rel_err(st.color.cpu().numpy(), ref_f.color.numpy(), k) < IMG_TOL
    assert np.all(st.color.cpu().numpy()[:, pm == 0] == 0)
    gc, gd, ga = synth.upstream_grads(100, 70, 7)
    gc, gd, ga = gc * k[None], gd * k, ga * k
    g2 = renderer.backward(dsc, dview, rcam(cam), st, torch.from_numpy(gc).cuda(),
                           torch.from_numpy(gd).cuda(), torch.from_numpy(ga).cuda(),
                           pixel_mask=torch.from_numpy(pm).cuda(),
                           gauss_mask=torch.from_numpy(gm).cuda())
    assert grad_err(g2["means"].cpu().numpy(), ref.means.numpy()) < GRAD_TOL


def test_empty_and_fully_culled_scenes(renderer):
    say("test_empty_and_fully_culled_scenes")
    cam = synth.Camera(40, 24, 32.0, 32.0, 20.0, 12.0)
    empty = synth.Scene(*(np.zeros(s, np.float32) for s in ((0, 3), (0, 3), (0, 4), (0,), (0, 3))))
    st = renderer.forward(dev_scene(empty), torch.from_numpy(eye_view()).cuda(), rcam(cam))
    torch.cuda.synchronize()
    assert st.color.abs().max().item() == 0 and st.final_T.min().item() == 1.0
    assert (st.last_idx == -1).all()
    behind = synth.make_scene(synth.SceneSpec("b", 40, 24, 50, 9), cam)
    behind.means[:, 2] = -1.0       # all behind the camera
    st = renderer.forward(dev_scene(behind), torch.from_numpy(eye_view()).cuda(), rcam(cam))
    g = renderer.backward(dev_scene(behind), torch.from_numpy(eye_view()).cuda(), rcam(cam), st,
                          torch.ones(3, 24, 40).cuda(), torch.ones(24, 40).cuda())
    torch.cuda.synchronize()
    assert st.alpha.abs().max().item() == 0 and st.visible.sum().item() == 0
    assert g["means"].abs().max().item() == 0 and g["pose"].abs().max().item() == 0


def test_capacity_overflow_is_reported_then_recovers():
    say("test_capacity_overflow")
    sc, cam, view = _case("c0")
    r = rtgs.Renderer(0, check="deferred", pairs_per_gaussian=0.1, min_capacity=256)
    dsc = dev_scene(sc)
    st = r.forward(dsc, torch.from_numpy(view).cuda(), rcam(cam))
    code, pairs, _ = rtgs.rtgs_query(r.handle, True)
    assert code == rtgs.RTGS_ERR_CAPACITY and pairs > st.cap
    r.grow(pairs)
    st2 = r.forward(dsc, torch.from_numpy(view).cuda(), rcam(cam))
    assert r.verify() == pairs
    ref = oracle.render(sc.arrays(), view, cam_tuple(cam))
    keep = ~ref.flags.numpy()
    assert rel_err(st2.color.cpu().numpy(), ref.color.numpy(), keep) < IMG_TOL


def test_backward_gaussians_touching_many_tiles(renderer):
    """Per-Gaussian gradients when some Gaussians cover most of a 40 x 32 tile
    frame: six such Gaussians in one merge workgroup (32 consecutive indices;
    the merge hands each one to the whole workgroup), one alone in another
    workgroup, and some with a few hundred tiles (summed by their own lanes);
    dense upstream gradients."""
    say("test_backward_gaussians_touching_many_tiles")
    cam = synth.make_camera(640, 512)
    rng = np.random.default_rng(21)
    n = 400
    z = rng.uniform(2.0, 6.0, n)
    u = rng.uniform(0, 640, n)
    v = rng.uniform(0, 512, n)
    sig_px = rng.uniform(3.0, 8.0, n)
    logit = rng.uniform(-1.0, 2.0, n)
    big = np.r_[0:6, 70]        # 0-5 in workgroup 0, 70 alone in workgroup 2
    mid = np.r_[40:44]
    u[big], v[big], sig_px[big], logit[big] = 320, 256, 150.0, -3.0
    z[big] = 3.4 + 0.2 * np.arange(len(big))    # distinct depths: no order ties
    sig_px[mid], logit[mid] = 40.0, -2.0
    means = np.stack([(u - cam.cx) * z / cam.fx, (v - cam.cy) * z / cam.fy, z], 1)
    log_s = np.log(sig_px * z / cam.fx)[:, None] + rng.uniform(-0.2, 0.2, (n, 3))
    q = rng.normal(size=(n, 4))
    sc = synth.Scene(means.astype(np.float32), log_s.astype(np.float32),
                     (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(np.float32),
                     logit.astype(np.float32), rng.random((n, 3)).astype(np.float32))
    view = eye_view()
    st = renderer.forward(dev_scene(sc), torch.from_numpy(view).cuda(), rcam(cam))
    dbg = st.stage()
    stg = dbg["stage"]
    _, ids = binning.tile_lists(stg[:, 0], stg[:, 1], stg[:, 7], stg[:, 8], stg[:, 6],
                                np.ones(n, bool), cam.width, cam.height)
    slots = np.bincount(ids, minlength=n)
    say(f"  slots: big {slots[big].min()}..{slots[big].max()}, "
        f"mid {slots[mid].min()}..{slots[mid].max()}, others max {np.delete(slots, np.r_[big, mid]).max()}")
    assert slots[big].min() > 1024 and 128 < slots[mid].min() and slots[mid].max() <= 1024
    g, ref, _ = _grad_case(renderer, sc, cam, view)
    for name in ("means", "log_scales", "quats", "opacity_logits", "colors"):
        r = getattr(ref, name).numpy()
        e1, e2 = grad_err(g[name], r), norm_err(g[name], r)
        say(f"  {name}: rel {e1:.2e} norm {e2:.2e}")
        assert e1 < GRAD_TOL and e2 < GRAD_TOL, name
    assert rel_err(g["pose"], ref.pose.numpy()) < GRAD_TOL


@pytest.mark.parametrize("n,span,lo,hi", [(900, 8, 700, 1024), (2500, 8, 1025, 4096),
                                          (6000, 8, 4097, 8192), (9000, 8, 8193, 10 ** 9),
                                          (9000, 24, 1025, 4096)])
def test_long_tile_lists_take_each_sort_path(renderer, n, span, lo, hi):
    # n small Gaussians over a span x span pixel square from (4, 4): one tile
    # (span 8) or four (span 24); the longest list selects the path: the
    # one-workgroup merge sort (<= 1024 keys), the queued 1024-thread merge
    # sort (<= 4096), the 8-keys-per-thread merge sort (<= 8192) or the
    # in-place global sort
    say(f"test_long_tile_lists n={n} span={span}")
    cam = synth.Camera(32, 32, 25.6, 25.6, 16.0, 16.0)
    rng = np.random.default_rng(8)
    z = rng.uniform(1, 3, n)
    u = rng.uniform(4, 4 + span, n)
    v = rng.uniform(4, 4 + span, n)
    means = np.stack([(u - 16) * z / 25.6, (v - 16) * z / 25.6, z], 1)
    sc = synth.Scene(means.astype(np.float32), np.full((n, 3), -5.5, np.float32),
                     np.tile(np.float32([1, 0, 0, 0]), (n, 1)),
                     np.full(n, -4.0, np.float32), rng.random((n, 3)).astype(np.float32))
    st = renderer.forward(dev_scene(sc), torch.from_numpy(eye_view()).cuda(), rcam(cam))
    dbg = st.stage()
    stg = dbg["stage"]
    valid = np.ones(n, bool)
    ranges, ids = binning.tile_lists(stg[:, 0], stg[:, 1], stg[:, 7], stg[:, 8], stg[:, 6],
                                     valid, 32, 32)
    longest = (ranges[:, 1] - ranges[:, 0]).max()
    say(f"  longest list {longest}")
    assert lo <= longest <= hi
    assert np.array_equal(dbg["ranges"], ranges)
    assert np.array_equal(dbg["ids"], ids)
    ref = oracle.render(sc.arrays(), eye_view(), cam_tuple(cam))
    keep = ~ref.flags.numpy()
    assert rel_err(st.color.cpu().numpy(), ref.color.numpy(), keep) < IMG_TOL


@pytest.mark.parametrize("n,lo,hi", [(900, 700, 1024), (2500, 1025, 4096), (6000, 4097, 8192),
                                     (9000, 8193, 10 ** 9)])
def test_long_tile_lists_with_depth_ties_on_each_sort_path(renderer, n, lo, hi):
    """As above, with every Gaussian at one of three exactly equal depths: the
    lists are ordered by depth, then by Gaussian index (Step 2), on every sort
    path, bit for bit."""
    say(f"test_long_tile_lists_with_depth_ties n={n}")
    cam = synth.Camera(32, 32, 25.6, 25.6, 16.0, 16.0)
    rng = np.random.default_rng(9)
    z = rng.choice(np.float32([1.5, 2.0, 2.5]), n)
    u = rng.uniform(4, 12, n)
    v = rng.uniform(4, 12, n)
    means = np.stack([(u - 16) * z / 25.6, (v - 16) * z / 25.6, z], 1).astype(np.float32)
    assert np.array_equal(means[:, 2], z)        # camera depth = z exactly (identity view)
    sc = synth.Scene(means, np.full((n, 3), -5.5, np.float32),
                     np.tile(np.float32([1, 0, 0, 0]), (n, 1)),
                     np.full(n, -4.0, np.float32), rng.random((n, 3)).astype(np.float32))
    st = renderer.forward(dev_scene(sc), torch.from_numpy(eye_view()).cuda(), rcam(cam))
    dbg = st.stage()
    stg = dbg["stage"]
    assert len(np.unique(stg[:, 6])) == 3
    ranges, ids = binning.tile_lists(stg[:, 0], stg[:, 1], stg[:, 7], stg[:, 8], stg[:, 6],
                                     np.ones(n, bool), 32, 32)
    longest = (ranges[:, 1] - ranges[:, 0]).max()
    say(f"  longest list {longest}")
    assert lo <= longest <= hi
    assert np.array_equal(dbg["ranges"], ranges)
    assert np.array_equal(dbg["ids"], ids)


def test_chunk_with_more_pairs_than_the_emit_stages(renderer):
    """Chunks of 1024 Gaussians that each cover about 30 tiles of an 8 x 8
    tile frame hold about 30k pairs, more than the emit orders by tile in LDS
    (12288), so they are written straight into their chunk-major block; the
    lists still equal the definition (tile, then depth, then index)."""
    say("test_chunk_with_more_pairs_than_the_emit_stages")
    cam = synth.Camera(128, 128, 102.4, 102.4, 64.0, 64.0)
    rng = np.random.default_rng(9)
    n = 2500
    z = rng.uniform(1, 3, n)
    u = rng.uniform(20, 108, n)
    v = rng.uniform(20, 108, n)
    sig_px = rng.uniform(10.0, 14.0, n)
    means = np.stack([(u - 64) * z / 102.4, (v - 64) * z / 102.4, z], 1)
    log_s = np.log(sig_px * z / 102.4)[:, None] + np.zeros((1, 3))
    sc = synth.Scene(means.astype(np.float32), log_s.astype(np.float32),
                     np.tile(np.float32([1, 0, 0, 0]), (n, 1)),
                     np.full(n, 2.0, np.float32), rng.random((n, 3)).astype(np.float32))
    st = renderer.forward(dev_scene(sc), torch.from_numpy(eye_view()).cuda(), rcam(cam))
    dbg = st.stage()
    stg = dbg["stage"]
    ranges, ids = binning.tile_lists(stg[:, 0], stg[:, 1], stg[:, 7], stg[:, 8], stg[:, 6],
                                     np.ones(n, bool), 128, 128)
    per_chunk = len(ids) / ((n + 1023) // 1024)
    say(f"  pairs {len(ids)}, about {per_chunk:.0f} per chunk")
    assert per_chunk > 12288
    assert np.array_equal(dbg["ranges"], ranges)
    assert np.array_equal(dbg["ids"], ids)


@pytest.mark.parametrize("j", [2, 3, 4])
def test_downsampled_frame_renders_one_sample_per_block(renderer, j):
    """A frame masked to one pixel in 2^j renders with coarse tiles of 16x16
    samples.  Per pixel it is bitwise the same as the masked 16x16-tile render
    (same arithmetic, same fragment order); tile lists are bit-exact against
    the replay at the coarse tile size; gradients match the oracle."""
    say(f"test_downsampled_frame j={j}")
    cam = synth.Camera(200, 120, 160.0, 160.0, 100.0, 60.0)        # ragged coarse tiles
    sc = synth.make_scene(synth.SceneSpec("ds", 200, 120, 3000, 77 + j), cam)
    view = view_from(synth.pose_offset(70 + j, 0.02, 1.0))
    dsc = dev_scene(sc)
    dview = torch.from_numpy(view).cuda()
    full = renderer.forward(dsc, dview, rcam(cam))
    mask = torch.empty(120, 200, dtype=torch.uint8, device="cuda")
    rtgs.downsample_mask(full.final_T, j, mask)
    a = renderer.forward(dsc, dview, rcam(cam), pixel_mask=mask, sample_log2=j)
    b = renderer.forward(dsc, dview, rcam(cam), pixel_mask=mask, sample_log2=0)
    torch.cuda.synchronize()
    for k in ("color", "depth", "alpha", "final_T"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    assert (a.last_idx[mask == 0] == -1).all()
    # coarse tile lists, bit-exact
    dbg = a.stage()
    stg = dbg["stage"]
    valid = oracle.render(sc.arrays(), view, cam_tuple(cam), pixels=[0]).proj.valid.numpy()
    bw, bh = 2 ** ((j + 1) // 2), 2 ** (j // 2)
    ranges, ids = binning.tile_lists(stg[:, 0], stg[:, 1], stg[:, 7], stg[:, 8], stg[:, 6], valid,
                                     200, 120, 16 * bw, 16 * bh)
    assert np.array_equal(dbg["ranges"], ranges)
    assert np.array_equal(dbg["ids"], ids)
    # images and gradients against the oracle on the mask
    pm = mask.cpu().numpy()
    ref_f = oracle.render(sc.arrays(), view, cam_tuple(cam), pixel_mask=pm)
    keep = ~ref_f.flags.numpy()
    assert rel_err(a.color.cpu().numpy(), ref_f.color.numpy(), keep) < IMG_TOL
    gc, gd, ga = synth.upstream_grads(200, 120, 80 + j)
    gc, gd, ga = gc * keep[None], gd * keep, ga * keep
    g = renderer.backward(dsc, dview, rcam(cam), a, torch.from_numpy(gc).cuda(),
                          torch.from_numpy(gd).cuda(), torch.from_numpy(ga).cuda(),
                          pixel_mask=mask)
    torch.cuda.synchronize()
    _, ref = oracle.render_with_grads(sc.arrays(), view, cam_tuple(cam), gc, gd, ga,
                                      pixel_mask=pm)
    for name in ("means", "log_scales", "quats", "opacity_logits", "colors"):
        assert grad_err(g[name].cpu().numpy(), getattr(ref, name).numpy()) < GRAD_TOL, name
    assert rel_err(g["pose"].cpu().numpy(), ref.pose.numpy()) < GRAD_TOL
