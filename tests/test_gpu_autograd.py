"""The autograd Function (render_fwd / render_bwd as torch.autograd.Function):
gradients to every map parameter and to a pose parametrised as
Exp(xi) T0 at xi != 0, against the float64 oracle, with each state policy;
saved per-pixel state, saved fragments and recomputed state give
bitwise-identical gradients."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_06644_amd import autograd, pose, rtgs, synth
from tests.gpu_util import GRAD_TOL, cam_tuple, grad_err, eye_view, rcam, rel_err, say

pytestmark = pytest.mark.gpu


def _leaves(sc):
    return [torch.from_numpy(a).cuda().requires_grad_(True) for a in sc.arrays()]


def _loss(c, d, a, gc, gd, ga):
    return (c * gc).sum() + (d * gd).sum() + (a * ga).sum()


@pytest.mark.parametrize("state", ["save", "fragments"])
def test_autograd_matches_oracle_with_pose_off_zero(state):
    say(f"test_autograd_matches_oracle_with_pose_off_zero state={state}")
    spec = synth.CONFIGS["c0"]
    cam = synth.make_camera(spec.width, spec.height)
    sc = synth.make_scene(spec, cam)
    xi0 = synth.pose_offset(41, 0.02, 1.0)
    t0 = eye_view()
    params = _leaves(sc)
    xi = torch.tensor(xi0, dtype=torch.float32, device="cuda", requires_grad=True)
    vm = pose.apply_left(xi, torch.from_numpy(t0).cuda())
    # the oracle sees the same float32 view matrix
    vm32 = vm.detach().cpu().numpy()
    ref_f = oracle.render(sc.arrays(), vm32, cam_tuple(cam))
    keep = ~ref_f.flags.numpy()
    gc, gd, ga = synth.upstream_grads(cam.width, cam.height, 9)
    gc, gd, ga = gc * keep[None], gd * keep, ga * keep
    c, d, a, _ = autograd.render(*params, vm, rcam(cam), state=state)
    _loss(c, d, a, torch.from_numpy(gc).cuda(), torch.from_numpy(gd).cuda(),
          torch.from_numpy(ga).cuda()).backward()
    torch.cuda.synchronize()
    _, ref = oracle.render_with_grads(sc.arrays(), vm32, cam_tuple(cam), gc, gd, ga)
    for p, name in zip(params, ("means", "log_scales", "quats", "opacity_logits", "colors")):
        e = grad_err(p.grad.cpu().numpy(), getattr(ref, name).numpy())
        say(f"  {name}: {e:.2e}")
        assert e < GRAD_TOL, name
    # dL/dxi through the oracle's own exponential, in float64 on the CPU
    xi64 = torch.tensor(xi0, dtype=torch.float64, requires_grad=True)
    vm64 = oracle.apply_left(xi64, torch.tensor(t0, dtype=torch.float64))
    (gxi,) = torch.autograd.grad(vm64, xi64, ref.viewmat)
    e = rel_err(xi.grad.cpu().numpy(), gxi.numpy())
    say(f"  xi: {e:.2e}  {xi.grad.cpu().numpy()}  {gxi.numpy()}")
    assert e < 1e-4


def test_saved_and_recomputed_state_give_identical_gradients():
    say("test_saved_and_recomputed_state")
    spec = synth.CONFIGS["c0"]
    cam = synth.make_camera(spec.width, spec.height)
    sc = synth.make_scene(spec, cam)
    gc, gd, ga = (torch.from_numpy(x).cuda() for x in synth.upstream_grads(128, 128, 10))
    vm = torch.from_numpy(eye_view()).cuda()
    grads = []
    for state in ("save", "recompute", "fragments"):
        params = _leaves(sc)
        v = vm.clone().requires_grad_(True)
        c, d, a, _ = autograd.render(*params, v, rcam(cam), state=state)
        _loss(c, d, a, gc, gd, ga).backward()
        grads.append([p.grad.clone() for p in params] + [v.grad.clone()])
    torch.cuda.synchronize()
    for other in grads[1:]:
        for x, y in zip(grads[0], other):
            assert torch.equal(x, y)


def test_c3_saved_vs_recompute_at_1200x680_500k():
    """The differentiation workload: 1200x680, 500,000 Gaussians, gradients to
    the pose and all map parameters.  The three state policies give the same
    gradients bit for bit; time and peak memory of each are printed."""
    say("test_c3_saved_vs_recompute")
    spec = synth.CONFIGS["c3"]
    cam = synth.make_camera(spec.width, spec.height)
    sc = synth.make_scene(spec, cam)
    r = rtgs.Renderer(0, check="every")
    gc = torch.randn(3, cam.height, cam.width, device="cuda") * 1e-6
    gd = torch.randn(cam.height, cam.width, device="cuda") * 1e-6
    vm = torch.from_numpy(view_c3()).cuda()
    out = {}
    for state in ("save", "recompute", "fragments", "save", "recompute", "fragments"):
        params = _leaves(sc)
        v = vm.clone().requires_grad_(True)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        c, d, a, _ = autograd.render(*params, v, rcam(cam), renderer=r, state=state)
        ((c * gc).sum() + (d * gd).sum()).backward()
        e1.record()
        torch.cuda.synchronize()
        out[state] = (e0.elapsed_time(e1), torch.cuda.max_memory_allocated() - base,
                      [p.grad for p in params] + [v.grad])
    for k in ("save", "recompute", "fragments"):
        say(f"  {k}: {out[k][0]:.3f} ms, peak +{out[k][1] / 2**20:.1f} MiB")
    for k in ("recompute", "fragments"):
        for x, y in zip(out["save"][2], out[k][2]):
            assert torch.equal(x, y), k


def view_c3():
    return synth.identity_viewmat()
