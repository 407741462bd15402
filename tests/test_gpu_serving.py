"""Serving on the GPU: a session's results are the same alone and in the mix
(the batched launches do each session's arithmetic exactly as a single-session
launch does, so the comparison is bitwise), and the engine runs a short
open-loop trace in both modes."""
import pytest
import torch

from paper_2510_06644_amd import rtgs, serving, synth
from paper_2510_06644_amd.serving import Engine, GpuExecutor, ServeConfig, SessionSpec
from tests.gpu_util import dev_scene, rcam, say, view_from

pytestmark = pytest.mark.gpu

SPECS = [SessionSpec(160, 120, 5_000, "c0", 11), SessionSpec(320, 240, 20_000, "c0", 12),
         SessionSpec(128, 96, 3_000, "c2", 13)]


def test_batched_render_equals_single_session_renders():
    say("test_batched_render_equals_single_session_renders")
    h = rtgs.Handle(0)
    items, singles = [], []
    for k, sp in enumerate(SPECS):
        cam = synth.make_camera(sp.width, sp.height)
        sc = synth.make_scene(synth.SceneSpec("s", sp.width, sp.height, sp.n, sp.seed), cam)
        view = torch.from_numpy(view_from(synth.pose_offset(60 + k, 0.02, 1.0))).cuda()
        d = dev_scene(sc)
        mk = lambda: dict(scene=d, viewmat=view, cam=rcam(cam),
                          color=torch.empty(3, sp.height, sp.width, device="cuda"),
                          depth=torch.empty(sp.height, sp.width, device="cuda"),
                          alpha=torch.empty(sp.height, sp.width, device="cuda"),
                          final_T=torch.empty(sp.height, sp.width, device="cuda"),
                          last_idx=torch.empty(sp.height, sp.width, dtype=torch.int32,
                                               device="cuda"))
        items.append(mk())
        singles.append(mk())
    cap = 400_000
    ns = [s.n for s in SPECS]
    ws_ = [s.width for s in SPECS]
    hs = [s.height for s in SPECS]
    wsb = torch.empty(rtgs.rtgs_workspace_size_batched(ns, ws_, hs, cap), dtype=torch.uint8,
                      device="cuda")
    rtgs.render_fwd_batched(h, items, wsb, cap)
    single_ws = []
    for it, sp in zip(singles, SPECS):
        w1 = torch.empty(rtgs.rtgs_workspace_size(sp.n, sp.width, sp.height, cap),
                         dtype=torch.uint8, device="cuda")
        rtgs.render_fwd_batched(h, [it], w1, cap)
        single_ws.append(w1)
    torch.cuda.synchronize()
    for a, b in zip(items, singles):
        for k in ("color", "depth", "alpha", "final_T"):
            assert torch.equal(a[k], b[k]), k
    # backward: gradients to everything
    gens = torch.Generator(device="cuda").manual_seed(5)
    for a, b, sp in zip(items, singles, SPECS):
        gc = torch.randn(3, sp.height, sp.width, device="cuda", generator=gens)
        gd = torch.randn(sp.height, sp.width, device="cuda", generator=gens)
        for it in (a, b):
            it["dL_dcolor"], it["dL_ddepth"] = gc, gd
            n = sp.n
            it.update(g_means=torch.empty(n, 3, device="cuda"),
                      g_log_scales=torch.empty(n, 3, device="cuda"),
                      g_quats=torch.empty(n, 4, device="cuda"),
                      g_opacity_logits=torch.empty(n, device="cuda"),
                      g_colors=torch.empty(n, 3, device="cuda"),
                      g_pose6=torch.empty(6, device="cuda"),
                      g_viewmat=torch.empty(3, 4, device="cuda"))
    flags = rtgs.RTGS_GRAD_MAP | rtgs.RTGS_GRAD_POSE
    rtgs.render_bwd_batched(h, items, wsb, cap, grad_flags=flags)
    for it, w1 in zip(singles, single_ws):
        rtgs.render_bwd_batched(h, [it], w1, cap, grad_flags=flags)
    torch.cuda.synchronize()
    for a, b in zip(items, singles):
        for k in ("g_means", "g_log_scales", "g_quats", "g_opacity_logits", "g_colors",
                  "g_pose6", "g_viewmat"):
            assert torch.equal(a[k], b[k]), k


def _state(ex):
    return {s: ([p.detach().clone() for p in S["params"]], S["viewmat"].clone())
            for s, S in ex.sessions.items()}


def test_each_session_is_the_same_alone_and_in_the_mix():
    say("test_each_session_is_the_same_alone_and_in_the_mix")
    trace = [(0.0, s, 0) for s in range(len(SPECS))] + [(0.0, s, 1) for s in range(len(SPECS))]
    out = {}
    for mode in ("serial", "batched"):
        cfg = ServeConfig(track_iters=3, map_iters=2, keyframe_every=2, mode=mode)
        ex = GpuExecutor(0, n_targets=2)
        eng = Engine(SPECS, ex, cfg)
        rep = eng.run(trace)
        assert rep["frames"] == len(trace)
        out[mode] = (_state(ex), rep)
        ex.verify()
    a, b = out["serial"][0], out["batched"][0]
    for s in a:
        for x, y in zip(a[s][0], b[s][0]):
            assert torch.equal(x, y)
        assert torch.equal(a[s][1], b[s][1])
    assert out["batched"][1]["mean_batch"] > out["serial"][1]["mean_batch"]


def test_short_open_loop_trace_both_modes():
    say("test_short_open_loop_trace_both_modes")
    specs = [SessionSpec(320, 240, 20_000, "c0", 20 + k) for k in range(4)]
    trace = serving.poisson_trace(len(specs), 30.0, 0.6, 9)
    for mode in ("batched", "serial"):
        ex = GpuExecutor(0, n_targets=2)
        eng = Engine(specs, ex, ServeConfig(mode=mode, downsample=True))
        rep = eng.run(trace)
        say(f"  {mode}: {rep['frames']} frames p50 {rep['p50_ms']:.1f} ms p99 "
            f"{rep['p99_ms']:.1f} ms iters/s {rep['iters_per_s']:.0f} batch {rep['mean_batch']:.1f}")
        assert rep["frames"] == len(trace)
        assert rep["p50_ms"] > 0


SERVED = dict(track_iters=4, map_iters=3, keyframe_every=3, downsample=True,
              async_mapping=True, map_every=2, overlap_frames=True, map_lag=3)


def test_pruned_async_overlapping_serving_keeps_maps_consistent():
    """The served form of the algorithm: pruning per tracked frame, keyframe
    mapping as background jobs, overlapping frames.  Every frame finishes,
    every keyframe's job runs, each map loses some and at most half of its
    Gaussians, and the map and Adam moments keep one row count."""
    say("test_pruned_async_overlapping_serving_keeps_maps_consistent")
    specs = [SessionSpec(320, 240, 20_000, "c0", 40 + k) for k in range(3)]
    trace = serving.poisson_trace(len(specs), 60.0, 0.4, 13)
    ex = GpuExecutor(0, n_targets=2, prune=True, prune_ratio=0.2)
    eng = Engine(specs, ex, ServeConfig(**SERVED))
    rep = eng.run(trace)
    say(f"  {rep['frames']} frames, {rep['map_jobs']} map jobs, p99 {rep['p99_ms']:.1f} ms")
    assert rep["frames"] == len(trace)
    keys = sum(1 for f in eng.finished if f.keyframe)
    assert rep["map_jobs"] == keys
    ex.verify()
    assert ex.overflows == 0
    for s in range(len(specs)):
        S = ex.sessions[s]
        n = S["params"][0].shape[0]
        assert S["n0"] // 2 <= n < S["n0"], (n, S["n0"])   # pruned, at most 50%
        assert n == S["n0"] - S["removed"]
        assert S["version"] == sum(1 for j in eng.map_finished if j.session == s)
        opt = S["opt"]
        for t in list(S["params"]) + opt.exp_avg + opt.exp_avg_sq:
            assert t.shape[0] == n and bool(torch.isfinite(t).all())
        assert S["inflight"] == 0


def test_served_algorithm_is_the_same_alone_and_in_the_mix():
    """The served form with pruning, downsampling, background keyframe
    mapping and overlapping frames is a function of the trace alone: every
    frame's end pose and every session's final map are bitwise the same when
    the trace is served one item at a time and when it is batched."""
    say("test_served_algorithm_is_the_same_alone_and_in_the_mix")
    specs = [SessionSpec(320, 240, 20_000, "c0", 50 + k) for k in range(3)]
    trace = serving.poisson_trace(len(specs), 60.0, 0.4, 17)
    out = {}
    for mode in ("serial", "batched"):
        ex = GpuExecutor(0, n_targets=2, prune=True, prune_ratio=0.2, record_poses=True)
        eng = Engine(specs, ex, ServeConfig(mode=mode, **SERVED))
        rep = eng.run(trace)
        ex.verify()
        assert ex.overflows == 0 and rep["frames"] == len(trace)
        say(f"  {mode}: {rep['frames']} frames, mean batch {rep['mean_batch']:.2f}, "
            f"{rep['map_jobs']} map jobs")
        out[mode] = (ex, rep, eng)
    a, b = out["serial"][0], out["batched"][0]
    assert out["batched"][1]["mean_batch"] > out["serial"][1]["mean_batch"] == 1.0
    assert a.frame_poses.keys() == b.frame_poses.keys()
    for k in a.frame_poses:
        assert torch.equal(a.frame_poses[k], b.frame_poses[k]), k
    downsampled = sum(1 for f in out["batched"][2].finished if f.mask is not None)
    assert downsampled > 0
    for s in range(len(specs)):
        A, B = a.sessions[s], b.sessions[s]
        assert A["version"] == B["version"] > 0
        assert A["removed"] == B["removed"] > 0
        for x, y in zip(A["params"], B["params"]):
            assert torch.equal(x, y)
        for x, y in zip(A["opt"].exp_avg + A["opt"].exp_avg_sq,
                        B["opt"].exp_avg + B["opt"].exp_avg_sq):
            assert torch.equal(x, y)


def test_served_algorithm_with_fused_launches_equals_unfused():
    """The executor's fused form (the forward writes the loss gradient, map
    jobs update their maps inside the backward) serves the same algorithm as
    its unfused form (a loss pass, the backward's gradients, adam_step): every
    frame's end pose and every session's final map and Adam moments bitwise
    equal, with pruning, downsampling and background keyframe mapping."""
    say("test_served_algorithm_with_fused_launches_equals_unfused")
    specs = [SessionSpec(320, 240, 20_000, "c0", 60 + k) for k in range(3)]
    trace = serving.poisson_trace(len(specs), 60.0, 0.4, 19)
    out = {}
    for fused in (False, True):
        ex = GpuExecutor(0, n_targets=2, prune=True, prune_ratio=0.2, record_poses=True,
                         fused=fused)
        eng = Engine(specs, ex, ServeConfig(mode="batched", **SERVED))
        rep = eng.run(trace)
        ex.verify()
        assert ex.overflows == 0 and rep["frames"] == len(trace)
        say(f"  fused={fused}: {rep['frames']} frames, {rep['map_jobs']} map jobs")
        out[fused] = ex
    a, b = out[False], out[True]
    assert a.frame_poses.keys() == b.frame_poses.keys()
    for k in a.frame_poses:
        assert torch.equal(a.frame_poses[k], b.frame_poses[k]), k
    for s in range(len(specs)):
        A, B = a.sessions[s], b.sessions[s]
        assert A["version"] == B["version"] > 0
        assert A["removed"] == B["removed"] > 0
        for x, y in zip(A["params"], B["params"]):
            assert torch.equal(x, y)
        for x, y in zip(A["opt"].exp_avg + A["opt"].exp_avg_sq,
                        B["opt"].exp_avg + B["opt"].exp_avg_sq):
            assert torch.equal(x, y)
