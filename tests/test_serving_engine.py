"""Serving engine logic on the CPU with the modelled executor: arrivals,
continuous batching, admission by HBM and workspace budgets, per-session
ordering, the downsampling schedule, and batched versus serial latency."""
import numpy as np

from paper_2510_06644_amd import serving
from paper_2510_06644_amd.serving import Engine, FakeExecutor, ServeConfig, SessionSpec


def _specs():
    return serving.serving_mix()


def test_poisson_trace_is_seeded_and_has_the_rate():
    a = serving.poisson_trace(16, 30.0, 20.0, 7)
    b = serving.poisson_trace(16, 30.0, 20.0, 7)
    assert a == b
    assert abs(len(a) / (16 * 20.0) - 30.0) < 1.5
    per = [sum(1 for e in a if e[1] == s) for s in range(16)]
    assert min(per) > 450
    assert all(a[i][0] <= a[i + 1][0] for i in range(len(a) - 1))


def _run(cfg, specs=None, duration=3.0, rate=30.0, seed=3, **fx):
    specs = specs or _specs()
    ex = FakeExecutor(**fx)
    eng = Engine(specs, ex, cfg)
    rep = eng.run(serving.poisson_trace(len(specs), rate, duration, seed), warmup_s=0.5)
    return eng, ex, rep


def test_every_frame_completes_once_in_order_per_session():
    eng, ex, rep = _run(ServeConfig())
    trace = serving.poisson_trace(16, 30.0, 3.0, 3)
    assert len(eng.finished) == len(trace)
    seen = {}
    for f in sorted(eng.finished, key=lambda f: f.done_time):
        assert seen.get(f.session, -1) < f.index
        seen[f.session] = f.index
    # never two frames of one session in the same group
    for phase, sessions in ex.log:
        assert len(sessions) == len(set(sessions))
    # keyframes (every 8th) carry the mapping iterations
    iters = sum(10 + (20 if f.keyframe else 0) for f in eng.finished)
    assert eng.iters == iters


def test_batched_beats_serial_on_the_same_trace():
    _, _, batched = _run(ServeConfig(mode="batched"))
    _, _, serial = _run(ServeConfig(mode="serial"))
    assert batched["frames"] == serial["frames"]
    assert batched["mean_batch"] > 2
    assert batched["p99_ms"] < serial["p99_ms"]
    assert batched["iters_per_s"] > serial["iters_per_s"]


def test_hbm_budget_admission_evicts_idle_sessions_and_drops_nothing():
    specs = [SessionSpec(320, 240, 20_000, seed=i) for i in range(6)]
    ex0 = FakeExecutor()
    per = ex0.session_bytes(specs[0])
    cfg = ServeConfig(hbm_budget=2.5 * per)          # two sessions resident at a time
    eng, ex, rep = _run(cfg, specs, duration=1.0, rate=10.0)
    assert len(eng.finished) == len(serving.poisson_trace(6, 10.0, 1.0, 3))
    assert eng.max_resident <= cfg.hbm_budget
    for phase, sessions in ex.log:
        assert len(sessions) <= 2


def test_workspace_budget_bounds_the_batch():
    specs = _specs()
    ex0 = FakeExecutor()
    big = ex0.step_bytes(specs[-1], None)
    cfg = ServeConfig(ws_budget=2.5 * big)
    eng, ex, rep = _run(cfg, duration=1.0)
    for phase, sessions in ex.log:
        total = sum(ex0.step_bytes(specs[s], None) for s in sessions)
        assert total <= cfg.ws_budget or len(sessions) == 1


def test_downsampling_schedule_follows_keyframes():
    eng = Engine([SessionSpec(64, 64, 10)], FakeExecutor(), ServeConfig(downsample=True))
    for i in range(12):
        eng.submit(0.01 * i, 0, i)
    js = [f.log2_ratio for f in eng.pending]
    assert js == [0, 4, 3, 2, 2, 2, 2, 2, 0, 4, 3, 2]
    assert [f.keyframe for f in eng.pending][:9] == [True] + [False] * 7 + [True]


def test_async_mapping_runs_keyframe_jobs_beside_tracking():
    """Keyframe mapping as a background job: every frame finishes when its
    tracking ends; every keyframe's job runs (20 iterations), a session's
    jobs one at a time in keyframe order; frame latency drops against
    mapping in line."""
    cfg = ServeConfig(async_mapping=True)
    eng, ex, rep = _run(cfg)
    trace = serving.poisson_trace(16, 30.0, 3.0, 3)
    assert len(eng.finished) == len(trace)
    keys = sum(1 for f in eng.finished if f.keyframe)
    assert rep["map_jobs"] == keys > 0
    assert eng.iters == 10 * len(eng.finished) + 20 * rep["map_jobs"]
    for phase, sessions in ex.log:
        assert len(sessions) == len(set(sessions))
    for s in range(16):
        idx = [j.index for j in sorted(eng.map_finished, key=lambda j: j.done_time)
               if j.session == s]
        assert idx == sorted(idx)
    for j in eng.map_finished:
        assert j.done_time >= j.arrival
    _, _, sync = _run(ServeConfig())
    assert rep["p99_ms"] < sync["p99_ms"]


def test_frames_wait_for_their_map_version_and_start_pose():
    """Frame i starts after frame i - pose_lag has finished and after the
    jobs of the keyframes k <= i - map_lag (its map version); the version is
    a function of the index alone."""
    for overlap in (False, True):
        cfg = ServeConfig(async_mapping=True, overlap_frames=overlap)
        eng, ex, rep = _run(cfg, duration=2.0)
        fin = {(f.session, f.index): f for f in eng.finished}
        jobs = {(j.session, j.index): j for j in eng.map_finished}
        lag = cfg.pose_lag
        assert lag == (2 if overlap else 1)
        for (s, i), f in fin.items():
            assert f.version == eng.version_needed(i)
            assert f.version == (max(0, (i - 8) // 8 + 1) if i >= 8 else 0)
            if i - lag >= 0:
                assert fin[(s, i - lag)].done_time <= f.started + 1e-12
            for k in range(0, i - cfg.map_lag + 1, cfg.keyframe_every):
                assert jobs[(s, k)].done_time <= f.started + 1e-12


def test_async_mapping_serial_runs_one_item_at_a_time():
    eng, ex, rep = _run(ServeConfig(mode="serial", async_mapping=True), duration=1.0,
                        rate=5.0)
    for phase, sessions in ex.log:
        assert len(sessions) == 1
    # no step runs a tracking frame and a map job together
    steps = [len(x[1]) for x in ex.log]
    assert sum(steps) == eng.iters and len(ex.log) == eng.steps
    assert len(eng.finished) == len(serving.poisson_trace(16, 5.0, 1.0, 3))


def test_overlapping_frames_of_a_session():
    """overlap_frames: a session's next frame may start before the previous
    one ends; frames of a session still finish in arrival order, every frame
    completes, and the latency drops against in-order admission."""
    cfg = ServeConfig(async_mapping=True, overlap_frames=True)
    eng, ex, rep = _run(cfg)
    trace = serving.poisson_trace(16, 30.0, 3.0, 3)
    assert len(eng.finished) == len(trace)
    seen = {}
    for f in sorted(eng.finished, key=lambda f: (f.done_time, f.index)):
        assert seen.get(f.session, -1) < f.index
        seen[f.session] = f.index
    assert any(len(s) != len(set(s)) for ph, s in ex.log if ph == "track")
    _, _, inorder = _run(ServeConfig(async_mapping=True))
    assert rep["p99_ms"] <= inorder["p99_ms"]

