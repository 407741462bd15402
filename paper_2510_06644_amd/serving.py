"""Serving many SLAM sessions on one GPU with continuous batching.

Each session keeps its Gaussian map, pose and optimiser state resident in HBM.
Frames arrive per session (a seeded Poisson process); a frame needs
``track_iters`` tracking iterations (gradients to the pose only) and, on
keyframes (every ``keyframe_every``-th frame), ``map_iters`` mapping
iterations (gradients to every Gaussian parameter) afterwards (Sec. 2.2:
tracking on every frame, mapping on keyframes).  Non-keyframes may be
rendered on a pixel mask chosen by the dynamic-downsampling schedule
(Sec. 4.2) from the session's last transmittance image.

Continuous batching at iteration granularity: every engine step runs one
iteration of every admitted frame, all tracking frames in one batched
render_fwd / render_bwd pair (one launch per stage for all sessions, one tile
space, one sort) and all mapping frames in another.  Frames that arrive while
others run join at the next step, as batch slots and memory free up.
Admission is by HBM budget: a session opens only if its resident footprint
fits, and a frame joins a step only while the step's workspace stays within
the workspace budget.  The engine never waits for the GPU between steps; each
step records an event, and a frame's completion time is the GPU time of the
event of its last iteration.

``mode="serial"`` serves the same trace one session-frame at a time (FIFO,
single-session launches, no overlap): the baseline for the batched mode.

Executors: ``GpuExecutor`` runs the HIP library; ``FakeExecutor`` models
iteration cost on the CPU (tests of admission, batching and fairness without
a GPU).
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import heapq
import math
import time

import numpy as np

from . import synth

# --------------------------------------------------------------------------- workload


@dataclasses.dataclass(frozen=True)
class SessionSpec:
    width: int
    height: int
    n: int
    kind: str = "c0"          # scene distribution (synth.CONFIGS key)
    seed: int = 0

    @property
    def pixels(self):
        return self.width * self.height


def serving_mix(seed=4000):
    """The 16-session mix: 6 x (320x240, 20k), 6 x (640x480, 100k),
    4 x (1200x680, 500k)."""
    out = []
    k = 0
    for count, w, h, n, kind in synth.SERVING_CLASSES:
        for _ in range(count):
            out.append(SessionSpec(w, h, n, kind, seed + k))
            k += 1
    return out


@dataclasses.dataclass
class Frame:
    session: int
    index: int
    arrival: float
    keyframe: bool
    track_left: int
    map_left: int
    log2_ratio: int = 0
    started: float = -1.0
    done_event: object = None
    done_time: float = -1.0
    pose_from: int = -1             # frame whose end pose (and final T) this one starts from
    version: int = 0                # map version it renders (async mapping)

    @property
    def remaining(self):
        return self.track_left + self.map_left

    @property
    def phase(self):
        return "track" if self.track_left > 0 else "map"


@dataclasses.dataclass
class MapJob:
    """The mapping iterations of one keyframe, run beside the session's later
    tracking frames when mapping is asynchronous (ServeConfig.async_mapping):
    the keyframe's result (its pose) is ready when its tracking ends, and its
    map update follows, as in keyframe-based SLAM systems that map in a
    separate thread.  A session's jobs run one at a time in keyframe order;
    each turns map version v into v + 1."""
    session: int
    index: int
    arrival: float                  # the keyframe's arrival
    created: float
    map_left: int
    frame: object                   # the keyframe (its target frame)
    log2_ratio: int = 0
    started: float = -1.0
    done_event: object = None
    done_time: float = -1.0

    @property
    def phase(self):
        return "map"

    @property
    def remaining(self):
        return self.map_left


def poisson_trace(n_sessions, rate_hz, duration_s, seed):
    """Per-session exponential inter-arrival times; list of (t, session, index)
    sorted by time."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ev = []
    for s in range(n_sessions):
        t, i = 0.0, 0
        while True:
            t += rng.exponential(1.0 / rate_hz)
            if t >= duration_s:
                break
            ev.append((t, s, i))
            i += 1
    ev.sort()
    return ev


@dataclasses.dataclass
class ServeConfig:
    track_iters: int = 10
    map_iters: int = 20
    keyframe_every: int = 8
    downsample: bool = False        # dynamic downsampling of non-keyframes
    m: int = 2                      # resolution growth factor of the schedule
    max_batch: int = 16             # frames per engine step
    hbm_budget: float = 200e9       # resident maps + optimiser state (bytes)
    ws_budget: float = 40e9         # per-step workspace (bytes)
    mode: str = "batched"           # or "serial"
    # keyframe mapping as a per-session background job (MapJob); a frame's
    # latency is then the time to its pose (end of tracking)
    async_mapping: bool = False
    # with async_mapping: while tracking frames are in flight, map jobs advance
    # on one engine step in map_every (tracking first); 1 = every step
    map_every: int = 1
    max_map_batch: int = 16         # map jobs in flight at once (async_mapping)
    # a session's next frame may start before its previous frame's tracking
    # ends (at most two frames of a session in flight)
    overlap_frames: bool = False
    # with async_mapping, frame i renders map version V(i): the map after the
    # jobs of the keyframes k <= i - map_lag, waiting for it if it is not
    # ready; a fixed version per frame keeps every result a function of the
    # trace alone, whatever the batching
    map_lag: int = 8

    @property
    def pose_lag(self):
        """Frame i starts from the end pose of frame i - pose_lag (and a
        downsampled frame takes its pixel mask from that frame's final
        transmittance): the previous frame, or the one before it when frames
        overlap."""
        return 2 if self.overlap_frames else 1


# --------------------------------------------------------------------------- engine


class Engine:
    """Admission + continuous batching over an executor."""

    def __init__(self, specs, executor, cfg: ServeConfig, clock=None):
        self.specs = list(specs)
        self.ex = executor
        self.cfg = cfg
        self.clock = clock or getattr(executor, "clock", time.perf_counter)
        self.open = [False] * len(self.specs)
        self.pending = collections.deque()     # frames waiting (arrived)
        self.active = []                       # frames admitted, in progress
        self.finished = []
        self.resident = 0.0
        self.max_resident = 0.0
        self.steps = 0
        self.iters = 0
        self.batch_sizes = []
        self.last_key = [-1] * len(self.specs)
        ns = len(self.specs)
        self.next_admit = [0] * ns             # next frame index to admit per session
        self.track_done = [set() for _ in range(ns)]
        self.jobs_done = [0] * ns              # finished map jobs = published map version
        self.map_queue = [collections.deque() for _ in range(ns)]   # jobs not started
        self.map_active = []
        self.map_finished = []

    # ---- dependencies ------------------------------------------------------
    def version_needed(self, i):
        """Map version frame i renders: the number of keyframes k <= i - map_lag
        (their jobs come first); 0 without asynchronous mapping."""
        c = self.cfg
        if not c.async_mapping or c.map_iters <= 0:
            return 0
        v = i - c.map_lag
        return v // c.keyframe_every + 1 if v >= 0 else 0

    def _ready(self, f):
        """Frame f may start: the session's earlier frames have started, the
        frame it starts from has finished, and its map version is published."""
        s = f.session
        if f.index != self.next_admit[s]:
            return False
        src = f.index - self.cfg.pose_lag
        if src >= 0 and src not in self.track_done[s]:
            return False
        return self.jobs_done[s] >= self.version_needed(f.index)

    @property
    def map_pending(self):
        return sum(len(q) for q in self.map_queue)

    # ---- admission -------------------------------------------------------
    def _try_open(self, s):
        """Make session s resident, evicting idle sessions (no frame or map job
        admitted or waiting) to host memory if the HBM budget requires it."""
        if self.open[s]:
            return True
        need = self.ex.session_bytes(self.specs[s])
        if self.resident + need > self.cfg.hbm_budget:
            waiting = ({f.session for f in self.pending} | {f.session for f in self.active}
                       | {j.session for j in self.map_active}
                       | {v for v, q in enumerate(self.map_queue) if q})
            for v in range(len(self.specs)):
                if self.resident + need <= self.cfg.hbm_budget:
                    break
                if self.open[v] and v not in waiting:
                    self.close_session(v)
            if self.resident + need > self.cfg.hbm_budget:
                return False
        self.ex.open_session(s, self.specs[s])
        self.resident += need
        self.max_resident = max(self.max_resident, self.resident)
        self.open[s] = True
        return True

    def close_session(self, s):
        if self.open[s]:
            self.ex.close_session(s)
            self.resident -= self.ex.session_bytes(self.specs[s])
            self.open[s] = False

    def submit(self, t, s, index):
        key = index % self.cfg.keyframe_every == 0
        j = 0
        if self.cfg.downsample and not key:
            k = self.last_key[s] if self.last_key[s] >= 0 else index - 1
            j = _log2_ratio(index, k, self.cfg.m)
        if key:
            self.last_key[s] = index
        maps = self.cfg.map_iters if key and not self.cfg.async_mapping else 0
        src = index - self.cfg.pose_lag
        self.pending.append(Frame(s, index, t, key, self.cfg.track_iters, maps, j,
                                  pose_from=src if src >= 0 else -1,
                                  version=self.version_needed(index)))

    def _admit(self, now):
        serial = self.cfg.mode == "serial"
        if serial and (self.active or self.map_active):
            return                            # one item at a time
        cap = 1 if serial else self.cfg.max_batch
        ws = sum(self.ex.step_bytes(self.specs[f.session], f) for f in self.active)
        keep = collections.deque()
        while self.pending and len(self.active) < cap:
            f = self.pending.popleft()
            if not self._ready(f):
                keep.append(f)
                continue
            need = self.ex.step_bytes(self.specs[f.session], f)
            if ws + need > self.cfg.ws_budget and self.active:
                keep.append(f)
                continue
            if not self._try_open(f.session):
                keep.append(f)
                continue
            f.started = now
            self.ex.start_frame(f, self.specs[f.session])
            self.active.append(f)
            self.next_admit[f.session] += 1
            release = getattr(self.ex, "release_versions", None)
            if release:                       # versions below this one are not rendered again
                release(f.session, self.version_needed(self.next_admit[f.session]))
            ws += need
        keep.extend(self.pending)
        self.pending = keep
        if self.cfg.async_mapping:
            self._admit_maps(now)

    def _admit_maps(self, now):
        serial = self.cfg.mode == "serial"
        if serial and (self.active or self.map_active):
            return                            # one item at a time, tracking first
        cap = 1 if serial else min(self.cfg.max_batch, self.cfg.max_map_batch)
        ws = sum(self.ex.step_bytes(self.specs[j.session], j) for j in self.map_active)
        busy = {j.session for j in self.map_active}
        heads = [q[0] for q in self.map_queue if q]
        for j in sorted(heads, key=lambda x: (x.created, x.session)):
            if len(self.map_active) >= cap:
                break
            s = j.session
            if s in busy:
                continue
            need = self.ex.step_bytes(self.specs[s], j)
            if ws + need > self.cfg.ws_budget and self.map_active:
                continue
            if not self._try_open(s):
                continue
            self.map_queue[s].popleft()
            j.started = now
            self.ex.start_map(j, self.specs[s])
            self.map_active.append(j)
            busy.add(s)
            ws += need

    # ---- one engine step ---------------------------------------------------
    def _finish_frame(self, f, now):
        self.ex.finish_frame(f, self.specs[f.session])
        self.finished.append(f)
        self.track_done[f.session].add(f.index)
        if self.cfg.async_mapping and f.keyframe and self.cfg.map_iters > 0:
            self.map_queue[f.session].append(
                MapJob(f.session, f.index, f.arrival, now, self.cfg.map_iters, f))

    def step(self, now):
        if self.cfg.async_mapping:
            return self._step_async(now)
        self._admit(now)
        if not self.active:
            return False
        groups = {"track": [], "map": []}
        for f in self.active:
            groups[f.phase].append(f)
        for phase in ("track", "map"):
            g = groups[phase]
            if not g:
                continue
            ev = self.ex.run_iteration(phase, g, [self.specs[f.session] for f in g])
            for f in g:
                if phase == "track":
                    f.track_left -= 1
                else:
                    f.map_left -= 1
                if f.remaining == 0:
                    f.done_event = ev
            self.iters += len(g)
        self.steps += 1
        self.batch_sizes.append(len(self.active))
        still = []
        for f in self.active:
            if f.remaining == 0:
                self._finish_frame(f, now)
            else:
                still.append(f)
        self.active = still
        return True

    def _step_async(self, now):
        """One iteration of every admitted tracking frame, then one of every
        admitted keyframe map job."""
        self._admit(now)
        if not self.active and not self.map_active:
            return False
        map_turn = not self.active or self.steps % max(1, self.cfg.map_every) == 0
        for phase, group in (("track", self.active), ("map", self.map_active)):
            if not group or (phase == "map" and not map_turn):
                continue
            ev = self.ex.run_iteration(phase, group, [self.specs[x.session] for x in group])
            for x in group:
                if phase == "track":
                    x.track_left -= 1
                else:
                    x.map_left -= 1
                if x.remaining == 0:
                    x.done_event = ev
            self.iters += len(group)
        self.steps += 1
        self.batch_sizes.append(len(self.active) + len(self.map_active))
        still = []
        for f in self.active:
            if f.remaining > 0:
                still.append(f)
            else:
                self._finish_frame(f, now)
        self.active = still
        still = []
        for j in self.map_active:
            if j.remaining > 0:
                still.append(j)
            else:
                self.ex.finish_map(j, self.specs[j.session])
                self.jobs_done[j.session] += 1
                self.map_finished.append(j)
        self.map_active = still
        return True

    def preopen(self):
        """Open (make resident) every session the HBM budget admits."""
        for s in range(len(self.specs)):
            self._try_open(s)

    def run(self, trace, warmup_s=0.0):
        """Open-loop: frames are submitted when their arrival time passes; the
        report leaves out frames that arrived in the first warmup_s seconds."""
        self.preopen()
        self.ex.start_clock()
        t0 = self.clock()
        i = 0
        while True:
            now = self.clock() - t0
            while i < len(trace) and trace[i][0] <= now:
                t, s, idx = trace[i]
                self.submit(t, s, idx)
                i += 1
            if not self.step(now):
                if i >= len(trace) and not self.pending and not self.map_pending:
                    break
                if i >= len(trace):
                    # nothing runs, nothing more arrives, yet work is left
                    raise RuntimeError(f"serving engine stalled: {len(self.pending)} frames, "
                                       f"{self.map_pending} map jobs waiting")
                wait = trace[i][0] - (self.clock() - t0)
                if wait > 0:
                    self.ex.idle(wait)
        self.ex.sync()
        for f in self.finished + self.map_finished:
            f.done_time = self.ex.event_time(f.done_event)
        return self.report(warmup_s=warmup_s)

    def report(self, warmup_s=0.0):
        lat = {}
        for f in self.finished:
            if f.arrival < warmup_s:
                continue
            key = f"{self.specs[f.session].width}x{self.specs[f.session].height}"
            lat.setdefault(key, []).append(f.done_time - f.arrival)
        every = [x for v in lat.values() for x in v]
        span = max((f.done_time for f in self.finished + self.map_finished), default=0.0)
        maps = [j.done_time - j.arrival for j in self.map_finished if j.arrival >= warmup_s]

        def pct(v, q):
            return float(np.percentile(np.asarray(v) * 1e3, q)) if v else float("nan")

        return {
            "frames": len(self.finished),
            "frames_measured": len(every),
            "p50_ms": pct(every, 50), "p99_ms": pct(every, 99),
            "per_class": {k: {"frames": len(v), "p50_ms": pct(v, 50), "p99_ms": pct(v, 99)}
                          for k, v in sorted(lat.items())},
            "iters": self.iters, "steps": self.steps,
            "iters_per_s": self.iters / span if span > 0 else float("nan"),
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "span_s": span,
            "max_resident_bytes": self.max_resident,
            "async_mapping": self.cfg.async_mapping,
            "map_jobs": len(self.map_finished),
            "map_p50_ms": pct(maps, 50), "map_p99_ms": pct(maps, 99),
        }


def _log2_ratio(n, k, m):
    """Downsampling schedule of Sec. 4.2 for non-keyframe n after keyframe k."""
    if n <= k:
        return 0
    return max(2, 4 - int(math.floor((n - k - 1) * math.log2(m) + 1e-12)))


# --------------------------------------------------------------------------- fake executor


class FakeExecutor:
    """CPU model of the GPU: an iteration of a batch costs
    launch + sum over frames of (a * pixels + b * gaussians), with a higher
    per-launch cost when frames are served one by one.  Time is simulated."""

    def __init__(self, launch_s=2e-4, per_pixel_s=1.5e-9, per_gauss_s=1.0e-9,
                 bytes_per_gauss=400, ws_per_gauss=60):
        self.launch_s = launch_s
        self.a = per_pixel_s
        self.b = per_gauss_s
        self.bpg = bytes_per_gauss
        self.wpg = ws_per_gauss
        self.now = 0.0
        self.opened = set()
        self.log = []

    def clock(self):
        return self.now

    def start_clock(self):
        pass

    def session_bytes(self, spec):
        return spec.n * self.bpg + 16 * spec.pixels * 8

    def step_bytes(self, spec, frame):
        return spec.n * self.wpg + 12 * spec.pixels

    def open_session(self, s, spec):
        self.opened.add(s)

    def close_session(self, s):
        self.opened.discard(s)

    def start_frame(self, f, spec):
        pass

    def finish_frame(self, f, spec):
        pass

    def start_map(self, job, spec):
        pass

    def finish_map(self, job, spec):
        pass

    def run_iteration(self, phase, frames, specs):
        cost = self.launch_s
        for f, sp in zip(frames, specs):
            frac = 1.0 / (2 ** f.log2_ratio) if phase == "track" else 1.0
            cost += self.a * sp.pixels * frac + self.b * sp.n * (2.0 if phase == "map" else 1.0)
        self.now += cost
        self.log.append((phase, tuple(f.session for f in frames)))
        return self.now

    def idle(self, dt):
        self.now += dt

    def sync(self):
        pass

    def event_time(self, ev):
        return ev


# --------------------------------------------------------------------------- GPU executor


class GpuExecutor:
    """Runs sessions on the HIP library with batched launches.

    A session's map exists in versions: version 0 at open, and version v + 1
    written by its v + 1-th keyframe map job (asynchronous mapping) into
    tensors of its own, so frames that render version v meanwhile see it
    unchanged.  Without asynchronous mapping the frames' own mapping
    iterations update the single version in place (a session's frames then
    run one after another)."""

    def __init__(self, device=0, lr_pose=(1e-3, 3e-3), track_noise_seed=0, n_targets=4,
                 capacity_factor=2.0, prune=False, prune_ratio=0.1, prune_cap=0.5,
                 prune_lam=0.8, record_poses=False, fused=True):
        import torch

        from . import rtgs
        self.torch = torch
        self.rtgs = rtgs
        self.dev = torch.device("cuda", device)
        self.handle = rtgs.Handle(device)
        self.sessions = {}
        self.lr_rho, self.lr_phi = lr_pose
        self.n_targets = n_targets
        self.capacity_factor = capacity_factor
        self.base_event = None
        self.base_wall = None
        self.overflows = 0
        # adaptive pruning (Sec. 4.1) per tracked frame: the frame's first
        # iteration scores the map (Eq. 7) and masks up to prune_ratio of its
        # visible Gaussians for the frame's other iterations; a keyframe's
        # map job removes the Gaussians its keyframe masked, never more than
        # prune_cap of the initial map in all
        # fused: the forward writes the loss gradient and map jobs update their
        # maps inside the backward; otherwise a loss pass and adam_step (the
        # same results, bit for bit)
        self.fused = fused
        self.prune = prune
        self.prune_ratio = prune_ratio
        self.prune_cap = prune_cap
        self.prune_lam = prune_lam
        self.record_poses = record_poses
        self.frame_poses = {}    # (session, frame) -> end pose, with record_poses
        # every launch goes to the stream current at construction
        self.stream_obj = torch.cuda.current_stream(self.dev)
        self.stream = rtgs.stream_ptr(self.stream_obj)

    # ---- footprint -----------------------------------------------------------
    def session_bytes(self, spec):
        # parameters, their gradients and two Adam moments (56 B each), target
        # frames (16 B per pixel each), per-frame outputs
        return spec.n * 56 * 4 + self.n_targets * 16 * spec.pixels + 40 * spec.pixels

    def _cap(self, spec):
        return int(self.capacity_factor * (12 * spec.n + 4 * _tiles(spec.width, spec.height)))

    def step_bytes(self, spec, frame):
        return self.rtgs.rtgs_workspace_size(spec.n, spec.width, spec.height, self._cap(spec))

    def _eye(self):
        return self.torch.eye(3, 4, dtype=self.torch.float32, device=self.dev).contiguous()

    # ---- sessions ------------------------------------------------------------
    def open_session(self, s, spec):
        if s in self.sessions:
            self._restore(s)
            return
        torch = self.torch
        cfg = synth.CONFIGS[spec.kind]
        sspec = synth.SceneSpec(f"s{s}", spec.width, spec.height, spec.n, spec.seed,
                                cfg.log_scale_mean, cfg.log_scale_std, cfg.z_near, cfg.z_far,
                                cfg.transparent_frac)
        cam = synth.make_camera(spec.width, spec.height)
        sc = synth.make_scene(sspec, cam)
        params = [torch.from_numpy(a).to(self.dev) for a in sc.arrays()]
        rc = self.rtgs.Cam(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)
        # targets: the scene seen from small pose offsets (the frames of a slow
        # trajectory), plus sensor noise; rendered once at session open
        r = self.rtgs.Renderer(self.dev.index, check="every")
        targets = []
        for k in range(self.n_targets):
            xi = torch.tensor(synth.pose_offset(spec.seed * 31 + k, 0.01, 0.5),
                              dtype=torch.float64, device=self.dev)
            from .pose import apply_left
            vm = apply_left(xi, self._eye())
            st = r.forward(tuple(params), vm.contiguous(), rc)
            g = torch.Generator(device=self.dev).manual_seed(spec.seed + k)
            targets.append((st.color + 0.01 * torch.randn(st.color.shape, generator=g,
                                                          device=self.dev),
                            st.depth + 0.01 * torch.randn(st.depth.shape, generator=g,
                                                          device=self.dev)))
        from .optim import MapAdam
        maps = [p.clone() for p in params]
        opt = MapAdam(maps, eps=1e-15)
        self.sessions[s] = dict(
            spec=spec, cam=rc, params=maps, opt=opt, targets=targets,
            versions={0: maps}, version=0,
            viewmat=self._eye(),           # end pose of the latest finished frame
            poses={}, final_T={},          # frame index -> end pose / last final T
            out_map=self._outs(spec),
            n0=spec.n, removed=0, inflight=0)
        torch.cuda.synchronize(self.dev)

    def _outs(self, spec):
        torch = self.torch
        return dict(color=torch.empty(3, spec.height, spec.width, device=self.dev),
                    depth=torch.empty(spec.height, spec.width, device=self.dev),
                    alpha=torch.empty(spec.height, spec.width, device=self.dev),
                    final_T=torch.empty(spec.height, spec.width, device=self.dev),
                    last_idx=torch.empty(spec.height, spec.width, dtype=torch.int32,
                                         device=self.dev))

    def close_session(self, s):
        """Evict an idle session: its latest map version, Adam moments, poses
        and targets move to host memory (older versions and transmittance
        images are dropped)."""
        S = self.sessions.get(s)
        if S is None or S.get("offloaded"):
            return
        S["params"] = [p.cpu() for p in S["params"]]
        S["versions"] = {S["version"]: S["params"]}
        S["opt"].to("cpu").rebind(S["params"])
        S["viewmat"] = S["viewmat"].cpu()
        S["poses"] = {k: v.cpu() for k, v in S["poses"].items()}
        S["final_T"] = {}
        S["targets"] = [(c.cpu(), d.cpu()) for c, d in S["targets"]]
        S["out_map"] = {k: v.cpu() for k, v in S["out_map"].items()}
        S["offloaded"] = True

    def _restore(self, s):
        S = self.sessions[s]
        S["params"] = [p.to(self.dev) for p in S["params"]]
        S["versions"] = {S["version"]: S["params"]}
        S["opt"].to(self.dev).rebind(S["params"])
        S["viewmat"] = S["viewmat"].to(self.dev)
        S["poses"] = {k: v.to(self.dev) for k, v in S["poses"].items()}
        S["targets"] = [(c.to(self.dev), d.to(self.dev)) for c, d in S["targets"]]
        S["out_map"] = {k: v.to(self.dev) for k, v in S["out_map"].items()}
        S["offloaded"] = False

    # ---- frames ----------------------------------------------------------------
    def _bind(self, x, S, spec, params, phase):
        """The ctypes records of a frame or map job, built once: its session
        record (map version, pose, masks, outputs, upstream and output
        gradients), loss record, and pose or Adam records.  Each iteration
        then only copies them into the call's arrays."""
        torch, rtgs = self.torch, self.rtgs
        n = params[0].shape[0]
        o = x.out
        x.gc = torch.empty_like(o["color"])
        x.gd = torch.empty_like(o["depth"])
        it = dict(scene=tuple(p.detach() for p in params), viewmat=x.viewmat, cam=S["cam"],
                  pixel_mask=x.mask, sample_log2=x.log2_ratio if x.mask is not None else 0,
                  color=o["color"], depth=o["depth"], alpha=o["alpha"], final_T=o["final_T"],
                  last_idx=o["last_idx"], visible=x.visible, dL_dcolor=x.gc, dL_ddepth=x.gd)
        if phase == "track":
            it["g_pose6"] = x.gpose
            if x.first:                             # scores the map on its first iteration
                x.g_means = torch.empty(n, 3, device=self.dev)
                x.g_cov3d = torch.empty(n, 6, device=self.dev)
                it.update(g_means=x.g_means, g_cov3d=x.g_cov3d)
        else:
            x.grads = [torch.empty_like(p) for p in params]
            x.g_cov3d = torch.empty(n, 6, device=self.dev)   # read when some job scores
            it.update(g_means=x.grads[0], g_log_scales=x.grads[1], g_quats=x.grads[2],
                      g_opacity_logits=x.grads[3], g_colors=x.grads[4], g_cov3d=x.g_cov3d)
        # L1 colour + 0.5 L1 depth over the active pixels, its gradient written
        # by the forward as it writes the image (or by a loss pass)
        if self.fused:
            x.l1c = rtgs.l1_loss(x.target[0], x.target[1], x.gc, x.gd,
                                 x.pcount if x.mask is not None else None, 1.0, 0.5)
            it["l1"] = x.l1c
        else:
            x.cl = rtgs.loss_item(o["color"], o["depth"], x.target[0], x.target[1], x.gc, x.gd,
                                  x.mask, x.pcount if x.mask is not None else None)
        x.keep = it
        x.cs = rtgs.session_struct(it)
        x.n = n
        x.phase_bound = phase

    def start_frame(self, f, spec):
        """A frame tracks its own pose, from the end pose of frame f.pose_from
        (the identity for a session's first frames), with its own Adam state
        and output buffers, on map version f.version.  A downsampled frame
        takes its pixel mask from frame f.pose_from's final transmittance."""
        torch = self.torch
        S = self.sessions[f.session]
        if f.version not in S["versions"]:
            raise RuntimeError(f"session {f.session}: map version {f.version} is gone "
                               f"(have {sorted(S['versions'])})")
        S["inflight"] += 1
        f.params = S["versions"][f.version]
        n = f.params[0].shape[0]
        f.first = self.prune
        f.gmask = None
        f.visible = torch.empty(n, dtype=torch.uint8, device=self.dev)
        f.target = S["targets"][f.index % self.n_targets]
        f.viewmat = (S["poses"][f.pose_from].clone() if f.pose_from >= 0 else self._eye())
        f.m = torch.zeros(6, device=self.dev)
        f.v = torch.zeros(6, device=self.dev)
        f.t = 0
        f.gpose = torch.zeros(6, device=self.dev)
        f.out = self._outs(spec)
        f.mask = None
        f.pcount = None
        if f.log2_ratio > 0 and f.pose_from in S["final_T"]:
            f.mask = torch.empty(spec.height, spec.width, dtype=torch.uint8, device=self.dev)
            f.pcount = torch.zeros(1, dtype=torch.int32, device=self.dev)
            self.rtgs.downsample_mask(S["final_T"][f.pose_from], f.log2_ratio, f.mask,
                                      f.pcount, stream=self.stream_obj)
        self._bind(f, S, spec, f.params, "track")
        f.cp = self.rtgs.pose_item(f.viewmat, f.gpose, f.m, f.v, self.lr_rho, self.lr_phi)

    def finish_frame(self, f, spec):
        S = self.sessions[f.session]
        S["viewmat"] = f.viewmat
        S["poses"][f.index] = f.viewmat
        S["final_T"][f.index] = f.out["final_T"]
        for d in (S["poses"], S["final_T"]):           # what no later frame reads
            for k in [k for k in d if k < f.index - 4]:
                del d[k]
        f.pose_end = f.viewmat                      # a keyframe's tracked pose
        if self.record_poses:
            self.frame_poses[(f.session, f.index)] = f.viewmat
        S["inflight"] -= 1
        f.gmask = f.cs = f.l1c = f.cl = f.cp = f.keep = f.grads = None

    def start_map(self, job, spec):
        """A keyframe's map job: version v + 1 starts as a copy of the latest
        version v and is trained at the keyframe's tracked pose; frames on
        version v keep rendering it meanwhile.  When pruning, the job's first
        iteration also scores its map (Eq. 7) and masks up to prune_ratio of
        the Gaussians it sees; its later iterations render without them, and
        they are removed (map and Adam moments) when the job ends (Sec. 4.1:
        mask for K iterations, then remove)."""
        torch, rtgs = self.torch, self.rtgs
        S = self.sessions[job.session]
        base = S["versions"][S["version"]]
        new = [p.clone() for p in base]
        opt = S["opt"]
        opt.rebind(new)
        job.params = new
        job.target = job.frame.target
        job.mask = None
        job.pcount = None
        job.viewmat = job.frame.pose_end
        job.first = self.prune
        job.gmask = None
        job.visible = torch.empty(new[0].shape[0], dtype=torch.uint8, device=self.dev)
        job.out = S["out_map"]
        self._bind(job, S, spec, new, "map")
        if not self.fused:
            job.ca = (rtgs.CAdamGroup * len(new))(*[
                rtgs.adam_group(p, g, m, v, lr) for p, g, m, v, lr in
                zip(new, job.grads, opt.exp_avg, opt.exp_avg_sq, opt.lrs)])
            return
        # the job's Adam update runs inside its backward (RTGS_GRAD_ADAM,
        # bitwise the update of adam_step), so its map gradients need not be
        # written, except dL/dmu while the job scores its map (dL/dSigma stays:
        # a launch in which another job scores asks every session for it)
        job.cadam = opt.fused()
        job.cs.adam = ctypes.pointer(job.cadam)
        job.cs.g_log_scales = job.cs.g_quats = job.cs.g_opacity_logits = job.cs.g_colors = None
        if not job.first:
            job.cs.g_means = None

    def _remove_masked(self, S, job):
        """Permanent removal of the Gaussians the job masked (stable
        compaction of the map and its Adam moments)."""
        torch, rtgs = self.torch, self.rtgs
        mask, job.gmask = job.gmask, None
        n = job.params[0].shape[0]
        job.ev_count.synchronize()                  # recorded iterations ago
        k = n - int(job.h_count.item())
        if k >= n:
            return
        opt = S["opt"]
        srcs = list(job.params) + list(opt.exp_avg) + list(opt.exp_avg_sq)
        outs = [torch.empty((k,) + tuple(t.shape[1:]), dtype=t.dtype, device=t.device)
                for t in srcs]
        cnt = torch.empty(1, dtype=torch.int32, device=self.dev)
        rtgs.compact_by_mask(mask, list(zip(srcs, outs)), cnt, stream=self.stream_obj)
        npar = len(job.params)
        job.params = outs[:npar]
        opt.rebind(job.params)
        opt.exp_avg = outs[npar:2 * npar]
        opt.exp_avg_sq = outs[2 * npar:]
        S["removed"] += n - k

    def finish_map(self, job, spec):
        """Publish the job's map as the session's next version."""
        S = self.sessions[job.session]
        if job.gmask is not None:
            self._remove_masked(S, job)
        S["version"] += 1
        S["versions"][S["version"]] = job.params
        S["params"] = job.params
        job.cs = job.l1c = job.cl = job.ca = job.cadam = job.keep = job.grads = None

    def release_versions(self, s, keep_from):
        """Forget map versions below keep_from (frames that render them hold
        their own references)."""
        S = self.sessions[s]
        for v in [v for v in S["versions"] if v < keep_from and v != S["version"]]:
            del S["versions"][v]

    # ---- one iteration for a group of frames -----------------------------------
    def run_iteration(self, phase, frames, specs):
        torch, rtgs = self.torch, self.rtgs
        st = self.stream
        k = len(frames)
        cap = 0
        for x in frames:
            if getattr(x, "phase_bound", None) != phase:     # a frame's in-line mapping
                self._bind(x, self.sessions[x.session], self.sessions[x.session]["spec"],
                           x.params, phase)
            cap += self._cap(self.sessions[x.session]["spec"])
        arr = (rtgs.CSession * k)(*[x.cs for x in frames])
        ws = torch.empty(rtgs.rtgs_workspace_size_batched(
            [x.n for x in frames], [x.out["depth"].shape[1] for x in frames],
            [x.out["depth"].shape[0] for x in frames], cap), dtype=torch.uint8, device=self.dev)
        # the forward also writes each frame's loss gradient (its session's l1)
        rtgs.render_fwd_batched_c(self.handle, arr, k, ws, cap, rtgs.RTGS_FWD_SAVE_STATE, st)
        if not self.fused:                  # one loss launch for the group
            rtgs.loss_l1_grad_batched_c((rtgs.CLossItem * k)(*[x.cl for x in frames]), k, 1.0,
                                        0.5, st)
        scoring = [x for x in frames if x.first]
        if phase == "track":
            flags = rtgs.RTGS_GRAD_POSE | (rtgs.RTGS_GRAD_SCORE if scoring else 0)
            rtgs.render_bwd_batched_c(self.handle, arr, k, ws, cap, flags, st)
            for f in frames:
                f.t += 1
                f.cp.step = f.t
            # Adam on xi = (rho, phi) for every frame, then T <- Exp(-step) T
            rtgs.pose_update_c((rtgs.CPoseItem * k)(*[f.cp for f in frames]), k, 0.9, 0.999,
                               1e-8, st)
        else:
            # map jobs update their maps inside the backward; frames that map
            # in line take one adam_step launch for every session of the group
            fused = [x for x in frames if getattr(x, "cadam", None) is not None]
            flags = (rtgs.RTGS_GRAD_MAP | (rtgs.RTGS_GRAD_COV3D if scoring else 0)
                     | (rtgs.RTGS_GRAD_ADAM if fused else 0))
            for x in fused:                          # read by the call through x.cs.adam
                x.cadam.step = self.sessions[x.session]["opt"].t + 1
            rtgs.render_bwd_batched_c(self.handle, arr, k, ws, cap, flags, st)
            for x in fused:
                self.sessions[x.session]["opt"].t += 1
            groups = []
            for x in frames:
                if getattr(x, "cadam", None) is not None:
                    continue
                opt = getattr(x, "opt", None) or self.sessions[x.session]["opt"]
                if getattr(x, "ca", None) is None:            # in-line mapping of a frame
                    x.ca = (rtgs.CAdamGroup * len(x.params))(*[
                        rtgs.adam_group(p, g, m, v, lr) for p, g, m, v, lr in
                        zip(x.params, x.grads, opt.exp_avg, opt.exp_avg_sq, opt.lrs)])
                opt.t += 1
                for grp in x.ca:
                    grp.step = opt.t
                    groups.append(grp)
            if groups:
                rtgs.adam_step_c(self.handle, (rtgs.CAdamGroup * len(groups))(*groups),
                                 len(groups), 0.9, 0.999, 1e-15, st)
        for x in scoring:
            self._mask_lowest(self.sessions[x.session], x)
            x.first = False
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        return ev

    def _mask_lowest(self, S, x):
        """Mask of a frame or map job (Sec. 4.1, Eq. 7): up to prune_ratio of
        the visible Gaussians with the lowest importance, within what the 50%
        cap still allows for the map version it renders.  A frame renders its
        later iterations without them; a job also removes them when it ends."""
        torch, rtgs = self.torch, self.rtgs
        n = x.params[0].shape[0]
        budget = max(0.0, self.prune_cap * S["n0"] - (S["n0"] - n))
        ratio = min(self.prune_ratio, budget / max(n, 1), 0.5)
        mask = torch.zeros(n, dtype=torch.uint8, device=self.dev)
        g_means = x.grads[0] if x.phase_bound == "map" else x.g_means
        job = isinstance(x, MapJob)
        count = torch.zeros(1, dtype=torch.int32, device=self.dev) if job else None
        rtgs.prune_by_grad(self.handle, g_means, x.g_cov3d, x.visible, None, self.prune_lam,
                           ratio, mask, count, stream=self.stream_obj)
        if job:
            x.h_count = torch.zeros(1, dtype=torch.int32).pin_memory()
            x.h_count.copy_(count, non_blocking=True)
            x.ev_count = torch.cuda.Event()
            x.ev_count.record()
        x.gmask = mask
        x.keep["gauss_mask"] = mask
        x.cs.g.gauss_mask = mask.data_ptr()
        if not job:                                   # the score outputs were one-off
            x.cs.g_means = None
            x.cs.g_cov3d = None
            x.g_means = x.g_cov3d = None
        elif getattr(x, "cadam", None) is not None:   # a fused job needs dL/dmu no more
            x.cs.g_means = None

    # ---- clock ----------------------------------------------------------------
    def clock(self):
        return time.perf_counter()

    def warmup(self, specs, iters=2):
        """Untimed tracking and mapping iterations per open session (first
        launches, allocator growth) on throwaway copies of the map: no session
        state changes."""
        from .optim import MapAdam
        for s in list(self.sessions):
            S = self.sessions[s]
            spec = S["spec"]
            for phase in ("track", "map"):
                f = Frame(s, 0, 0.0, True, 1, 1)
                self.start_frame(f, spec)
                f.params = [p.clone() for p in f.params]
                f.opt = MapAdam(f.params, eps=1e-15)
                f.phase_bound = None
                f.first = self.prune and phase == "track"
                for _ in range(iters):
                    self.run_iteration(phase, [f], [spec])
                S["inflight"] -= 1
        self.sync()

    def start_clock(self):
        torch = self.torch
        torch.cuda.synchronize(self.dev)
        self.base_event = torch.cuda.Event(enable_timing=True)
        self.base_event.record()
        torch.cuda.synchronize(self.dev)
        self.base_wall = 0.0

    def idle(self, dt):
        time.sleep(min(dt, 0.002))

    def sync(self):
        self.torch.cuda.synchronize(self.dev)

    def event_time(self, ev):
        return self.base_event.elapsed_time(ev) / 1e3

    def verify(self):
        code, pairs, _ = self.rtgs.rtgs_query(self.handle, True)
        if code != self.rtgs.RTGS_OK:
            self.overflows += 1
        return pairs


def _tiles(w, h):
    return ((w + 15) // 16) * ((h + 15) // 16)
