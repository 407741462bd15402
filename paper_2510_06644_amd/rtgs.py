"""ctypes binding of librtgs (include/rtgs.h): argument marshalling only.

Every step of the rasterizer runs in the HIP library; this module turns torch
tensors into device pointers and the current HIP stream into a handle.  There
is no fallback: if librtgs.so is missing or a tensor is not on the GPU the
call raises.

The entry points keep the C names (``render_fwd``, ``render_bwd``,
``render_fwd_batched``, ``render_bwd_batched``, ``prune_by_grad``,
``downsample_mask``, ``rtgs_query`` ...).  ``Renderer`` adds workspace and
pair-capacity management on top.
"""
from __future__ import annotations

import ctypes
import math
import dataclasses
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librtgs.so")

RTGS_OK = 0
RTGS_ERR_INVALID_ARG = -1
RTGS_ERR_CAPACITY = -2
RTGS_ERR_HIP = -3
RTGS_ERR_WORKSPACE = -4
RTGS_FWD_SAVE_STATE = 1
RTGS_FWD_STATS = 2
RTGS_FWD_REUSE_LISTS = 4
RTGS_FWD_SAVE_FRAGMENTS = 16
RTGS_FWD_BALANCE_LANES = 32
RTGS_PROFILE_STAGES = 16
STAGES = ("init", "preprocess", "scan", "emit", "sort", "raster_fwd", "adam", "raster_bwd",
          "preprocess_bwd", "pose_reduce", "bin_count", "merge")
RTGS_GRAD_POSE = 1
RTGS_GRAD_MAP = 2
RTGS_GRAD_COV3D = 4
RTGS_GRAD_RECOMPUTE_STATE = 8
RTGS_GRAD_SCORE = 16
RTGS_GRAD_SAVED_FRAGMENTS = 32
RTGS_GRAD_BALANCED_LANES = 64
RTGS_GRAD_ADAM = 128
RTGS_STATE_IDLE = 0
RTGS_STATE_EXECUTING = 1
RTGS_MAX_SESSIONS = 64
RTGS_SAMPLE_SHIFT = 8

EXPORTS = (
    "rtgs_last_error", "rtgs_create", "rtgs_destroy", "rtgs_workspace_size",
    "rtgs_workspace_size_batched", "render_fwd", "render_bwd", "render_fwd_batched",
    "render_bwd_batched", "prune_by_grad", "downsample_mask", "rtgs_downsample_log2_ratio",
    "rtgs_query", "rtgs_debug_stage", "rtgs_selftest_wave_sum", "rtgs_profile_enable",
    "rtgs_profile_read", "adam_step", "loss_l1_grad", "pose_update", "compact_by_mask",
    "rtgs_compact_scratch_size", "rtgs_tile_rects", "tile_pair_change", "loss_l1_grad_batched",
    "compact_by_mask_static",
)

vp = ctypes.c_void_p
i32 = ctypes.c_int32
i64 = ctypes.c_int64
u64 = ctypes.c_uint64
f32 = ctypes.c_float


class CLossItem(ctypes.Structure):
    _fields_ = [("color", vp), ("depth", vp), ("target_color", vp), ("target_depth", vp),
                ("pixel_mask", vp), ("n_active_dev", vp), ("dL_dcolor", vp), ("dL_ddepth", vp),
                ("width", i32), ("height", i32)]


class CCompactItem(ctypes.Structure):
    _fields_ = [("src", vp), ("dst", vp), ("row_bytes", i32), ("dst_rows", i32)]


class CGaussians(ctypes.Structure):
    _fields_ = [("means", vp), ("log_scales", vp), ("quats", vp), ("opacity_logits", vp),
                ("colors", vp), ("gauss_mask", vp), ("n", i32)]


class CCamera(ctypes.Structure):
    _fields_ = [("width", i32), ("height", i32), ("fx", f32), ("fy", f32), ("cx", f32),
                ("cy", f32), ("viewmat", vp)]


class CMapAdam(ctypes.Structure):
    _fields_ = [("exp_avg", vp * 5), ("exp_avg_sq", vp * 5), ("lr", f32 * 5), ("step", i32),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double)]


class CL1Loss(ctypes.Structure):
    _fields_ = [("target_color", vp), ("target_depth", vp), ("n_active_dev", vp),
                ("w_color", f32), ("w_depth", f32), ("dL_dcolor", vp), ("dL_ddepth", vp)]


class CSession(ctypes.Structure):
    _fields_ = [("g", CGaussians), ("cam", CCamera), ("pixel_mask", vp), ("sample_log2", i32),
                ("color", vp), ("depth", vp), ("alpha", vp), ("final_T", vp), ("last_idx", vp),
                ("visible", vp), ("stats", vp), ("dL_dcolor", vp), ("dL_ddepth", vp), ("dL_dalpha", vp),
                ("g_means", vp), ("g_log_scales", vp), ("g_quats", vp),
                ("g_opacity_logits", vp), ("g_colors", vp), ("g_pose6", vp), ("g_viewmat", vp),
                ("g_cov3d", vp), ("lane_work", vp), ("lane_work_out", vp),
                ("adam", ctypes.POINTER(CMapAdam)), ("l1", ctypes.POINTER(CL1Loss))]


class CPoseItem(ctypes.Structure):
    _fields_ = [("viewmat", vp), ("g_pose6", vp), ("exp_avg", vp), ("exp_avg_sq", vp),
                ("lr_rho", f32), ("lr_phi", f32), ("step", i32)]


class CAdamGroup(ctypes.Structure):
    _fields_ = [("param", vp), ("grad", vp), ("exp_avg", vp), ("exp_avg_sq", vp), ("n", i64),
                ("lr", f32), ("step", i32)]


_lib = None
_lock = threading.Lock()


class RtgsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librtgs error {code}: {msg}")
        self.code = code


def lib():
    """Load librtgs.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -c 'import __graft_entry__ as g; g.build()'`")
            L = ctypes.CDLL(LIB_PATH)
            L.rtgs_last_error.restype = ctypes.c_char_p
            L.rtgs_create.argtypes = [ctypes.POINTER(vp), i32]
            L.rtgs_destroy.argtypes = [vp]
            L.rtgs_workspace_size.argtypes = [i32, i32, i32, i64, i32, ctypes.POINTER(u64)]
            L.rtgs_workspace_size_batched.argtypes = [vp, vp, vp, i32, i64, i32,
                                                      ctypes.POINTER(u64)]
            L.render_fwd.argtypes = [vp, ctypes.POINTER(CGaussians), ctypes.POINTER(CCamera), vp,
                                     vp, u64, i64, vp, vp, vp, vp, vp, vp, i32, vp]
            L.render_bwd.argtypes = [vp, ctypes.POINTER(CGaussians), ctypes.POINTER(CCamera), vp,
                                     vp, u64, i64, vp, vp, vp, vp, vp, i32,
                                     vp, vp, vp, vp, vp, vp, vp, vp, vp]
            L.render_fwd_batched.argtypes = [vp, ctypes.POINTER(CSession), i32, vp, u64, i64,
                                             i32, vp]
            L.render_bwd_batched.argtypes = [vp, ctypes.POINTER(CSession), i32, vp, u64, i64,
                                             i32, vp]
            L.prune_by_grad.argtypes = [vp, vp, vp, vp, vp, i32, f32, f32, vp, vp, vp, vp]
            L.downsample_mask.argtypes = [vp, i32, i32, i32, vp, vp, vp]
            L.rtgs_compact_scratch_size.argtypes = [i32]
            L.rtgs_compact_scratch_size.restype = u64
            L.compact_by_mask.argtypes = [vp, i32, ctypes.POINTER(CCompactItem), i32, vp, u64,
                                          vp, vp]
            L.compact_by_mask_static.argtypes = [vp, i32, ctypes.POINTER(CCompactItem), i32, vp,
                                                 vp]
            L.rtgs_tile_rects.argtypes = [i32, i32, i32, i32, i64, vp, u64, vp, vp]
            L.tile_pair_change.argtypes = [vp, vp, vp, i32, vp, vp]
            L.loss_l1_grad_batched.argtypes = [ctypes.POINTER(CLossItem), i32, f32, f32, vp]
            L.pose_update.argtypes = [ctypes.POINTER(CPoseItem), i32, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, vp]
            L.loss_l1_grad.argtypes = [vp, vp, vp, vp, vp, vp, i32, i32, f32, f32, vp, vp, vp]
            L.adam_step.argtypes = [vp, ctypes.POINTER(CAdamGroup), i32, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, vp]
            L.rtgs_downsample_log2_ratio.argtypes = [i32, i32, i32, i32]
            L.rtgs_query.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i32)]
            L.rtgs_debug_stage.argtypes = [vp, vp, vp, vp, i32, i64, vp, u64, vp, vp, vp, vp,
                                           i64, vp]
            L.rtgs_selftest_wave_sum.argtypes = [vp, vp, i32, vp]
            L.rtgs_profile_enable.argtypes = [vp, i32]
            L.rtgs_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(i64)]
            for name in EXPORTS:
                getattr(L, name).restype = getattr(L, name).restype or i32
            L.rtgs_last_error.restype = ctypes.c_char_p
            _lib = L
    return _lib


def _check(code):
    if code != RTGS_OK:
        raise RtgsError(code, lib().rtgs_last_error().decode())
    return code


def _p(t):
    """Device pointer of a tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("librtgs takes GPU tensors only")
    if not t.is_contiguous():
        raise ValueError("librtgs takes contiguous tensors only")
    return ctypes.c_void_p(t.data_ptr())


def _f32(t, shape=None, name="tensor"):
    if t is None:
        return None
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Handle:
    """Owns an rtgs_handle_t (one per stream)."""

    def __init__(self, device: int = 0):
        self.ptr = ctypes.c_void_p()
        _check(lib().rtgs_create(ctypes.byref(self.ptr), int(device)))
        self.device = device

    def close(self):
        if self.ptr:
            lib().rtgs_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------- C entry points
def rtgs_workspace_size(n, width, height, pair_capacity, flags=0):
    out = u64()
    _check(lib().rtgs_workspace_size(int(n), int(width), int(height), int(pair_capacity),
                                     int(flags), ctypes.byref(out)))
    return int(out.value)


def rtgs_workspace_size_batched(ns, widths, heights, pair_capacity, flags=0):
    k = len(ns)
    a = (i32 * k)(*ns)
    w = (i32 * k)(*widths)
    h = (i32 * k)(*heights)
    out = u64()
    _check(lib().rtgs_workspace_size_batched(a, w, h, k, int(pair_capacity), int(flags),
                                             ctypes.byref(out)))
    return int(out.value)


@dataclasses.dataclass
class Cam:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


def _gauss(means, log_scales, quats, opacity_logits, colors, gauss_mask):
    n = means.shape[0]
    _f32(means, (n, 3), "means")
    _f32(log_scales, (n, 3), "log_scales")
    _f32(quats, (n, 4), "quats")
    _f32(opacity_logits, (n,), "opacity_logits")
    _f32(colors, (n, 3), "colors")
    if gauss_mask is not None and (gauss_mask.dtype != torch.uint8 or gauss_mask.numel() != n):
        raise ValueError("gauss_mask must be uint8 [n]")
    return CGaussians(_p(means), _p(log_scales), _p(quats), _p(opacity_logits), _p(colors),
                      _p(gauss_mask), n)


def _cam(cam: Cam, viewmat):
    _f32(viewmat, None, "viewmat")
    if viewmat.numel() != 12:
        raise ValueError("viewmat must hold 12 floats (3x4 row-major)")
    return CCamera(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx),
                   float(cam.cy), _p(viewmat))


def render_fwd(handle, means, log_scales, quats, opacity_logits, colors, viewmat, cam,
               ws, pair_capacity, out_color, out_depth, out_alpha, final_T=None, last_idx=None,
               visible=None, gauss_mask=None, pixel_mask=None, flags=RTGS_FWD_SAVE_STATE,
               stream=None):
    g = _gauss(means, log_scales, quats, opacity_logits, colors, gauss_mask)
    c = _cam(cam, viewmat)
    _check(lib().render_fwd(handle.ptr, ctypes.byref(g), ctypes.byref(c), _p(pixel_mask),
                            _p(ws), ws.numel() * ws.element_size(), int(pair_capacity),
                            _p(out_color), _p(out_depth), _p(out_alpha), _p(final_T),
                            _p(last_idx), _p(visible), int(flags), _stream(stream)))


def render_bwd(handle, means, log_scales, quats, opacity_logits, colors, viewmat, cam, ws,
               pair_capacity, final_T, last_idx, dL_dcolor, dL_ddepth, dL_dalpha=None,
               grad_flags=RTGS_GRAD_POSE | RTGS_GRAD_MAP, g_means=None, g_log_scales=None,
               g_quats=None, g_opacity_logits=None, g_colors=None, g_pose6=None, g_cov3d=None,
               gauss_mask=None, pixel_mask=None, stream=None, g_viewmat=None):
    g = _gauss(means, log_scales, quats, opacity_logits, colors, gauss_mask)
    c = _cam(cam, viewmat)
    _check(lib().render_bwd(handle.ptr, ctypes.byref(g), ctypes.byref(c), _p(pixel_mask),
                            _p(ws), ws.numel() * ws.element_size(), int(pair_capacity),
                            _p(final_T), _p(last_idx), _p(dL_dcolor), _p(dL_ddepth),
                            _p(dL_dalpha), int(grad_flags), _p(g_means), _p(g_log_scales),
                            _p(g_quats), _p(g_opacity_logits), _p(g_colors), _p(g_pose6),
                            _p(g_viewmat), _p(g_cov3d), _stream(stream)))


def session_struct(it):
    """One CSession from a dict with the keys of CSession (tensors or None)
    plus 'scene' (means, log_scales, quats, opacity_logits, colors),
    'viewmat', 'cam' (Cam), optional 'gauss_mask', 'sample_log2', 'adam'
    (a CMapAdam, e.g. MapAdam.fused()) and 'l1' (a CL1Loss, l1_loss()).  The
    struct holds raw pointers: the tensors and the CMapAdam / CL1Loss must
    outlive its use."""
    s = CSession()
    s.g = _gauss(*it["scene"], it.get("gauss_mask"))
    s.cam = _cam(it["cam"], it["viewmat"])
    s.sample_log2 = int(it.get("sample_log2", 0))
    for name in ("pixel_mask", "color", "depth", "alpha", "final_T", "last_idx", "visible",
                 "stats",
                 "dL_dcolor", "dL_ddepth", "dL_dalpha", "g_means", "g_log_scales", "g_quats",
                 "g_opacity_logits", "g_colors", "g_pose6", "g_viewmat", "g_cov3d",
                 "lane_work", "lane_work_out"):
        setattr(s, name, _p(it.get(name)))
    if it.get("adam") is not None:
        s.adam = ctypes.pointer(it["adam"])
    if it.get("l1") is not None:
        s.l1 = ctypes.pointer(it["l1"])
    return s


def l1_loss(target_color, target_depth, dL_dcolor, dL_ddepth, n_active=None, w_color=1.0,
            w_depth=0.5):
    """A CL1Loss: the forward of a session carrying it also writes the
    gradients loss_l1_grad would (same arguments, the forward's own colour,
    depth and pixel mask).  The tensors must outlive its use."""
    _, h, w = target_color.shape
    for t, shp in ((target_color, (3, h, w)), (dL_dcolor, (3, h, w)), (target_depth, (h, w)),
                   (dL_ddepth, (h, w))):
        _f32(t, shp)
    return CL1Loss(_p(target_color), _p(target_depth), _p(n_active), float(w_color),
                   float(w_depth), _p(dL_dcolor), _p(dL_ddepth))


def make_sessions(items):
    """items: list of dicts as `session_struct` takes; returns the ctypes
    array and the tensors it points to (keep them alive)."""
    arr = (CSession * len(items))()
    keep = []
    for i, it in enumerate(items):
        arr[i] = session_struct(it)
        keep.append(it)
    return arr, keep


def stream_ptr(stream=None):
    """The hipStream_t of a torch stream (default: the current one), to pass
    to the *_c calls below without a lookup per call."""
    return _stream(stream)


def render_fwd_batched(handle, sessions, ws, pair_capacity, flags=RTGS_FWD_SAVE_STATE,
                       stream=None):
    arr, _keep = make_sessions(sessions)
    render_fwd_batched_c(handle, arr, len(sessions), ws, pair_capacity, flags, _stream(stream))


def render_bwd_batched(handle, sessions, ws, pair_capacity,
                       grad_flags=RTGS_GRAD_POSE | RTGS_GRAD_MAP, stream=None):
    arr, _keep = make_sessions(sessions)
    render_bwd_batched_c(handle, arr, len(sessions), ws, pair_capacity, grad_flags,
                         _stream(stream))


# Calls on prebuilt ctypes arrays (session_struct, CLossItem, CPoseItem,
# CAdamGroup) and a stream pointer (stream_ptr): for loops that issue the same
# frames' calls many times, so that marshalling happens once per frame.
def render_fwd_batched_c(handle, arr, n, ws, pair_capacity, flags, stream):
    _check(lib().render_fwd_batched(handle.ptr, arr, n, _p(ws), ws.numel() * ws.element_size(),
                                    int(pair_capacity), int(flags), stream))


def render_bwd_batched_c(handle, arr, n, ws, pair_capacity, grad_flags, stream):
    _check(lib().render_bwd_batched(handle.ptr, arr, n, _p(ws), ws.numel() * ws.element_size(),
                                    int(pair_capacity), int(grad_flags), stream))


def loss_item(c, d, tc, td, gc, gd, mask=None, cnt=None):
    """A CLossItem for loss_l1_grad_batched_c (validated once)."""
    _, h, w = c.shape
    for t, shp in ((c, (3, h, w)), (tc, (3, h, w)), (gc, (3, h, w)), (d, (h, w)),
                   (td, (h, w)), (gd, (h, w))):
        _f32(t, shp, "loss image")
        _p(t)
    if mask is not None and (mask.dtype != torch.uint8 or tuple(mask.shape) != (h, w)):
        raise ValueError("pixel_mask must be uint8 [H, W]")
    if mask is not None and cnt is None:
        raise ValueError("a pixel mask needs its device active-pixel count")
    return CLossItem(*(t.data_ptr() if t is not None else None
                       for t in (c, d, tc, td, mask, cnt, gc, gd)), w, h)


def loss_l1_grad_batched_c(arr, n, w_color, w_depth, stream):
    _check(lib().loss_l1_grad_batched(arr, n, float(w_color), float(w_depth), stream))


def pose_item(vm, g, m, v, lr_rho, lr_phi, step=1):
    """A CPoseItem for pose_update_c (validated once; set .step per call)."""
    _f32(vm, (3, 4), "viewmat")
    for t in (g, m, v):
        _f32(t, (6,), "pose vector")
    return CPoseItem(_p(vm), _p(g), _p(m), _p(v), float(lr_rho), float(lr_phi), int(step))


def pose_update_c(arr, n, beta1, beta2, eps, stream):
    _check(lib().pose_update(arr, n, float(beta1), float(beta2), float(eps), stream))


def adam_group(p, g, m, v, lr, step=1):
    """A CAdamGroup for adam_step_c (validated once; set .step per call)."""
    for t in (p, g, m, v):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != p.numel():
            raise ValueError("adam_step: contiguous float32 tensors of one size expected")
    return CAdamGroup(_p(p), _p(g), _p(m), _p(v), p.numel(), float(lr), int(step))


def adam_step_c(handle, arr, n, beta1, beta2, eps, stream):
    _check(lib().adam_step(handle.ptr, arr, n, float(beta1), float(beta2), float(eps), stream))


def prune_by_grad(handle, g_means, g_cov3d, visible, mask_in, lam, max_ratio, mask_out,
                  n_masked=None, score_out=None, stream=None):
    n = g_means.shape[0]
    _check(lib().prune_by_grad(handle.ptr, _p(g_means), _p(g_cov3d), _p(visible), _p(mask_in),
                               n, float(lam), float(max_ratio), _p(mask_out), _p(n_masked),
                               _p(score_out), _stream(stream)))


def loss_l1_grad_batched(items, w_color=1.0, w_depth=0.5, stream=None):
    """items: iterable of (color, depth, target_color, target_depth, dL_dcolor,
    dL_ddepth, pixel_mask or None, n_active or None); loss_l1_grad for each,
    one launch per 32 frames."""
    items = list(items)
    arr = (CLossItem * max(len(items), 1))()
    for k, (c, d, tc, td, gc, gd, mask, cnt) in enumerate(items):
        arr[k] = loss_item(c, d, tc, td, gc, gd, mask, cnt)
    loss_l1_grad_batched_c(arr, len(items), w_color, w_depth, _stream(stream))


RTGS_COMPACT_MAX_ITEMS = 24


RTGS_COMPACT_STATIC_MAX_ROWS = 16776192


def _compact_items(n, pairs):
    pairs = list(pairs)
    if len(pairs) > RTGS_COMPACT_MAX_ITEMS:
        raise ValueError(f"compact_by_mask: at most {RTGS_COMPACT_MAX_ITEMS} arrays")
    arr = (CCompactItem * max(len(pairs), 1))()
    for k, (src, dst) in enumerate(pairs):
        if not (src.is_contiguous() and dst.is_contiguous()) or src.dtype != dst.dtype:
            raise ValueError("compact_by_mask: contiguous src / dst of one dtype")
        if src.shape[0] != n or src.shape[1:] != dst.shape[1:]:
            raise ValueError("compact_by_mask: src has n rows and dst the same row shape")
        row = math.prod(src.shape[1:]) * src.element_size()
        _p(src), _p(dst)            # device, contiguous
        arr[k] = CCompactItem(src.data_ptr(), dst.data_ptr(), row, dst.shape[0])
    return arr, len(pairs)


def compact_by_mask(drop, pairs, n_kept, scratch=None, stream=None):
    """Stable removal of the rows i with drop[i] != 0 (drop: device uint8 [n]):
    for each (src, dst) pair of contiguous device tensors with n rows, dst[:k]
    receives the kept rows of src in order (k is written to the device int32
    n_kept).  dst needs at least the kept rows."""
    n = drop.numel()
    arr, k = _compact_items(n, pairs)
    need = int(lib().rtgs_compact_scratch_size(n))
    if scratch is None:
        scratch = torch.empty(max(need, 4), dtype=torch.uint8, device=drop.device)
    _check(lib().compact_by_mask(_p(drop), n, arr, k, _p(scratch),
                                 scratch.numel() * scratch.element_size(), _p(n_kept),
                                 _stream(stream)))


def compact_by_mask_static(drop, pairs, n_kept, stream=None):
    """compact_by_mask with the library's static device scratch: no allocation
    (n at most RTGS_COMPACT_STATIC_MAX_ROWS; calls on one GPU must not
    overlap)."""
    n = drop.numel()
    arr, k = _compact_items(n, pairs)
    _check(lib().compact_by_mask_static(_p(drop), n, arr, k, _p(n_kept), _stream(stream)))


def rtgs_tile_rects(st, rect_out, stream=None):
    """Tile rectangles (x0, y0, x1, y1) of the Gaussians of a full forward's
    state st into rect_out (device int32 [n, 4])."""
    _check(lib().rtgs_tile_rects(st.n, st.cam.width, st.cam.height, int(st.sample_log2), st.cap,
                                 _p(st.ws), st.ws.numel() * st.ws.element_size(), _p(rect_out),
                                 _stream(stream)))


def tile_pair_change(rect_ref, rect_cur, skip, out, stream=None):
    """out (device int64 [2]) = (pairs in exactly one of the two rectangles,
    pairs of rect_ref), over the Gaussians with skip == 0 (skip may be None)."""
    n = rect_ref.shape[0]
    if tuple(rect_cur.shape) != (n, 4) or tuple(rect_ref.shape) != (n, 4):
        raise ValueError("tile_pair_change: two [n, 4] rectangle arrays")
    _check(lib().tile_pair_change(_p(rect_ref), _p(rect_cur), _p(skip), n, _p(out),
                                  _stream(stream)))


def pose_update(items, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """items: iterable of (viewmat [3,4], g_pose6 [6], exp_avg [6], exp_avg_sq [6],
    lr_rho, lr_phi, step); Adam on xi then viewmat <- Exp(-step) viewmat, in
    place on the device."""
    items = list(items)
    arr = (CPoseItem * max(len(items), 1))()
    for k, (vm, g, m, v, lr_rho, lr_phi, step) in enumerate(items):
        arr[k] = pose_item(vm, g, m, v, lr_rho, lr_phi, step)
    pose_update_c(arr, len(items), beta1, beta2, eps, _stream(stream))


def loss_l1_grad(color, depth, target_color, target_depth, dL_dcolor, dL_ddepth,
                 pixel_mask=None, n_active=None, w_color=1.0, w_depth=0.5, stream=None):
    """dL/dC and dL/dD of the L1 colour + w_depth L1 depth loss (means over
    the active pixels); n_active is a device int32 count (required with a
    mask)."""
    _, h, w = color.shape
    for t, shp in ((color, (3, h, w)), (target_color, (3, h, w)), (dL_dcolor, (3, h, w)),
                   (depth, (h, w)), (target_depth, (h, w)), (dL_ddepth, (h, w))):
        _f32(t, shp)
    _check(lib().loss_l1_grad(_p(color), _p(depth), _p(target_color), _p(target_depth),
                              _p(pixel_mask), _p(n_active), w, h, float(w_color), float(w_depth),
                              _p(dL_dcolor), _p(dL_ddepth), _stream(stream)))


def adam_step(handle, groups, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """groups: iterable of (param, grad, exp_avg, exp_avg_sq, lr, step); the
    four tensors are contiguous float32 device tensors of one size, updated in
    place."""
    groups = list(groups)
    arr = (CAdamGroup * max(len(groups), 1))()
    for k, (p, g, m, v, lr, step) in enumerate(groups):
        arr[k] = adam_group(p, g, m, v, lr, step)
    adam_step_c(handle, arr, len(groups), beta1, beta2, eps, _stream(stream))


def downsample_mask(final_T, log2_ratio, mask_out, n_active=None, stream=None):
    h, w = final_T.shape
    _check(lib().downsample_mask(_p(final_T), w, h, int(log2_ratio), _p(mask_out),
                                 _p(n_active), _stream(stream)))


def rtgs_downsample_log2_ratio(is_keyframe, n, k, m=2):
    r = lib().rtgs_downsample_log2_ratio(int(bool(is_keyframe)), int(n), int(k), int(m))
    if r < 0:
        _check(r)
    return r


def rtgs_query(handle, blocking=True):
    """(status, pairs_needed, state); status is RTGS_OK or RTGS_ERR_CAPACITY."""
    pairs = i64()
    state = i32()
    code = lib().rtgs_query(handle.ptr, int(bool(blocking)), ctypes.byref(pairs),
                            ctypes.byref(state))
    if code not in (RTGS_OK, RTGS_ERR_CAPACITY):
        _check(code)
    return code, int(pairs.value), int(state.value)


def rtgs_debug_stage(ns, widths, heights, pair_capacity, ws, stage=None, rect=None,
                     ranges=None, ids=None, stream=None, sample_log2=None):
    k = len(ns)
    a = (i32 * k)(*ns)
    w = (i32 * k)(*widths)
    h = (i32 * k)(*heights)
    j = None if sample_log2 is None else (i32 * k)(*sample_log2)
    _check(lib().rtgs_debug_stage(a, w, h, j, k, int(pair_capacity), _p(ws),
                                  ws.numel() * ws.element_size(), _p(stage), _p(rect),
                                  _p(ranges), _p(ids), 0 if ids is None else ids.numel(),
                                  _stream(stream)))


def rtgs_profile_enable(handle, stages):
    """Enable HIP-event timing for the named stages (iterable of names)."""
    mask = 0
    for s in stages:
        mask |= 1 << STAGES.index(s)
    _check(lib().rtgs_profile_enable(handle.ptr, mask))


def rtgs_profile_read(handle):
    """{stage: (total_ms, launches)} for stages with launches; clears."""
    ms = (ctypes.c_double * RTGS_PROFILE_STAGES)()
    cnt = (i64 * RTGS_PROFILE_STAGES)()
    _check(lib().rtgs_profile_read(handle.ptr, ms, cnt))
    return {STAGES[i]: (ms[i], int(cnt[i])) for i in range(len(STAGES)) if cnt[i] > 0}


def rtgs_selftest_wave_sum(inp, out, stream=None):
    """inp: [n_waves * 10 * 64], out: [n_waves * 10] device float tensors."""
    if out.numel() % 10 or inp.numel() != out.numel() * 64:
        raise ValueError("rtgs_selftest_wave_sum: 640 inputs and 10 outputs per wave")
    _check(lib().rtgs_selftest_wave_sum(_p(inp), _p(out), out.numel() // 10, _stream(stream)))


# --------------------------------------------------------------------------- managed renderer
def _tiles(w, h):
    return ((w + 15) // 16) * ((h + 15) // 16)


class Renderer:
    """Workspace + pair-capacity management around render_fwd / render_bwd.

    check="every": after each forward, a blocking rtgs_query verifies the
    pair capacity and re-renders with a larger buffer if it overflowed (one
    host sync per forward).  check="deferred": no per-call sync; call
    ``verify()`` at a point of your choosing (it raises if any forward since
    the last verify overflowed, after growing the capacity)."""

    def __init__(self, device=0, check="every", pairs_per_gaussian=12.0, min_capacity=1 << 16):
        self.handle = Handle(device)
        self.device = torch.device("cuda", device)
        self.check = check
        self.ppg = pairs_per_gaussian
        self.min_cap = min_capacity
        self.cap = 0
        self.ws = None

    def _ensure(self, ns, ws_, hs, cap):
        cap = max(int(cap), self.min_cap)
        if cap > self.cap:
            self.cap = cap
        need = rtgs_workspace_size_batched(ns, ws_, hs, self.cap)
        if self.ws is None or self.ws.numel() < need:
            self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        return self.ws, self.cap

    def workspace(self, ns, widths, heights):
        est = int(self.ppg * sum(ns)) + 4 * sum(_tiles(w, h) for w, h in zip(widths, heights))
        return self._ensure(ns, widths, heights, max(self.cap, est))

    def grow(self, needed):
        self.cap = max(self.cap, int(needed * 1.25) + 1024)

    def verify(self):
        code, pairs, _ = rtgs_query(self.handle, True)
        if code == RTGS_ERR_CAPACITY:
            self.grow(pairs)
            raise RtgsError(code, f"pair capacity exceeded: {pairs} needed")
        return pairs

    # ------------------------------------------------------------------ managed calls
    def forward(self, scene, viewmat, cam: Cam, gauss_mask=None, pixel_mask=None,
                save_state=True, stream=None, sample_log2=0, reuse_lists_of=None,
                save_fragments=False, balance=False, lane_work=None, lane_work_out=None,
                l1=None):
        """Render one frame; returns a FwdState (outputs + the workspace the
        matching backward needs).  Each forward gets its own workspace from
        torch's caching allocator, so several forwards may await backward.

        reuse_lists_of: a FwdState of an earlier full forward of the same
        frame geometry; its tile lists and depth order are reused (projection
        only, no binning or sort) and its workspace is shared, so that
        state's own backward must already have run.

        save_fragments: also save every blended fragment's alpha (the
        backward then reads it instead of re-evaluating Eq. 2); the workspace
        grows by 2 KB per pair of capacity.

        balance: assign each wave's lanes the samples of similar previous work
        (lane_work, uint16 [H, W], the lane_work_out of an earlier balanced
        forward of this geometry, or None) and write this forward's work to
        lane_work_out (or None).

        l1: (target_color, target_depth, n_active or None[, w_color, w_depth])
        to have the forward also write the loss gradients (FwdState.dL_dcolor,
        .dL_ddepth) that loss_l1_grad would compute from its image."""
        n = scene[0].shape[0]
        if save_fragments and (not save_state or reuse_lists_of is not None):
            raise ValueError("save_fragments needs save_state and a full forward")
        fflag = RTGS_FWD_SAVE_FRAGMENTS if save_fragments else 0
        dev = scene[0].device
        h, w = cam.height, cam.width
        l1s = None
        if l1 is not None:
            tc, td, cnt, *wts = l1
            gc, gd = torch.empty(3, h, w, device=dev), torch.empty(h, w, device=dev)
            l1s = l1_loss(tc, td, gc, gd, cnt, *wts)
        if reuse_lists_of is not None:
            ref = reuse_lists_of
            if (ref.n, ref.cam.width, ref.cam.height, ref.sample_log2) != (n, w, h, sample_log2):
                raise ValueError("reuse_lists_of: different frame geometry")
            out = FwdState(ws=ref.ws, cap=ref.cap, cam=cam, n=n, sample_log2=sample_log2,
                           color=torch.empty(3, h, w, device=dev),
                           depth=torch.empty(h, w, device=dev),
                           alpha=torch.empty(h, w, device=dev),
                           final_T=torch.empty(h, w, device=dev) if save_state else None,
                           last_idx=(torch.empty(h, w, dtype=torch.int32, device=dev)
                                     if save_state else None),
                           visible=torch.empty(n, dtype=torch.uint8, device=dev),
                           pairs=ref.pairs)
            if l1s is not None:
                out.dL_dcolor, out.dL_ddepth = gc, gd
                render_fwd_batched(self.handle, [dict(
                    scene=scene, viewmat=viewmat, cam=cam, gauss_mask=gauss_mask,
                    pixel_mask=pixel_mask, sample_log2=sample_log2, color=out.color,
                    depth=out.depth, alpha=out.alpha, final_T=out.final_T,
                    last_idx=out.last_idx, visible=out.visible, l1=l1s)], ref.ws, ref.cap,
                    flags=(RTGS_FWD_SAVE_STATE if save_state else 0) | RTGS_FWD_REUSE_LISTS,
                    stream=stream)
                return out
            render_fwd(self.handle, *scene, viewmat, cam, ref.ws, ref.cap, out.color, out.depth,
                       out.alpha, out.final_T, out.last_idx, out.visible, gauss_mask=gauss_mask,
                       pixel_mask=pixel_mask,
                       flags=(RTGS_FWD_SAVE_STATE if save_state else 0) | RTGS_FWD_REUSE_LISTS
                       | (int(sample_log2) << RTGS_SAMPLE_SHIFT), stream=stream)
            return out
        est = int(self.ppg * n) + 4 * _tiles(w, h)
        cap = max(self.cap, est, self.min_cap)
        while True:
            need = rtgs_workspace_size(n, w, h, cap, fflag)
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
            out = FwdState(ws=ws, cap=cap, cam=cam, n=n, sample_log2=sample_log2,
                           frags=save_fragments,
                           color=torch.empty(3, h, w, device=dev),
                           depth=torch.empty(h, w, device=dev),
                           alpha=torch.empty(h, w, device=dev),
                           final_T=torch.empty(h, w, device=dev) if save_state else None,
                           last_idx=(torch.empty(h, w, dtype=torch.int32, device=dev)
                                     if save_state else None),
                           visible=torch.empty(n, dtype=torch.uint8, device=dev))
            if l1s is not None:
                out.dL_dcolor, out.dL_ddepth = gc, gd
            if balance or l1s is not None:
                out.balanced = balance
                render_fwd_batched(self.handle, [dict(
                    scene=scene, viewmat=viewmat, cam=cam, gauss_mask=gauss_mask,
                    pixel_mask=pixel_mask, sample_log2=sample_log2, color=out.color,
                    depth=out.depth, alpha=out.alpha, final_T=out.final_T,
                    last_idx=out.last_idx, visible=out.visible, lane_work=lane_work,
                    lane_work_out=lane_work_out, l1=l1s)], ws, cap,
                    flags=(RTGS_FWD_SAVE_STATE if save_state else 0) | fflag
                    | (RTGS_FWD_BALANCE_LANES if balance else 0), stream=stream)
            else:
                render_fwd(self.handle, *scene, viewmat, cam, ws, cap, out.color, out.depth,
                           out.alpha, out.final_T, out.last_idx, out.visible,
                           gauss_mask=gauss_mask, pixel_mask=pixel_mask,
                           flags=(RTGS_FWD_SAVE_STATE if save_state else 0) | fflag
                           | (int(sample_log2) << RTGS_SAMPLE_SHIFT), stream=stream)
            self.cap = max(self.cap, cap)
            if self.check != "every":
                return out
            code, pairs, _ = rtgs_query(self.handle, True)
            out.pairs = pairs
            if code == RTGS_OK:
                return out
            self.grow(pairs)
            cap = self.cap

    def backward(self, scene, viewmat, cam: Cam, st: "FwdState", dL_dcolor, dL_ddepth,
                 dL_dalpha=None, pose=True, map_grads=True, cov3d=False, score=False,
                 gauss_mask=None,
                 pixel_mask=None, stream=None, adam=None):
        """Gradients of the last forward.  With adam (a MapAdam over the
        scene tensors) the map is updated in the same pass instead of
        returning its gradients (RTGS_GRAD_ADAM), and adam's step advances."""
        if adam is not None:
            return self._backward_adam(scene, viewmat, cam, st, dL_dcolor, dL_ddepth, dL_dalpha,
                                       pose, cov3d, gauss_mask, pixel_mask, stream, adam)
        n = st.n
        dev = scene[0].device
        flags = (RTGS_GRAD_POSE if pose else 0) | (RTGS_GRAD_MAP if map_grads else 0)
        flags |= RTGS_GRAD_COV3D if cov3d else 0
        # score: dL/dmu and dL/dSigma only (importance-score inputs), on the
        # pose-only raster path
        flags |= RTGS_GRAD_SCORE if score and not map_grads else 0
        if st.final_T is None:
            flags |= RTGS_GRAD_RECOMPUTE_STATE
        if st.frags:
            flags |= RTGS_GRAD_SAVED_FRAGMENTS
        if st.balanced:
            flags |= RTGS_GRAD_BALANCED_LANES
        flags |= int(st.sample_log2) << RTGS_SAMPLE_SHIFT
        g = {}
        if map_grads:
            g["means"] = torch.empty(n, 3, device=dev)
            g["log_scales"] = torch.empty(n, 3, device=dev)
            g["quats"] = torch.empty(n, 4, device=dev)
            g["opacity_logits"] = torch.empty(n, device=dev)
            g["colors"] = torch.empty(n, 3, device=dev)
        if cov3d:
            g["cov3d"] = torch.empty(n, 6, device=dev)
        if score and not map_grads:
            g["means"] = torch.empty(n, 3, device=dev)
            g["cov3d"] = torch.empty(n, 6, device=dev)
        if pose:
            g["pose"] = torch.empty(6, device=dev)
            g["viewmat"] = torch.empty(3, 4, device=dev)
        render_bwd(self.handle, *scene, viewmat, cam, st.ws, st.cap, st.final_T, st.last_idx,
                   dL_dcolor.contiguous(), dL_ddepth.contiguous(),
                   None if dL_dalpha is None else dL_dalpha.contiguous(), flags,
                   g.get("means"), g.get("log_scales"), g.get("quats"), g.get("opacity_logits"),
                   g.get("colors"), g.get("pose"), g.get("cov3d"), gauss_mask=gauss_mask,
                   pixel_mask=pixel_mask, stream=stream, g_viewmat=g.get("viewmat"))
        return g

    def _backward_adam(self, scene, viewmat, cam, st, dL_dcolor, dL_ddepth, dL_dalpha, pose,
                       cov3d, gauss_mask, pixel_mask, stream, adam):
        for p, q in zip(adam.params, scene):
            if p.data_ptr() != q.data_ptr():
                raise ValueError("adam must hold the scene tensors being rendered")
        n = st.n
        dev = scene[0].device
        flags = RTGS_GRAD_MAP | RTGS_GRAD_ADAM | (RTGS_GRAD_POSE if pose else 0)
        flags |= RTGS_GRAD_COV3D if cov3d else 0
        if st.final_T is None:
            flags |= RTGS_GRAD_RECOMPUTE_STATE
        if st.frags:
            flags |= RTGS_GRAD_SAVED_FRAGMENTS
        if st.balanced:
            flags |= RTGS_GRAD_BALANCED_LANES
        g = {}
        if cov3d:
            g["cov3d"] = torch.empty(n, 6, device=dev)
        if pose:
            g["pose"] = torch.empty(6, device=dev)
            g["viewmat"] = torch.empty(3, 4, device=dev)
        state = adam.fused()
        item = dict(scene=scene, viewmat=viewmat, cam=cam, gauss_mask=gauss_mask,
                    pixel_mask=pixel_mask, sample_log2=st.sample_log2, final_T=st.final_T,
                    last_idx=st.last_idx, dL_dcolor=dL_dcolor.contiguous(),
                    dL_ddepth=dL_ddepth.contiguous(),
                    dL_dalpha=None if dL_dalpha is None else dL_dalpha.contiguous(),
                    g_pose6=g.get("pose"), g_viewmat=g.get("viewmat"), g_cov3d=g.get("cov3d"),
                    adam=state)
        arr, _keep = make_sessions([item])
        render_bwd_batched_c(self.handle, arr, 1, st.ws, st.cap, flags, _stream(stream))
        adam.t += 1
        return g


@dataclasses.dataclass
class FwdState:
    ws: torch.Tensor
    cap: int
    cam: Cam
    n: int
    color: torch.Tensor
    depth: torch.Tensor
    alpha: torch.Tensor
    final_T: torch.Tensor | None
    last_idx: torch.Tensor | None
    visible: torch.Tensor
    sample_log2: int = 0
    pairs: int = -1
    frags: bool = False
    balanced: bool = False
    dL_dcolor: torch.Tensor | None = None   # loss gradients written by the forward (l1=)
    dL_ddepth: torch.Tensor | None = None

    def stage(self):
        """Forward intermediates for tests: dict of numpy arrays."""
        n, w, h = self.n, self.cam.width, self.cam.height
        dev = self.ws.device
        j = self.sample_log2
        tw, th = 16 << ((j + 1) // 2), 16 << (j // 2)
        t = ((w + tw - 1) // tw) * ((h + th - 1) // th)
        stage = torch.empty(max(n, 1), 12, device=dev)
        rect = torch.empty(max(n, 1), 4, dtype=torch.int32, device=dev)
        ranges = torch.empty(t, 2, dtype=torch.int32, device=dev)
        ids = torch.empty(max(self.cap, 1), dtype=torch.int32, device=dev)
        rtgs_debug_stage([n], [w], [h], self.cap, self.ws, stage, rect, ranges, ids,
                         sample_log2=[j])
        torch.cuda.synchronize()
        rng = ranges.cpu().numpy()
        total = int(rng[:, 1].max()) if t else 0
        return {"stage": stage.cpu().numpy()[:n], "rect": rect.cpu().numpy()[:n],
                "ranges": rng, "ids": ids.cpu().numpy()[:total]}
