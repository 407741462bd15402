"""Shared test utilities: scene builders and the comparison metric."""
import numpy as np

from paper_2510_06644_amd import synth


def cam_tuple(cam):
    return (cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)


def one_gaussian_scene(mean, log_scale, opacity, color, quat=(1, 0, 0, 0)):
    """Scene arrays for explicitly placed Gaussians (lists of per-Gaussian values)."""
    mean = np.atleast_2d(np.asarray(mean, np.float64))
    n = mean.shape[0]
    ls = np.broadcast_to(np.asarray(log_scale, np.float64), (n, 3)) if np.ndim(log_scale) < 2 \
        else np.asarray(log_scale, np.float64)
    q = np.broadcast_to(np.asarray(quat, np.float64), (n, 4))
    o = np.broadcast_to(np.asarray(opacity, np.float64), (n,))
    eta = np.log(o) - np.log1p(-o)
    col = np.broadcast_to(np.asarray(color, np.float64), (n, 3))
    return synth.Scene(*(np.ascontiguousarray(a, np.float32) for a in (mean, ls, q, eta, col)))


def rel_err(x, r, floor_frac=1e-2):
    """max_i |x_i - r_i| / max(|r_i|, floor_frac * max|r|)."""
    x = np.asarray(x, np.float64).ravel()
    r = np.asarray(r, np.float64).ravel()
    if r.size == 0:
        return 0.0
    scale = max(np.abs(r).max(), 1e-30)
    den = np.maximum(np.abs(r), floor_frac * scale)
    return float((np.abs(x - r) / den).max())


def norm_err(x, r):
    x = np.asarray(x, np.float64).ravel()
    r = np.asarray(r, np.float64).ravel()
    return float(np.linalg.norm(x - r) / max(np.linalg.norm(r), 1e-30))
