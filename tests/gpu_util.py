"""Helpers shared by the GPU tests: device copies of seeded inputs, views built
with scipy (independent of both implementations), and the comparison rule."""
import sys

import numpy as np
import torch
from scipy.spatial.transform import Rotation

from paper_2510_06644_amd import rtgs, synth

IMG_TOL = 1e-4       # per-element, relative to max(|r|, 1e-2 max|r|)
GRAD_TOL = 1e-4      # per-Gaussian gradient vector, relative to max(|r_i|, 1e-2 max_j |r_j|)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_scene(scene):
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in scene.arrays())


def view_from(xi):
    """3x4 world->camera matrix Exp(xi) for xi = (rho, phi), float32, built
    with scipy's rotation-vector map; the translation is V(phi) rho."""
    xi = np.asarray(xi, np.float64)
    rho, phi = xi[:3], xi[3:]
    r = Rotation.from_rotvec(phi).as_matrix()
    th = np.linalg.norm(phi)
    k = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    if th < 1e-8:
        v = np.eye(3) + 0.5 * k
    else:
        v = np.eye(3) + (1 - np.cos(th)) / th ** 2 * k + (th - np.sin(th)) / th ** 3 * (k @ k)
    return np.concatenate([r, (v @ rho)[:, None]], 1).astype(np.float32)


def eye_view():
    return synth.identity_viewmat()


def rcam(cam):
    return rtgs.Cam(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)


def cam_tuple(cam):
    return (cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)


def rel_err(x, r, mask=None, floor_frac=1e-2):
    x = np.asarray(x, np.float64)
    r = np.asarray(r, np.float64)
    if mask is not None:
        x, r = x[..., mask], r[..., mask]
    x, r = x.ravel(), r.ravel()
    if r.size == 0:
        return 0.0
    scale = max(np.abs(r).max(), 1e-30)
    den = np.maximum(np.abs(r), floor_frac * scale)
    return float((np.abs(x - r) / den).max())


def grad_err(x, r, floor_frac=1e-2):
    """Relative error of per-Gaussian gradient vectors: row i of [N, k] is one
    Gaussian's gradient with respect to one parameter group; its error is
    |x_i - r_i| / max(|r_i|, floor_frac max_j |r_j|) in the Euclidean norm,
    and the result is the largest over the rows.  [N] arrays (one scalar per
    Gaussian) reduce to `rel_err`."""
    x = np.asarray(x, np.float64)
    r = np.asarray(r, np.float64)
    if r.ndim == 1:
        return rel_err(x, r, floor_frac=floor_frac)
    x, r = x.reshape(len(r), -1), r.reshape(len(r), -1)
    if r.size == 0:
        return 0.0
    rn = np.linalg.norm(r, axis=1)
    den = np.maximum(rn, floor_frac * max(rn.max(), 1e-30))
    return float((np.linalg.norm(x - r, axis=1) / den).max())


def norm_err(x, r):
    x = np.asarray(x, np.float64).ravel()
    r = np.asarray(r, np.float64).ravel()
    return float(np.linalg.norm(x - r) / max(np.linalg.norm(r), 1e-30))
