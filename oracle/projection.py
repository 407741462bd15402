"""Step 1-1, projection of 3D Gaussians to the image plane (oracle; test
infrastructure).

The paper names the outputs of this step (2D position, 2D covariance, colour,
opacity, depth; Sec. 2.1, Rendering Pipeline) but not its formulas.  Reading
used here (listed in the design doc): first-order EWA splatting as in 3D Gaussian
Splatting, which the paper builds on:

* p = R_c mu + t_c, depth z = p_z; culled if z <= 0.2 (near plane)
* u = fx x / z + cx,  v = fy y / z + cy
* J = [[fx/z, 0, -fx x~/z], [0, fy/z, -fy y~/z]] with x~ = clamp(x/z, +-1.3
  W/(2 fx)), y~ likewise (the clamp keeps far off-screen Gaussians bounded)
* Sigma' = J R_c Sigma R_c^T J^T + 0.3 I  (0.3 px^2 low-pass dilation)
* conic M = Sigma'^-1 = [[a, b], [b, c]]
* culled if det Sigma' <= 0, or 255 o < 1 (such a Gaussian cannot reach the
  1/255 alpha floor anywhere), or masked.

Pins: tests/test_oracle_pins.py (closed form of an isotropic Gaussian on the
optical axis and off axis, the clamp, the near-plane cull).
"""
import dataclasses

import torch

NEAR_Z = 0.2
DILATION = 0.3
FOV_CLAMP = 1.3
ALPHA_MIN = 1.0 / 255.0


@dataclasses.dataclass
class Projected:
    p: torch.Tensor        # [N,3] camera-space centre
    u: torch.Tensor        # [N]   pixel x of the centre
    v: torch.Tensor        # [N]
    z: torch.Tensor        # [N]   view-space depth
    cov2d: torch.Tensor    # [N,2,2]
    a: torch.Tensor        # [N] conic entries
    b: torch.Tensor
    c: torch.Tensor
    valid: torch.Tensor    # [N] bool, not culled


def project(means, cov3d, opacity, viewmat, cam, gauss_mask=None) -> Projected:
    """EWA projection of every Gaussian; cam = (W, H, fx, fy, cx, cy)."""
    w_img, h_img, fx, fy, cx, cy = cam
    rc = viewmat[:, :3]
    tc = viewmat[:, 3]
    p = means @ rc.T + tc
    x, y, z = p.unbind(-1)
    front = z > NEAR_Z
    zs = torch.where(front, z, torch.ones_like(z))       # keep culled rows finite
    lim_x = FOV_CLAMP * (w_img / 2.0) / fx
    lim_y = FOV_CLAMP * (h_img / 2.0) / fy
    xt = torch.clamp(x / zs, -lim_x, lim_x)
    yt = torch.clamp(y / zs, -lim_y, lim_y)
    zero = torch.zeros_like(zs)
    jac = torch.stack([fx / zs, zero, -fx * xt / zs,
                       zero, fy / zs, -fy * yt / zs], -1).reshape(-1, 2, 3)
    cov_cam = rc @ cov3d @ rc.T
    cov2d = jac @ cov_cam @ jac.transpose(1, 2)
    cov2d = cov2d + DILATION * torch.eye(2, dtype=cov2d.dtype)
    u = fx * x / zs + cx
    v = fy * y / zs + cy
    # the off-diagonal enters symmetrically, so dL/dSigma comes out symmetric
    sxx, syy = cov2d[:, 0, 0], cov2d[:, 1, 1]
    sxy = 0.5 * (cov2d[:, 0, 1] + cov2d[:, 1, 0])
    det = sxx * syy - sxy * sxy
    pos = det > 0
    dets = torch.where(pos, det, torch.ones_like(det))
    a = syy / dets
    b = -sxy / dets
    c = sxx / dets
    valid = front & pos & (255.0 * opacity >= 1.0)
    if gauss_mask is not None:
        valid = valid & ~gauss_mask.bool()
    return Projected(p, u, v, z, cov2d, a, b, c, valid)
