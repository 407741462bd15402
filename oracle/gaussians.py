"""Gaussian parameters -> activated attributes (oracle; test infrastructure).

Eq. (1) writes each Gaussian as (mu, Sigma, o, sh).  The paper does not fix a
parameterisation; the reading used here (listed in the design doc) is

* scales      s = exp(l)                      (per axis, l = log-scale)
* opacity     o = 1 / (1 + exp(-eta))        (eta = opacity logit)
* rotation    R(q / |q|), q = (w, x, y, z), Hamilton convention
* covariance  Sigma = R diag(s^2) R^T
* colour      RGB used as is (spherical harmonics of degree 0)

Pins: tests/test_oracle_pins.py (identity quaternion gives diag(s^2) exactly;
a rotation keeps the eigenvalues s^2; a quarter turn about z maps x to y).
"""
import torch


def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of the normalised quaternion q = (w, x, y, z); [..., 3, 3]."""
    q = q / torch.linalg.vector_norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    r = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
    ], -1)
    return r.reshape(q.shape[:-1] + (3, 3))


def covariance3d(log_scales: torch.Tensor, quats: torch.Tensor) -> torch.Tensor:
    """Sigma = R diag(exp(l)^2) R^T  (Eq. 1)."""
    s = torch.exp(log_scales)
    r = quat_to_rotmat(quats)
    return r @ torch.diag_embed(s * s) @ r.transpose(-1, -2)


def activate(log_scales, quats, opacity_logits):
    """(Sigma [N,3,3], opacity o [N])."""
    return covariance3d(log_scales, quats), torch.sigmoid(opacity_logits)
