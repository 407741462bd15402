"""SE(3) helpers for pose optimisation on the device (torch ops).

The rasterizer's pose gradient is taken with respect to a left perturbation
T = Exp(xi) T0, xi = (rho, phi) (translation first), at xi = 0.  Tracking
loops optimise xi and fold it back into the pose after each step
(re-linearisation), so xi stays near zero.
"""
import torch


def skew(w):
    z = torch.zeros_like(w[..., 0])
    return torch.stack([z, -w[..., 2], w[..., 1], w[..., 2], z, -w[..., 0],
                        -w[..., 1], w[..., 0], z], -1).reshape(w.shape[:-1] + (3, 3))


def exp_se3(xi):
    """Batched Exp: [..., 6] -> [..., 3, 4], Rodrigues with series near 0."""
    rho, phi = xi[..., :3], xi[..., 3:]
    th2 = (phi * phi).sum(-1, keepdim=True)[..., None]
    small = th2 < 1e-8
    th2s = torch.where(small, torch.ones_like(th2), th2)
    th = torch.sqrt(th2s)
    a = torch.where(small, 1 - th2 / 6, torch.sin(th) / th)
    b = torch.where(small, 0.5 - th2 / 24, (1 - torch.cos(th)) / th2s)
    c = torch.where(small, 1.0 / 6 - th2 / 120, (th - torch.sin(th)) / (th2s * th))
    k = skew(phi)
    k2 = k @ k
    eye = torch.eye(3, dtype=xi.dtype, device=xi.device).expand(k.shape)
    r = eye + a * k + b * k2
    v = eye + b * k + c * k2
    return torch.cat([r, v @ rho[..., None]], -1)


def compose(a, b):
    """a o b for [..., 3, 4] rigid transforms."""
    return torch.cat([a[..., :3] @ b[..., :3], a[..., :3] @ b[..., 3:] + a[..., 3:]], -1)


def apply_left(xi, viewmat):
    """Exp(xi) viewmat for xi [..., 6] and viewmat [..., 3, 4] (the
    re-linearisation step), computed in float64."""
    t = exp_se3(xi.to(torch.float64))
    return compose(t, viewmat.to(torch.float64)).to(viewmat.dtype)
