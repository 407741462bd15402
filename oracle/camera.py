"""Camera pose algebra (oracle; test infrastructure).

The pose is a world->camera rigid transform [R_c | t_c] (3x4, row-major).  The
paper optimises the pose from dL/dP (Sec. 2.2, Preprocessing BP); it does not
fix a parameterisation.  Reading used here: a left perturbation
T = Exp(xi) T0 with the tangent xi = (rho, phi), translation first.

Pins: tests/test_oracle_pins.py (Exp of a pure rotation is Rodrigues' formula
checked against scipy's rotation-vector map; Exp(0) = I; Exp(xi) Exp(-xi) = I).
"""
import torch


def hat(w: torch.Tensor) -> torch.Tensor:
    """Skew-symmetric matrix [w]_x with [w]_x v = w x v."""
    z = torch.zeros_like(w[..., 0])
    wx, wy, wz = w.unbind(-1)
    return torch.stack([z, -wz, wy, wz, z, -wx, -wy, wx, z], -1).reshape(
        w.shape[:-1] + (3, 3))


def se3_exp(xi: torch.Tensor) -> torch.Tensor:
    """Exp: se(3) -> SE(3) as a 3x4 matrix [R | V rho].

    R = I + A W + B W^2 and V = I + B W + C W^2 with W = [phi]_x,
    A = sin t / t, B = (1 - cos t) / t^2, C = (t - sin t) / t^3.
    Taylor series are used for small angles so the map is smooth at zero.
    """
    xi = xi.to(torch.float64)
    rho, phi = xi[:3], xi[3:]
    th2 = (phi * phi).sum()
    small = th2 < 1e-8
    th2s = torch.where(small, torch.ones_like(th2), th2)
    th = torch.sqrt(th2s)
    a = torch.where(small, 1 - th2 / 6 + th2 * th2 / 120, torch.sin(th) / th)
    b = torch.where(small, 0.5 - th2 / 24 + th2 * th2 / 720,
                    (1 - torch.cos(th)) / th2s)
    c = torch.where(small, 1.0 / 6 - th2 / 120 + th2 * th2 / 5040,
                    (th - torch.sin(th)) / (th2s * th))
    w = hat(phi)
    eye = torch.eye(3, dtype=torch.float64)
    r = eye + a * w + b * (w @ w)
    v = eye + b * w + c * (w @ w)
    return torch.cat([r, (v @ rho)[:, None]], 1)


def compose(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """(a o b) for 3x4 rigid transforms."""
    return torch.cat([a[:, :3] @ b[:, :3], (a[:, :3] @ b[:, 3:] + a[:, 3:])], 1)


def apply_left(xi: torch.Tensor, viewmat: torch.Tensor) -> torch.Tensor:
    """Exp(xi) * viewmat."""
    return compose(se3_exp(xi), viewmat.to(torch.float64))


def apply_left_linear(xi: torch.Tensor, viewmat: torch.Tensor) -> torch.Tensor:
    """(I + xi^) * viewmat: equal to Exp(xi) * viewmat to first order, so its
    derivative at xi = 0 is the pose gradient; used for autograd at xi = 0."""
    vm = viewmat.to(torch.float64)
    rho, phi = xi[:3], xi[3:]
    w = hat(phi)
    eye = torch.eye(3, dtype=torch.float64)
    return torch.cat([(eye + w) @ vm[:, :3], ((eye + w) @ vm[:, 3:] + rho[:, None])], 1)
