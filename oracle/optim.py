"""Map update of the mapping stage (oracle; test infrastructure).

Sec. 3.1: in mapping, the Gaussian gradients of Step 5 update the 3D
Gaussian parameters.  The paper names no optimiser; the reading used is Adam
without weight decay (the rule of 3DGS-style mapping), written out from its
definition in float64:

    m_t = beta1 m_{t-1} + (1 - beta1) g
    v_t = beta2 v_{t-1} + (1 - beta2) g^2
    p_t = p_{t-1} - lr (m_t / (1 - beta1^t)) / (sqrt(v_t / (1 - beta2^t)) + eps)

Pins: tests/test_oracle_pins.py (first step of a constant gradient is
p - lr g / (|g| + eps) exactly; several steps agree with torch.optim.Adam
in float64; the first pose step of a pure translation or pure rotation
gradient against scipy's rotation-vector map).
"""
import numpy as np


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One update at step count t (>= 1, this update included); returns new
    (p, m, v) as float64 arrays."""
    p, g, m, v = (np.asarray(x, dtype=np.float64) for x in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def pose_update(viewmat, g, m, v, t, lr_rho, lr_phi, beta1=0.9, beta2=0.999, eps=1e-8):
    """Tracking step on the left-perturbation tangent xi = (rho, phi) at 0:
    Adam with the learning rate lr_rho for rho and lr_phi for phi, then the
    re-linearisation viewmat <- Exp(-s) viewmat (Sec. 3.1: tracking updates
    the camera pose; the pose gradient is dL/dP of Step 5).  Returns the new
    (viewmat [3, 4], m, v) in float64."""
    import torch
    from .camera import apply_left
    lr = np.array([lr_rho] * 3 + [lr_phi] * 3, dtype=np.float64)
    zero = np.zeros(6)
    _, m1, v1 = adam_step(zero, g, m, v, t, 1.0, beta1, beta2, eps)
    mhat = m1 / (1.0 - beta1 ** t)
    vhat = v1 / (1.0 - beta2 ** t)
    s = lr * mhat / (np.sqrt(vhat) + eps)
    vm = apply_left(torch.tensor(-s, dtype=torch.float64),
                    torch.as_tensor(np.asarray(viewmat, dtype=np.float64)))
    return vm.numpy(), m1, v1
