"""CPU reference ("oracle") for the differentiable Gaussian-splatting rasterizer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the test-suite, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code with the HIP library.

Everything is plain PyTorch on the CPU in float64:

* ``gaussians``  - parameter activation and 3D covariance (Eq. 1).
* ``camera``     - SE(3) exponential and left perturbation of the pose.
* ``projection`` - Step 1-1: EWA projection to 2D mean / covariance / conic.
* ``composite``  - Steps 3-1 and 3-2: alpha (Eq. 2) and front-to-back
                   blending (Eq. 3) with early termination, brute force over
                   every Gaussian for every pixel, no tiles.
* ``render``     - the whole forward, and its exact derivative (Steps 4 and 5)
                   by automatic differentiation of that forward.
* ``binning``    - Step 1-2 and Step 2: tile lists and depth order, replayed
                   in float32 from the stage values of the kernel under test.
* ``selection``  - the importance score and mask selection (Eq. 7, Sec. 4.1)
                   and the downsampling schedule and pixel choice (Sec. 4.2).
* ``loss``       - the L1 colour + depth loss (Eq. 6, reading in DESIGN).
* ``optim``      - the map update (Adam, a reading: the paper names no
                   optimiser).

Parity status: every function here is pinned by tests under ``tests/`` against
closed forms, invariants, finite differences or brute force (see each module).
"""
from .gaussians import activate, quat_to_rotmat, covariance3d  # noqa: F401
from .camera import se3_exp, hat, apply_left  # noqa: F401
from .projection import project, Projected  # noqa: F401
from .composite import composite_pixels, Composite  # noqa: F401
from .render import render, render_with_grads, RenderOut, Grads  # noqa: F401
from .binning import tile_lists  # noqa: F401
from .selection import importance_score, prune_select, downsample_log2_ratio, downsample_select  # noqa: F401
from .loss import l1_loss_grads  # noqa: F401
from .optim import adam_step, pose_update  # noqa: F401
