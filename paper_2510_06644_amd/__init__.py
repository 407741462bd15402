"""MI355X-native differentiable tile-based Gaussian-splatting rasterizer.

The compute path lives in ``librtgs.so`` (HIP kernels for gfx950 behind a C
ABI, ``include/rtgs.h``).  ``rtgs`` is the thin ctypes binding with the same
entry-point names, ``autograd`` wraps it as a ``torch.autograd.Function``, and
``serving`` runs many SLAM sessions with continuous batching.  ``synth`` draws
seeded synthetic scenes.

Importing this package does not load the native library; the binding loads it
on first use and raises if it is missing.
"""
__all__ = ["synth", "rtgs", "autograd", "serving", "optim", "pose", "prune"]
