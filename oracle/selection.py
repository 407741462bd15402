"""Adaptive Gaussian pruning (Sec. 4.1, Eq. 7) and dynamic downsampling
(Sec. 4.2) as closed-form selections (oracle; test infrastructure).

Importance (Eq. 7): Score = ||dL/dmu||_2 + lambda ||dL/dSigma||, lambda = 0.8
(Sec. 6.1 hyper-parameters).  Readings: the Sigma norm is the
Frobenius norm of the symmetric world-frame gradient over all nine entries;
the mask is applied to the floor(rho V) lowest (score, index) among the V
visible, not yet masked Gaussians, with rho at most 0.5 (Sec. 6.2 caps the
pruning ratio at 50%).

Downsampling (Sec. 4.2): keyframes keep R0; a non-keyframe n after keyframe
k keeps min(R0/16 m^(n-k-1), R0/4) pixels.  As a pixel ratio 2^-j:
j = 0 for keyframes, otherwise j = max(2, 4 - floor((n-k-1) log2 m)), i.e.
4, 3, 2, 2, ... for m = 2.  The image is cut into blocks of 2^ceil(j/2) by
2^floor(j/2) pixels (4x4, 4x2, 2x2); each block keeps the one pixel whose
previous-forward final transmittance is lowest (the most covered pixel; the
paper's alpha-based choice), ties to the lowest raster index.

Pins: tests/test_oracle_pins.py (hand-built cases; the schedule 0, 4, 3, 2, 2).
"""
import math

import numpy as np


def sym6_frobenius(g6):
    """Frobenius norm of symmetric matrices stored as (xx, xy, xz, yy, yz, zz)."""
    g = np.asarray(g6, dtype=np.float64)
    xx, xy, xz, yy, yz, zz = g.T
    return np.sqrt(xx * xx + yy * yy + zz * zz + 2 * (xy * xy + xz * xz + yz * yz))


def importance_score(g_means, g_cov6, lam=0.8):
    gm = np.asarray(g_means, dtype=np.float64)
    return np.sqrt((gm * gm).sum(1)) + lam * sym6_frobenius(g_cov6)


def prune_select(score, visible, mask_in, ratio):
    """(mask_out u8 [N], number newly masked) from given float scores."""
    score = np.asarray(score)
    cand = np.asarray(visible, bool) & ~np.asarray(mask_in, bool)
    idx = np.nonzero(cand)[0]
    k = int(math.floor(ratio * len(idx)))
    order = np.lexsort((idx, score[idx]))          # (score, index) ascending
    chosen = idx[order[:k]]
    out = np.asarray(mask_in, bool).copy()
    out[chosen] = True
    return out.astype(np.uint8), k


def downsample_log2_ratio(is_keyframe, n, k, m=2):
    if is_keyframe:
        return 0
    if n <= k or m < 2:
        raise ValueError("non-keyframe must follow its keyframe; m >= 2")
    return max(2, 4 - int(math.floor((n - k - 1) * math.log2(m) + 1e-12)))


def block_shape(j):
    return 2 ** ((j + 1) // 2), 2 ** (j // 2)     # (width, height)


def downsample_select(final_t, j):
    """Pixel mask u8 [H,W]: per block, the lowest final T (ties: lowest index)."""
    t = np.asarray(final_t)
    h, w = t.shape
    bw, bh = block_shape(j)
    mask = np.zeros((h, w), np.uint8)
    for by in range(0, h, bh):
        for bx in range(0, w, bw):
            blk = t[by:by + bh, bx:bx + bw]
            best = None
            for yy in range(blk.shape[0]):
                for xx in range(blk.shape[1]):
                    val = blk[yy, xx]
                    if best is None or val < best[0]:
                        best = (val, yy, xx)
            mask[by + best[1], bx + best[2]] = 1
    return mask
