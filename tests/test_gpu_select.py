"""prune_by_grad (Sec. 4.1, Eq. 7) and downsample_mask (Sec. 4.2) on the GPU
against the oracle's selections.  The integer decisions are taken on the same
float32 values on both sides: the kernel's float32 score (itself compared
with the float64 score), and the given final transmittance."""
import numpy as np
import pytest
import torch

from oracle import selection
from paper_2510_06644_amd import rtgs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    return rtgs.Handle(0)


@pytest.mark.parametrize("n,ratio,with_vis,with_mask", [
    (50_000, 0.5, True, True), (50_000, 0.3, False, False), (1, 0.5, True, False),
    (7, 0.5, True, True), (100_000, 0.0, True, False), (0, 0.5, False, False)])
def test_prune_matches_oracle_selection(handle, n, ratio, with_vis, with_mask):
    say(f"test_prune n={n} ratio={ratio}")
    rng = np.random.default_rng(n + int(ratio * 10))
    gm = rng.normal(size=(n, 3)).astype(np.float32)
    gc = rng.normal(size=(n, 6)).astype(np.float32)
    zero = rng.random(n) < 0.1                 # exact zeros: many tied scores
    gm[zero] = 0
    gc[zero] = 0
    dup = rng.random(n) < 0.05                 # exact duplicates of row 0
    if n > 0:
        gm[dup] = gm[0]
        gc[dup] = gc[0]
    vis = (rng.random(n) < 0.8).astype(np.uint8) if with_vis else None
    mask = (rng.random(n) < 0.1).astype(np.uint8) if with_mask else None
    d = lambda a: None if a is None else torch.from_numpy(a).cuda()
    out = torch.full((max(n, 1),), 7, dtype=torch.uint8, device="cuda")[:n]
    score = torch.empty(max(n, 1), device="cuda")[:n]
    nm = torch.zeros(1, dtype=torch.int32, device="cuda")
    rtgs.prune_by_grad(handle, d(gm), d(gc), d(vis), d(mask), 0.8, ratio, out, nm, score)
    torch.cuda.synchronize()
    s32 = score.cpu().numpy()
    s64 = selection.importance_score(gm, gc, 0.8)
    if n:
        assert np.allclose(s32, s64, rtol=1e-6, atol=0)
    v = np.ones(n, np.uint8) if vis is None else vis
    m = np.zeros(n, np.uint8) if mask is None else mask
    want, k = selection.prune_select(s32, v, m, ratio)
    assert nm.item() == k
    assert np.array_equal(out.cpu().numpy(), want)


def test_prune_rejects_ratio_above_half(handle):
    x = torch.zeros(4, 3, device="cuda")
    with pytest.raises(rtgs.RtgsError):
        rtgs.prune_by_grad(handle, x, torch.zeros(4, 6, device="cuda"), None, None, 0.8, 0.6,
                           torch.zeros(4, dtype=torch.uint8, device="cuda"))


@pytest.mark.parametrize("w,h", [(37, 23), (1200, 680), (16, 16), (1, 5)])
def test_downsample_mask_matches_oracle(w, h):
    say(f"test_downsample {w}x{h}")
    rng = np.random.default_rng(w * h)
    t = (np.round(rng.random((h, w)) * 20) / 20).astype(np.float32)   # many ties
    tt = torch.from_numpy(t).cuda()
    for j in range(0, 5):
        out = torch.empty(h, w, dtype=torch.uint8, device="cuda")
        na = torch.zeros(1, dtype=torch.int32, device="cuda")
        rtgs.downsample_mask(tt, j, out, na)
        torch.cuda.synchronize()
        want = selection.downsample_select(t, j) if w * h < 5000 else None
        got = out.cpu().numpy()
        if want is not None:
            assert np.array_equal(got, want), j
        bw, bh = selection.block_shape(j)
        assert na.item() == got.sum() == ((w + bw - 1) // bw) * ((h + bh - 1) // bh)
        # every block keeps exactly its lowest-T pixel (checked on all sizes)
        for by in range(0, h, bh * max(1, h // (8 * bh))):
            for bx in range(0, w, bw * max(1, w // (8 * bw))):
                blk = t[by:by + bh, bx:bx + bw]
                sel = got[by:by + bh, bx:bx + bw]
                assert sel.sum() == 1
                iy, ix = np.argwhere(sel)[0]
                flat = blk.reshape(-1)
                assert blk[iy, ix] == flat.min() and iy * blk.shape[1] + ix == int(np.argmin(flat))
