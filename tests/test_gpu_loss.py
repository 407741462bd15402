"""Loss gradient on the GPU (loss_l1_grad) against the float64 oracle of
Eq. 6 as read here: every pixel, and a downsampling mask whose count comes
from the device.  The gradient is sign times a scale, so the comparison is
to one rounding of the scale."""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_06644_amd import rtgs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _frames(h, w, seed):
    g = torch.Generator().manual_seed(seed)
    c = torch.rand(3, h, w, generator=g)
    d = torch.rand(h, w, generator=g) * 4
    tc = c + 0.05 * torch.randn(3, h, w, generator=g)
    td = d + 0.05 * torch.randn(h, w, generator=g)
    tc[0, :3, :3] = c[0, :3, :3]            # exact ties: sign(0) = 0
    td[:2, :5] = d[:2, :5]
    return c, d, tc, td


@pytest.mark.parametrize("masked", [False, True])
def test_l1_gradient_matches_oracle(masked):
    say(f"test_l1_gradient_matches_oracle masked={masked}")
    h, w = 97, 131                            # ragged against 256-thread blocks
    c, d, tc, td = _frames(h, w, 3)
    mask = cnt = None
    if masked:
        ft = torch.rand(h, w, generator=torch.Generator().manual_seed(4)).cuda()
        mask = torch.empty(h, w, dtype=torch.uint8, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        rtgs.downsample_mask(ft, 2, mask, cnt)
    gc = torch.full((3, h, w), float("nan"), device="cuda")
    gd = torch.full((h, w), float("nan"), device="cuda")
    rtgs.loss_l1_grad(c.cuda(), d.cuda(), tc.cuda(), td.cuda(), gc, gd, pixel_mask=mask,
                      n_active=cnt)
    torch.cuda.synchronize()
    m = None if mask is None else mask.cpu().numpy()
    if masked:
        assert int(cnt.item()) == int(m.astype(bool).sum()) > 0
    _, rc, rd = oracle.l1_loss_grads(c.numpy(), d.numpy(), tc.numpy(), td.numpy(), m)
    np.testing.assert_allclose(gc.cpu().numpy(), rc.numpy(), rtol=2e-7, atol=0)
    np.testing.assert_allclose(gd.cpu().numpy(), rd.numpy(), rtol=2e-7, atol=0)
    assert (gc.cpu()[0, :3, :3] == 0).all()


def test_l1_gradient_rejects_mask_without_count():
    say("test_l1_gradient_rejects_mask_without_count")
    c, d, tc, td = (x.cuda() for x in _frames(8, 8, 5))
    with pytest.raises(rtgs.RtgsError) as e:
        rtgs.loss_l1_grad(c, d, tc, td, torch.empty_like(c), torch.empty_like(d),
                          pixel_mask=torch.ones(8, 8, dtype=torch.uint8, device="cuda"))
    assert e.value.code == rtgs.RTGS_ERR_INVALID_ARG


def test_batched_loss_equals_single_frame_calls():
    """loss_l1_grad_batched over frames of different sizes, with and without
    masks, gives bit for bit the single-frame results (34 frames: two
    launches)."""
    say("test_batched_loss_equals_single_frame_calls")
    items, singles = [], []
    for k in range(34):
        h, w = 17 + 7 * (k % 5), 23 + 11 * (k % 3)
        c, d, tc, td = (t.cuda() for t in _frames(h, w, 100 + k))
        mask = cnt = None
        if k % 2:
            ft = torch.rand(h, w, generator=torch.Generator().manual_seed(k)).cuda()
            mask = torch.empty(h, w, dtype=torch.uint8, device="cuda")
            cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
            rtgs.downsample_mask(ft, 2, mask, cnt)
        gc = torch.full((3, h, w), float("nan"), device="cuda")
        gd = torch.full((h, w), float("nan"), device="cuda")
        items.append((c, d, tc, td, gc, gd, mask, cnt))
        sc, sd = torch.empty_like(gc), torch.empty_like(gd)
        rtgs.loss_l1_grad(c, d, tc, td, sc, sd, pixel_mask=mask, n_active=cnt)
        singles.append((sc, sd))
    rtgs.loss_l1_grad_batched(items)
    torch.cuda.synchronize()
    for (c, d, tc, td, gc, gd, mask, cnt), (sc, sd) in zip(items, singles):
        assert torch.equal(gc, sc) and torch.equal(gd, sd)
