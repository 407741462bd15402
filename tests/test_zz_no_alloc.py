"""The allocation-free compaction (compact_by_mask_static) against
compact_by_mask: bit-exact, on two calls in a row on the same GPU, the
second with a smaller input (the static scratch keeps the first call's
contents), both through the C ABI."""
import numpy as np
import pytest
import torch

from paper_2510_06644_amd import rtgs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _arrays(n, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    drop = (torch.rand(n, generator=g, device="cuda") < 0.3).to(torch.uint8)
    a = torch.randn(n, 3, generator=g, device="cuda")
    b = torch.randint(0, 255, (n, 5), generator=g, device="cuda", dtype=torch.int32).to(torch.uint8)
    c = torch.randn(n, 14, generator=g, device="cuda")
    return drop, (a, b, c)


def _run(fn, drop, srcs):
    k = int((drop == 0).sum().item())
    dsts = [torch.full((k,) + tuple(s.shape[1:]), 7, dtype=s.dtype, device="cuda") for s in srcs]
    n_kept = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    fn(drop, list(zip(srcs, dsts)), n_kept)
    torch.cuda.synchronize()
    return dsts, int(n_kept.item())


@pytest.mark.parametrize("sizes", [(3_000_000, 70_001), (1025, 1)])
def test_static_compaction_equals_the_scratch_form_twice(sizes):
    for call, n in enumerate(sizes):
        say(f"test_static_compaction call {call} n={n}")
        drop, srcs = _arrays(n, 100 + call + n % 97)
        want, k_want = _run(rtgs.compact_by_mask, drop, srcs)
        got, k_got = _run(rtgs.compact_by_mask_static, drop, srcs)
        assert k_got == k_want == int((drop == 0).sum().item())
        for x, y in zip(got, want):
            assert torch.equal(x, y)
        keep = drop.cpu().numpy() == 0
        assert np.array_equal(got[0].cpu().numpy(), srcs[0].cpu().numpy()[keep])


def test_static_compaction_at_its_row_limit_and_empty():
    n = rtgs.RTGS_COMPACT_STATIC_MAX_ROWS
    say(f"test_static_compaction_at_its_row_limit n={n}")
    drop, (a, _, _) = _arrays(n, 5)
    want, k_want = _run(rtgs.compact_by_mask, drop, (a,))
    got, k_got = _run(rtgs.compact_by_mask_static, drop, (a,))
    assert k_got == k_want and torch.equal(got[0], want[0])
    drop = torch.zeros(0, dtype=torch.uint8, device="cuda")
    n_kept = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    rtgs.compact_by_mask_static(drop, [], n_kept)
    torch.cuda.synchronize()
    assert int(n_kept.item()) == 0
    big = torch.zeros(n + 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(rtgs.RtgsError) as e:
        rtgs.compact_by_mask_static(big, [], n_kept)
    assert e.value.code == rtgs.RTGS_ERR_WORKSPACE
