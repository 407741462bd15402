"""The mask-prune interval logic of Sec. 4.1 (host only)."""
import pytest

from paper_2510_06644_amd.prune import MaskPruneSchedule


def _kinds(s, ratios, n_iters):
    """Iteration kinds ('F' full, 'M' masked) with the change ratios handed
    to successive full iterations (the first gets None)."""
    out = []
    it = iter(ratios)
    for _ in range(n_iters):
        if s.next_is_full():
            s.start_window(None if not s.windows else next(it))
            out.append("F")
        else:
            s.step_masked()
            out.append("M")
    return "".join(out)


def test_first_window_is_k0_then_k_follows_the_5_percent_rule():
    s = MaskPruneSchedule(k0=5)
    # change above 5% -> K0 // 2 = 2; at or below -> 2 K0 = 10
    kinds = _kinds(s, [0.2, 0.05, 0.051], 1 + 5 + 1 + 2 + 1 + 10 + 1 + 2)
    assert kinds == "FMMMMM" + "FMM" + "FMMMMMMMMMM" + "FMM"
    assert [k for k, _ in s.windows] == [5, 2, 10, 2]
    assert [r for _, r in s.windows] == [None, 0.2, 0.05, 0.051]


def test_k_is_relative_to_k0_not_compounding():
    s = MaskPruneSchedule(k0=4)
    _kinds(s, [0.0, 0.0, 0.9, 0.9] + [0.0] * 20, 60)
    assert [k for k, _ in s.windows][:5] == [4, 8, 8, 2, 2]


def test_small_k0_and_misuse():
    s = MaskPruneSchedule(k0=1)
    assert _kinds(s, [0.5, 0.5], 5) == "FMFMF"   # K0 // 2 = 0 is taken as 1
    s = MaskPruneSchedule()
    with pytest.raises(RuntimeError):
        s.step_masked()
    with pytest.raises(ValueError):
        MaskPruneSchedule(k0=0)
