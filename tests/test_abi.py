"""The C-ABI library loads and exports every symbol include/rtgs.h declares;
host-only entry points validate their arguments (no GPU needed)."""
import ctypes
import os
import re

import pytest

from oracle import selection
from paper_2510_06644_amd import rtgs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtgs.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int32_t|uint64_t|const char\*)\s+(\w+)\s*\(", text,
                                 flags=re.M)))


def test_library_is_built_and_loads():
    assert os.path.exists(rtgs.LIB_PATH), "run __graft_entry__.build() first"
    assert rtgs.lib() is not None


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 15
    L = ctypes.CDLL(rtgs.LIB_PATH)
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(rtgs.EXPORTS)


def test_workspace_size_is_host_arithmetic():
    a = rtgs.rtgs_workspace_size(2000, 128, 128, 10000)
    b = rtgs.rtgs_workspace_size(2000, 128, 128, 20000)
    c = rtgs.rtgs_workspace_size(4000, 128, 128, 10000)
    assert 0 < a < b and a < c
    assert b - a >= 10000 * 12 - 2 * 256     # keys + ids, each region 256-aligned
    both = rtgs.rtgs_workspace_size_batched([2000, 100], [128, 64], [128, 48], 10000)
    assert both > a
    with pytest.raises(rtgs.RtgsError) as e:
        rtgs.rtgs_workspace_size(-1, 128, 128, 10)
    assert e.value.code == rtgs.RTGS_ERR_INVALID_ARG
    with pytest.raises(rtgs.RtgsError):
        rtgs.rtgs_workspace_size(10, 0, 128, 10)
    with pytest.raises(rtgs.RtgsError):
        rtgs.rtgs_workspace_size(10, 16, 16, -5)
    with pytest.raises(rtgs.RtgsError):
        rtgs.rtgs_workspace_size_batched([1] * 65, [16] * 65, [16] * 65, 10)


def test_downsample_schedule_matches_oracle():
    for key in (True, False):
        for n in range(11, 20):
            for m in (2, 3, 4, 8):
                want = selection.downsample_log2_ratio(key, n, 10, m)
                assert rtgs.rtgs_downsample_log2_ratio(key, n, 10, m) == want
    with pytest.raises(rtgs.RtgsError):
        rtgs.rtgs_downsample_log2_ratio(False, 10, 10, 2)
    with pytest.raises(rtgs.RtgsError):
        rtgs.rtgs_downsample_log2_ratio(False, 12, 10, 1)


def test_null_handle_and_bad_arguments_are_rejected_before_any_gpu_work():
    L = rtgs.lib()
    g = rtgs.CGaussians()
    c = rtgs.CCamera()
    code = L.render_fwd(None, ctypes.byref(g), ctypes.byref(c), None, None, 0, 0, None, None,
                        None, None, None, None, 0, None)
    assert code == rtgs.RTGS_ERR_INVALID_ARG
    assert b"handle" in L.rtgs_last_error()
    code = L.downsample_mask(None, 4, 4, 2, None, None, None)
    assert code == rtgs.RTGS_ERR_INVALID_ARG
    code = L.prune_by_grad(None, None, None, None, None, 0, 0.8, 0.5, None, None, None, None)
    assert code == rtgs.RTGS_ERR_INVALID_ARG
    pairs = ctypes.c_int64()
    st = ctypes.c_int32()
    assert L.rtgs_query(None, 1, ctypes.byref(pairs), ctypes.byref(st)) == rtgs.RTGS_ERR_INVALID_ARG
    assert L.rtgs_selftest_wave_sum(None, None, -1, None) == rtgs.RTGS_ERR_INVALID_ARG
    assert L.pose_update(None, -1, 0.9, 0.999, 1e-8, None) == rtgs.RTGS_ERR_INVALID_ARG
    assert L.compact_by_mask(None, -1, None, 0, None, 0, None, None) == rtgs.RTGS_ERR_INVALID_ARG
    items = (rtgs.CCompactItem * 1)(rtgs.CCompactItem(8, 8, 4, 10))
    scratch = ctypes.c_void_p(64)
    cnt = ctypes.c_void_p(128)
    # the same address as src and dst: overlap is refused on the host
    assert L.compact_by_mask(ctypes.c_void_p(256), 10, items, 1, scratch, 64, cnt,
                             None) == rtgs.RTGS_ERR_INVALID_ARG
    assert L.compact_by_mask(ctypes.c_void_p(256), 10, items, 25, scratch, 64, cnt,
                             None) == rtgs.RTGS_ERR_INVALID_ARG
    items2 = (rtgs.CCompactItem * 1)(rtgs.CCompactItem(1024, 4096, 4, 10))
    assert L.compact_by_mask(ctypes.c_void_p(256), 10, items2, 1, scratch, 0, cnt,
                             None) == rtgs.RTGS_ERR_WORKSPACE
    assert int(L.rtgs_compact_scratch_size(0)) == 4
    assert int(L.rtgs_compact_scratch_size(1024)) == 8
    assert int(L.rtgs_compact_scratch_size(1025)) == 12
    assert L.tile_pair_change(None, None, None, 5, None, None) == rtgs.RTGS_ERR_INVALID_ARG
    assert L.loss_l1_grad_batched(None, 3, 1.0, 0.5, None) == rtgs.RTGS_ERR_INVALID_ARG
    assert L.rtgs_tile_rects(4, 16, 16, 0, 1024, None, 0, None, None) == rtgs.RTGS_ERR_INVALID_ARG
    assert L.pose_update(None, 0, 1.5, 0.999, 1e-8, None) == rtgs.RTGS_ERR_INVALID_ARG
    assert L.adam_step(None, None, 0, 0.9, 0.999, 1e-8, None) == rtgs.RTGS_ERR_INVALID_ARG
    assert L.loss_l1_grad(None, None, None, None, None, None, 0, 4, 1.0, 0.5, None, None,
                          None) == rtgs.RTGS_ERR_INVALID_ARG


def test_missing_library_and_host_tensors_fail_loudly(monkeypatch):
    """No fallback: a missing librtgs.so raises, and a host tensor is refused
    before any pointer reaches the library."""
    import torch
    monkeypatch.setattr(rtgs, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "librtgs.so"))
    monkeypatch.setattr(rtgs, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        rtgs.lib()
    with pytest.raises(ValueError, match="GPU tensors only"):
        rtgs._p(torch.zeros(4))


def test_static_compaction_rejects_rows_beyond_its_scratch():
    # argument checks run on the host before any device call
    L = rtgs.lib()
    dummy = ctypes.c_void_p(16)          # never dereferenced: the call fails first
    n = rtgs.RTGS_COMPACT_STATIC_MAX_ROWS + 1
    code = L.compact_by_mask_static(dummy, n, None, 0, dummy, None)
    assert code == rtgs.RTGS_ERR_WORKSPACE
    assert b"maximum" in L.rtgs_last_error()
    assert L.compact_by_mask_static(None, 5, None, 0, dummy, None) == rtgs.RTGS_ERR_INVALID_ARG
    assert L.compact_by_mask_static(dummy, -1, None, 0, dummy, None) == rtgs.RTGS_ERR_INVALID_ARG
