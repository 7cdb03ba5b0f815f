"""The C-ABI library loads, exports every declared symbol, and its argument
checks (which run before any device call) behave as documented.  CPU only."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2203_02527_amd import ph0

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ph0.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ph0_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = ph0.lib()
    names = _declared()
    assert "ph0_barcodes_device" in names and len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(ph0.EXPORTED)


def test_workspace_bytes_and_arguments():
    ws = ph0.ph0_workspace_bytes(16384, 64, np.int8)
    E = 16384 * 16383 // 2
    assert ws >= 2 * 8 * E  # two key buffers dominate
    assert ws < 3 * 8 * E
    for n, d in [(0, 3), (-1, 3), (5, 0), (70000, 3)]:
        with pytest.raises(ph0.Ph0Error) as ei:
            ph0.ph0_workspace_bytes(n, d, np.int8)
        assert ei.value.code == -1
    with pytest.raises(TypeError):
        ph0.ph0_workspace_bytes(5, 3, np.int32)


def test_f32_workspace_bytes_and_arguments():
    # The real-valued entry holds the int16 grid copy and a flag beside the
    # int16 workspace; its argument checks run before any device work.
    base = ph0.ph0_workspace_bytes(3000, 2, np.int16)
    ws = ph0.ph0_workspace_bytes_f32(3000, 2)
    assert base + 2 * 3000 * 2 <= ws <= base + 2 * 3000 * 2 + 1024
    for n, d in [(0, 2), (70000, 2), (5, 0)]:
        with pytest.raises(ph0.Ph0Error) as ei:
            ph0.ph0_workspace_bytes_f32(n, d)
        assert ei.value.code == -1
    lib = ph0.lib()
    dummy = ctypes.c_void_p(16)  # never dereferenced: the checks fail first
    for lo, hi in [(1.0, 1.0), (2.0, 1.0), (float("nan"), 1.0), (0.0, float("inf"))]:
        rc = lib.ph0_barcodes_f32_device(dummy, 10, 2, lo, hi, dummy, dummy, 1 << 30, None, None)
        assert rc == -1 and b"finite lo < hi" in ph0.ph0_last_error().encode()
    rc = lib.ph0_barcodes_f32_device(dummy, 10, 2, 0.0, 1.0, dummy, dummy, 16, None, None)
    assert rc == -1 and b"workspace too small" in ph0.ph0_last_error().encode()
    rc = lib.ph0_barcodes_f32_device(None, 10, 2, 0.0, 1.0, dummy, dummy, 1 << 30, None, None)
    assert rc == -1


def test_key_layout_bit_budget():
    rc, ib, db = ph0.ph0_key_layout(16384, 64, np.int8)
    assert rc == 0 and ib == 14 and db == 22  # 64 * 255^2 < 2^22
    rc, ib, db = ph0.ph0_key_layout(256, 3, np.int16)
    assert rc == 0 and ib == 8 and db == 34
    rc, ib, db = ph0.ph0_key_layout(16384, 64, np.int16)
    assert rc == -2 and 2 * ib + db > 64  # full-range int16 does not fit
    rc, ib, _ = ph0.ph0_key_layout(2, 1, np.int8)
    assert rc == 0 and ib == 1


def test_host_entry_rejects_bad_arguments_before_device_use():
    with pytest.raises(ph0.Ph0Error) as ei:
        ph0.ph0_barcodes(np.zeros((0, 3), np.int8))
    assert ei.value.code == -1
    with pytest.raises(TypeError):
        ph0.ph0_barcodes(np.zeros((4, 3), np.float32))
    assert ph0.ph0_set_window(0) is None
    with pytest.raises(ph0.Ph0Error):
        ph0.ph0_set_window(-5)


def test_tuning_table_loader(tmp_path):
    from paper_2203_02527_amd import autotune

    assert autotune.load(str(tmp_path / "absent.json")) is None
    good = tmp_path / "good.json"
    good.write_text('{"chunk_mult": [8, 12, 16, 24], "blocks_per_cu": 1}')
    assert autotune.load(str(good))["chunk_mult"] == [8, 12, 16, 24]
    ok = tmp_path / "ok.json"
    ok.write_text('{"chunk_mult": [8, 12, 16, 24], "blocks_per_cu": 2, "waves_per_cloud": 16, '
                  '"digit_bits": 6}')
    assert autotune.load(str(ok))["digit_bits"] == 6
    for bad in ('{"chunk_mult": [8, 12, 16], "blocks_per_cu": 1}',
                '{"chunk_mult": [8, 12, 16, 0], "blocks_per_cu": 1}',
                '{"chunk_mult": [8, 12, 16, 24], "blocks_per_cu": 3}',
                '{"chunk_mult": [8, 12, 16, 24], "blocks_per_cu": 2, "waves_per_cloud": 12}',
                '{"chunk_mult": [8, 12, 16, 24], "blocks_per_cu": 2, "digit_bits": 9}'):
        p = tmp_path / "bad.json"
        p.write_text(bad)
        with pytest.raises(ValueError):
            autotune.load(str(p))
    if os.path.exists(autotune.TABLE):  # the committed table must load
        assert autotune.load() is not None


def test_h1_workspace_bytes_and_size_limit():
    n = 256
    E, T = n * (n - 1) // 2, n * (n - 1) * (n - 2) // 6
    ws = ph0.ph0_h1_workspace_bytes(n, 3, np.int16)
    assert ws >= 8 * E * ((E + 63) // 64) + 20 * T  # dense stored columns + triangle lists
    assert ph0.ph0_h1_workspace_bytes(3, 2, np.int8) > 0
    with pytest.raises(ph0.Ph0Error) as ei:
        ph0.ph0_h1_workspace_bytes(513, 3, np.int16)
    assert ei.value.code == -2
    with pytest.raises(ph0.Ph0Error) as ei:
        ph0.ph0_h1_workspace_bytes(0, 3, np.int16)
    assert ei.value.code == -1


def test_batched_host_entry_rejects_bad_tuning_text_before_device_use():
    pts = np.zeros((6, 3), np.int16)
    offsets = np.array([0, 2, 6], np.int64)
    for bad in ('', '[]', '{"chunk_mult": [1, 2, 3, 4, 5]}', '{"chunk_mult": [-1]}',
                '{"blocks": 1}', '{"blocks_per_cu": 1,}', '{"blocks_per_cu": 1} x',
                '{"chunk_mult": [1, 2', '{"chunk_mult"', '{"digit_bits": 9}',
                '{"waves_per_cloud": 12}', '{"waves_per_cloud": -8}'):
        with pytest.raises(ph0.Ph0Error) as ei:
            ph0.ph0_barcodes_batched(pts, offsets, tune_json=bad)
        assert ei.value.code == -1, bad
        assert "tuning" in str(ei.value), bad
    with pytest.raises(ph0.Ph0Error) as ei:  # offsets checked before any device call
        ph0.ph0_barcodes_batched(pts, np.array([1, 2, 6], np.int64), tune_json="{}")
    assert ei.value.code == -1


def test_noalloc_batched_entry_limits_checked_before_device_use():
    import ctypes

    f = ph0.lib().ph0_barcodes_batched_device_noalloc
    dummy = ctypes.c_void_p(16)  # never dereferenced: both calls fail in planning
    big = np.array([0, 40, 553], np.int64)  # a 513-point cloud
    rc = f(dummy, ph0.PH0_I16, big.ctypes.data_as(ctypes.c_void_p), 2, 3, dummy, None, None)
    assert rc == -1 and "allocation-free" in ph0.ph0_last_error()
    many = np.zeros(9_000_001, np.int64)  # 9 million empty clouds: 144 MB of fixed workspace
    rc = f(dummy, ph0.PH0_I16, many.ctypes.data_as(ctypes.c_void_p), many.size - 1, 3, dummy,
           None, None)
    assert rc == -3 and "available" in ph0.ph0_last_error()
