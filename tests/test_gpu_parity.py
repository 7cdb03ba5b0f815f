"""GPU parity: the HIP path against the CPU oracle, stage by stage, through
the C ABI.  Everything is integer, so every comparison is exact (tolerance 0).
"""
import hashlib
import json
import os
import zlib

import numpy as np
import pytest

import oracle
from paper_2203_02527_amd import ph0, synth
from tests.conftest import GOLDEN, golden_cases, load_fixture

pytestmark = pytest.mark.gpu

INF = 0xFFFFFFFF


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a HIP device"
    ph0.lib()
    return t


def _cloud(seed, n, d, lo, hi, dtype):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(n, d)).astype(dtype)


# (name, n, d, lo, hi, dtype): ragged tile tails, both distance paths, ties.
CASES = [
    ("n2_d1_i8", 2, 1, -5, 5, np.int8),
    ("n3_d2_i16", 3, 2, -100, 100, np.int16),
    ("n65_d3_i16", 65, 3, -100, 100, np.int16),
    ("n130_d3_tie", 130, 3, 0, 2, np.int8),
    ("n200_d8_i8_mfma", 200, 8, -128, 127, np.int8),
    ("n257_d16_i8", 257, 16, -128, 127, np.int8),
    ("n300_d64_i8", 300, 64, -20, 20, np.int8),
    ("n190_d100_i8", 190, 100, -128, 127, np.int8),
    ("n150_d300_i8", 150, 300, -128, 127, np.int8),
    ("n333_d5_i16", 333, 5, -16000, 16000, np.int16),
    ("n1000_d3_i16", 1000, 3, -1000, 1000, np.int16),
    ("n700_d2_tie", 700, 2, 0, 6, np.int8),
]


def _unpack(keys, n):
    k = keys.cpu().numpy().view(np.uint64)
    ib = (n - 1).bit_length()
    m = np.uint64((1 << ib) - 1)
    return (k >> np.uint64(2 * ib)).astype(np.int64), ((k >> np.uint64(ib)) & m).astype(np.int64), \
        (k & m).astype(np.int64)


def _dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_keys_match_oracle_distances(torch, case):
    name, n, d, lo, hi, dt = case
    x = _cloud(zlib.crc32(name.encode()) % 1000, n, d, lo, hi, dt)
    keys = ph0.ph0_keys_device(_dev(torch, x))
    torch.cuda.synchronize()
    delta, j, i = _unpack(keys, n)
    ref = oracle.sorted_edges(x)
    np.testing.assert_array_equal(delta, ref.colex_delta)
    jj = np.repeat(np.arange(n), np.arange(n))
    ii = np.arange(jj.size) - jj * (jj - 1) // 2
    np.testing.assert_array_equal(j, jj)
    np.testing.assert_array_equal(i, ii)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_sorted_keys_match_oracle(torch, case):
    name, n, d, lo, hi, dt = case
    x = _cloud(zlib.crc32(name.encode()) % 1000 + 1, n, d, lo, hi, dt)
    keys = ph0.ph0_sorted_keys_device(_dev(torch, x))
    torch.cuda.synchronize()
    delta, j, i = _unpack(keys, n)
    ref = oracle.sorted_edges(x)
    np.testing.assert_array_equal(delta, ref.delta)
    np.testing.assert_array_equal(j, ref.j)
    np.testing.assert_array_equal(i, ref.i)


def _check_full(torch, x, early=True):
    n = x.shape[0]
    ref = oracle.barcode(x)
    bars, st = ph0.ph0_barcodes_device(_dev(torch, x), with_stats=True)
    pr = ph0.ph0_pairs_device(_dev(torch, x))
    torch.cuda.synchronize()
    b = bars.cpu().numpy().view(np.uint32)
    assert (b[:, 0] == 0).all()
    np.testing.assert_array_equal(b[:, 1], ref.canonical)
    np.testing.assert_array_equal(pr.death_by_vertex.cpu().numpy().view(np.uint32),
                                  ref.death_by_vertex)
    np.testing.assert_array_equal(pr.killer_pos.cpu().numpy(), ref.killer_pos)
    np.testing.assert_array_equal(pr.partner.cpu().numpy(), ref.partner)
    if n > 1:
        assert st["E_eff"] == ref.E_eff
        assert st["additions"] == ref.additions
        assert st["distinct_eff"] == int(ref.canonical[-2])
        kp = ref.killer_pos
        se = oracle.sorted_edges(x)
        has = kp >= 0
        ke = pr.killer_edge.cpu().numpy().view(np.uint64)
        np.testing.assert_array_equal(ke[has] >> np.uint64(32), se.j[kp[has]].astype(np.uint64))
        np.testing.assert_array_equal(ke[has] & np.uint64(0xFFFFFFFF),
                                      se.i[kp[has]].astype(np.uint64))
        np.testing.assert_array_equal(pr.killer_sqdist.cpu().numpy()[has], se.delta[kp[has]])
    return st


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_barcode_matches_oracle(torch, case):
    name, n, d, lo, hi, dt = case
    x = _cloud(zlib.crc32(name.encode()) % 1000 + 2, n, d, lo, hi, dt)
    _check_full(torch, x)


@pytest.mark.parametrize("name", golden_cases())
def test_closed_form_cases(torch, name):
    pts, deaths, vdeaths = load_fixture(name)
    bars = ph0.ph0_barcodes_device(_dev(torch, pts)).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(bars[:, 1], deaths)
    pr = ph0.ph0_pairs_device(_dev(torch, pts))
    if vdeaths is not None:
        np.testing.assert_array_equal(pr.death_by_vertex.cpu().numpy().view(np.uint32), vdeaths)


def test_degenerate_inputs(torch):
    same = np.full((300, 4), 9, np.int8)  # all distances 0 -> no radix pass
    st = _check_full(torch, same)
    assert st["sort_passes"] == 0
    line = np.zeros((129, 1), np.int16)
    line[:, 0] = np.arange(129)
    _check_full(torch, line)
    ext = np.array([[-128] * 64, [127] * 64, [0] * 64, [-128] * 32 + [127] * 32], np.int8)
    _check_full(torch, ext)


def test_windows_give_identical_results(torch):
    x = synth.mixture_cloud(700, 16, 6, 10.0, seed=4)
    ref = oracle.barcode(x)
    try:
        for w in (1, 3, 64, 1000, 1 << 20):
            ph0.ph0_set_window(w)
            pr = ph0.ph0_pairs_device(_dev(torch, x))
            np.testing.assert_array_equal(pr.partner.cpu().numpy(), ref.partner)
            np.testing.assert_array_equal(pr.death_by_vertex.cpu().numpy().view(np.uint32),
                                          ref.death_by_vertex)
            assert pr.stats["additions"] == ref.additions
    finally:
        ph0.ph0_set_window(0)


def test_pairs_detail_at_n3000_int8_gram(torch):
    # Partners (the stored columns), per-vertex deaths and the addition count
    # on the int8 Gram path, several windows' worth of rounds.
    x = synth.mixture_cloud(3000, 16, 8, 10.0, seed=6)
    ref = oracle.barcode(x)
    pr = ph0.ph0_pairs_device(_dev(torch, x))
    np.testing.assert_array_equal(pr.partner.cpu().numpy(), ref.partner)
    np.testing.assert_array_equal(pr.death_by_vertex.cpu().numpy().view(np.uint32),
                                  ref.death_by_vertex)
    assert pr.stats["additions"] == ref.additions


def test_repeat_runs_are_bit_identical(torch):
    x = synth.mixture_cloud(2000, 16, 8, 10.0, seed=11)
    xd = _dev(torch, x)
    ws = ph0.alloc_workspace(2000, 16, x.dtype)
    first = ph0.ph0_pairs_device(xd, workspace=ws)
    for _ in range(3):
        again = ph0.ph0_pairs_device(xd, workspace=ws)
        assert torch.equal(first.partner, again.partner)
        assert torch.equal(first.death_by_vertex, again.death_by_vertex)


def test_host_entry_point(torch):
    x = _cloud(5, 400, 3, -100, 100, np.int16)
    bars, st = ph0.ph0_barcodes(x, with_stats=True)
    np.testing.assert_array_equal(bars[:, 1], oracle.barcode(x).canonical)
    one = ph0.ph0_barcodes(np.array([[1, 2, 3]], np.int16))
    assert one.tolist() == [[0, INF]]


def test_key_budget_error(torch):
    x = np.zeros((4097, 128), np.int16)
    x[0, :] = -32768
    x[1, :] = 32767
    stream = torch.cuda.Stream()
    with pytest.raises(ph0.Ph0Error) as ei:
        ph0.ph0_barcodes_device(_dev(torch, x), stream=stream)
    assert ei.value.code == -2
    # an error return leaves nothing queued on the caller's stream
    assert stream.query()


def test_batched_error_return_leaves_stream_idle(torch):
    # A fused cloud, then an oversized cloud (single-cloud path) whose key
    # budget fails: the call reports ERANGE with nothing left running.
    small = _cloud(9, 100, 64, -100, 100, np.int16)
    big = np.zeros((8193, 64), np.int16)  # 38 distance bits + 2 x 14 index bits
    big[0, :] = -32768
    big[1, :] = 32767
    pts = np.concatenate([small, big])
    offsets = np.array([0, 100, 8293], np.int64)
    stream = torch.cuda.Stream()
    with pytest.raises(ph0.Ph0Error) as ei:
        ph0.ph0_barcodes_batched_device(_dev(torch, pts), offsets, stream=stream)
    assert ei.value.code == -2
    assert stream.query()


def test_uniform_workload_n256(torch):
    _check_full(torch, synth.workload("uniform_n256_d3_i16", seed=0))


def test_mixture_workload_n4096(torch):
    st = _check_full(torch, synth.workload("mixture_n4096_d16_i8", seed=0))
    assert st["keys_path"] == 1
    assert st["sort_chunks"] >= 2  # several recomputed distance ranges


# Above 2^22 edges the keys of each distance range are recomputed and emitted
# in colex order instead of stored; these clouds exercise that path's edge
# cases: an outlier that puts the last pivot at the very end (so the ranges
# grow until the rest is sorted whole), massive ties (a few distinct
# distances, whole ranges in one histogram bin), and the vector ALU path.
def test_recomputed_ranges_outlier_forces_whole_sort(torch):
    x = _cloud(41, 3000, 3, -100, 100, np.int16)
    x[1234] = (16000, 16000, 16000)
    st = _check_full(torch, x)
    assert st["keys_path"] == 0 and st["E_eff"] > st["E"] // 2


def test_recomputed_ranges_long_grade_scan(torch):
    # The last pivot past 2^24 sorted edges: the grade pass holds more
    # per-256-position group counts (about 68,000) than one workgroup scans,
    # so they go through the block-wise scan.
    x = _cloud(44, 5900, 3, -100, 100, np.int16)
    x[4321] = (16000, 16000, 16000)
    st = _check_full(torch, x)
    assert st["E_eff"] > 256 * 65536


def _grid(u, lo, hi):
    # The int16 grid of the real-valued entry, in the same fp64 operations.
    return np.rint((u.astype(np.float64) - lo) * (32767.0 / (hi - lo))).astype(np.int16)


@pytest.mark.parametrize("n", [50, 700, 3000])
def test_real_valued_points_on_the_grid(torch, n):
    # The paper's workload (uniform points in the unit square) through the
    # real-valued entry: the barcode of the grid cloud, against the oracle.
    u = np.random.default_rng(100 + n).random((n, 2)).astype(np.float32)
    ref = oracle.barcode(_grid(u, 0.0, 1.0)).canonical
    bars = ph0.ph0_barcodes_f32_device(_dev(torch, u), 0.0, 1.0)
    np.testing.assert_array_equal(bars.cpu().numpy().view(np.uint32)[:, 1], ref)
    bars2, st = ph0.ph0_barcodes_f32_device(_dev(torch, u), 0.0, 1.0, with_stats=True)
    np.testing.assert_array_equal(bars2.cpu().numpy(), bars.cpu().numpy())
    assert st["n"] == n


def test_real_valued_points_degenerate_clouds(torch):
    # One point, two points, identical points, both interval ends, and
    # points near half-way between grid values (the same fp64 rounding on
    # both sides).
    clouds = [
        np.array([[0.25, 0.75]], np.float32),
        np.array([[0.0, 0.0], [1.0, 1.0]], np.float32),
        np.full((40, 2), 0.5, np.float32),
        np.array([[0.5 / 32767, 0.0], [1.5 / 32767, 0.0], [2.5 / 32767, 1.0], [0.0, 1.0]],
                 np.float32),
    ]
    for u in clouds:
        ref = oracle.barcode(_grid(u, 0.0, 1.0)).canonical
        bars = ph0.ph0_barcodes_f32_device(_dev(torch, u), 0.0, 1.0)
        np.testing.assert_array_equal(bars.cpu().numpy().view(np.uint32)[:, 1], ref)


def test_real_valued_points_other_interval_and_bad_values(torch):
    rng = np.random.default_rng(7)
    v = (rng.random((400, 3)) * 5.0 - 2.0).astype(np.float32)  # in [-2, 3)
    ref = oracle.barcode(_grid(v, -2.0, 3.0)).canonical
    bars = ph0.ph0_barcodes_f32_device(_dev(torch, v), -2.0, 3.0)
    np.testing.assert_array_equal(bars.cpu().numpy().view(np.uint32)[:, 1], ref)
    for bad in (3.5, -2.25, np.nan, np.inf):
        w = v.copy()
        w[17, 1] = bad
        with pytest.raises(ph0.Ph0Error) as ei:
            ph0.ph0_barcodes_f32_device(_dev(torch, w), -2.0, 3.0)
        assert ei.value.code == -1 and "outside" in str(ei.value)


def test_recomputed_ranges_massive_ties(torch):
    st = _check_full(torch, _cloud(42, 3100, 2, 0, 6, np.int8))
    assert st["E"] >= 1 << 22


def test_recomputed_ranges_mfma_ragged(torch):
    st = _check_full(torch, _cloud(43, 2990, 64, -128, 127, np.int8))
    assert st["keys_path"] == 1 and st["E"] >= 1 << 22


def _sha(a, dt):
    return hashlib.sha256(np.ascontiguousarray(a).astype(dt).tobytes()).hexdigest()


def _stored_records():
    names = (f[len("oracle_"):-len(".json")] for f in os.listdir(GOLDEN)
             if f.startswith("oracle_") and f.endswith(".json"))
    return sorted(r for r in names if r.rsplit("_s", 1)[0] in synth.WORKLOADS)


@pytest.mark.parametrize("record", _stored_records())
def test_workload_seeds_against_stored_oracle(torch, record):
    """Seeds 0-9 of the three single-cloud workloads, against the oracle's
    stored hashes (tests/golden/make_golden.py, oracle only)."""
    rec = json.load(open(os.path.join(GOLDEN, "oracle_%s.json" % record)))
    x = synth.workload(rec["workload"], seed=rec["seed"])
    assert _sha(x, x.dtype) == rec["points_sha256"]
    xd = _dev(torch, x)
    bars, st = ph0.ph0_barcodes_device(xd, with_stats=True)
    pr = ph0.ph0_pairs_device(xd)
    torch.cuda.synchronize()
    b = bars.cpu().numpy().view(np.uint32)
    assert _sha(b[:, 1], "<u4") == rec["canonical_sha256"]
    assert _sha(pr.death_by_vertex.cpu().numpy().view(np.uint32), "<u4") == \
        rec["death_by_vertex_sha256"]
    assert _sha(pr.killer_pos.cpu().numpy(), "<i8") == rec["killer_pos_sha256"]
    assert _sha(pr.partner.cpu().numpy(), "<i4") == rec["partner_sha256"]
    assert st["E_eff"] == rec["E_eff"] and st["additions"] == rec["additions"]
    assert st["E"] == rec["E"]


@pytest.mark.parametrize("n", [50, 150, 700, 3000])
def test_unit_square_workload(torch, n):
    # The paper's experiment: uniform points in [0,1]^2 on a fixed-point grid.
    _check_full(torch, synth.unit_square_cloud(n, seed=n))


# Single clouds of n <= 256 without statistics run in one workgroup (the fused
# kernel); with statistics they take the grid-wide passes.  Both must equal the
# oracle, at the size limit and beside it too.
@pytest.mark.parametrize("n,d,lo,hi,dtype", [
    (2, 1, -5, 5, np.int8),
    (3, 3, -100, 100, np.int16),
    (17, 2, 0, 2, np.int8),          # heavy ties
    (64, 64, -128, 127, np.int8),    # full int8 range, n * d = 4096
    (100, 16, -127, 127, np.int8),
    (128, 64, -128, 127, np.int8),   # n * d = 8192, the LDS limit
    (200, 3, -16000, 16000, np.int16),
    (256, 3, -100, 100, np.int16),   # the largest fused single cloud
    (257, 3, -100, 100, np.int16),   # the grid-wide path
])
def test_small_single_clouds_fused_and_grid_paths(torch, n, d, lo, hi, dtype):
    x = _cloud(n + 1000 * d, n, d, lo, hi, dtype)
    print("small single cloud n=%d d=%d %s" % (n, d, np.dtype(dtype).name), flush=True)
    ref = oracle.barcode(x).canonical
    xd = _dev(torch, x)
    fused = ph0.ph0_barcodes_device(xd)
    grid, _ = ph0.ph0_barcodes_device(xd, with_stats=True)
    torch.cuda.synchronize()
    for got in (fused, grid):
        b = got.cpu().numpy().view(np.uint32)
        assert (b[:, 0] == 0).all()
        np.testing.assert_array_equal(b[:, 1], ref)


def test_small_single_cloud_full_int16_range(torch):
    # 38 distance bits + 2 x 8 index bits: the widest keys a fused single cloud
    # can have (n * d <= 8192 keeps the distance bound below 2^48).
    x = _cloud(77, 200, 40, -1000, 1000, np.int16)
    x[0, :] = -32768
    x[1, :] = 32767
    bars = ph0.ph0_barcodes_device(_dev(torch, x))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(bars.cpu().numpy().view(np.uint32)[:, 1],
                                  oracle.barcode(x).canonical)
