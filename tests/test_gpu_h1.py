"""GPU parity of the H1 path (edge-by-triangle boundary matrix) against the
CPU oracle, through the C ABI: the bars, the edge-to-triangle pairing and the
number of column additions must be identical (all integer, tolerance 0).
The GPU reduces every column, so additions are compared with the oracle's
literal mode (no stop at the last pair)."""
import numpy as np
import pytest

import oracle
from paper_2203_02527_amd import ph0, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a HIP device"
    ph0.lib()
    return t


def _run(torch, x):
    print("h1 case n=%d d=%d %s" % (x.shape[0], x.shape[1], x.dtype), flush=True)
    xd = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    bars, toe, st = ph0.ph0_h1_device(xd, with_stats=True)
    torch.cuda.synchronize()
    return bars.cpu().numpy().view(np.uint32).reshape(-1, 2), toe.cpu().numpy(), st


def _check(torch, x):
    got, toe, st = _run(torch, x)
    ref = oracle.h1_barcode(x, early_exit=False)
    np.testing.assert_array_equal(got, ref.bars)
    np.testing.assert_array_equal(toe, ref.tri_of_edge)
    n = x.shape[0]
    assert st["pivots"] == n * (n - 1) // 2 - n + 1 == ref.pivots
    assert st["bars"] == ref.bars.shape[0] and st["zero_length"] == ref.zero_length
    assert st["additions"] == ref.additions
    return st


def _rand(seed, n, d, lo, hi, dtype):
    return np.random.default_rng(seed).integers(lo, hi + 1, size=(n, d)).astype(dtype)


@pytest.mark.parametrize("n,d,lo,hi,dtype", [
    (3, 2, -100, 100, np.int16),
    (7, 1, -3, 3, np.int8),      # collinear with ties
    (20, 2, 0, 2, np.int8),      # heavy ties
    (33, 3, -100, 100, np.int16),
    (64, 3, -100, 100, np.int16),
    (65, 4, -10, 10, np.int8),   # a ragged word of the dense columns
    (100, 16, -127, 127, np.int8),
])
def test_h1_random_clouds(torch, n, d, lo, hi, dtype):
    _check(torch, _rand(n, n, d, lo, hi, dtype))


def test_h1_square_and_trivial_sizes(torch):
    sq = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.int8)
    got, toe, st = _run(torch, sq)
    np.testing.assert_array_equal(got, [[1, 2]])
    for n in (1, 2):
        got, toe, st = _run(torch, np.zeros((n, 3), np.int16))
        assert got.shape == (0, 2) and (toe == -1).all()


def test_h1_workload_shapes(torch):
    # Circle and mixture clouds of the batch and serving workloads, and the
    # paper's unit square, at sizes the oracle finishes in seconds; more than
    # 64 words per dense column (two and four slots per lane).
    rng = np.random.default_rng(5)
    st = _check(torch, synth.circle_cloud(rng, 120))
    assert st["bars"] >= 1  # the circle's long cycle
    _check(torch, synth.mixture_cloud(128, 16, 3, 10.0, seed=9))
    _check(torch, synth.unit_square_cloud(150, seed=3))


def test_h1_repeated_calls_are_identical(torch):
    x = synth.uniform_cloud(90, 3, seed=12)
    a = _run(torch, x)
    b = _run(torch, x)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_h1_statistics_count_emergent_and_committed_pairs(torch):
    # Every pair is either emergent (the first triangle of an edge, whose
    # latest edge that is, stored unreduced) or committed by a round.  The
    # emergent ones are exactly the edges that are the latest edge of some
    # triangle, counted here from the sorted edge list.
    n = 80
    x = synth.uniform_cloud(n, 3, seed=4)
    got, toe, st = _run(torch, x)
    se = oracle.sorted_edges(x)
    pos = np.full((n, n), -1, np.int64)
    pos[se.i, se.j] = pos[se.j, se.i] = np.arange(se.delta.size)
    emergent = 0
    for q in range(se.delta.size):
        i, j = se.i[q], se.j[q]
        others = np.array([k for k in range(n) if k != i and k != j])
        emergent += bool(((pos[i, others] < q) & (pos[j, others] < q)).any())
    E = n * (n - 1) // 2
    assert st["pivots"] == E - n + 1
    assert st["emergent"] == emergent
    assert st["bars"] + st["zero_length"] == st["pivots"]
    assert st["walks"] >= st["T"] - st["emergent"]


@pytest.mark.parametrize("n", [362, 512])
def test_h1_full_size_properties(torch, n):
    # Beyond the oracle's reach in a test (its dense reduction of 8-22 M
    # triangle columns takes minutes): every positive edge is paired (E - n + 1
    # pairs, bars of positive length in canonical order), repeated calls are
    # bit-identical, and relabelling the points leaves the bars unchanged.
    # These sizes use 16 and 32 words per lane for the dense columns.
    x = synth.uniform_cloud(n, 3, seed=1)
    got, toe, st = _run(torch, x)
    E = n * (n - 1) // 2
    assert st["pivots"] == E - n + 1 == int((toe >= 0).sum())
    assert got.shape[0] == st["bars"] and (got[:, 0] < got[:, 1]).all()
    assert (np.diff(got[:, 0].astype(np.int64)) >= 0).all()
    again, toe2, _ = _run(torch, x)
    np.testing.assert_array_equal(again, got)
    np.testing.assert_array_equal(toe2, toe)
    perm = np.random.default_rng(n).permutation(n)
    permuted, _, _ = _run(torch, x[perm])
    np.testing.assert_array_equal(permuted, got)


def test_h1_benchmark_cloud_against_stored_oracle(torch):
    # The cloud the benchmark times (uniform N=256, d=3 int16, seed 0), against
    # the oracle's stored record (tests/golden/make_golden.py --h1 256 0, oracle
    # only; literal mode, about a minute on one core).
    import hashlib
    import json
    import os

    from tests.conftest import GOLDEN

    rec = json.load(open(os.path.join(GOLDEN, "oracle_h1_uniform_n256_d3_i16_s0.json")))
    x = synth.uniform_cloud(256, 3, seed=0)
    assert hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest() == rec["points_sha256"]
    got, toe, st = _run(torch, x)
    assert hashlib.sha256(got.astype("<u4").tobytes()).hexdigest() == rec["bars_sha256"]
    assert hashlib.sha256(toe.astype("<i8").tobytes()).hexdigest() == rec["tri_of_edge_sha256"]
    assert st["pivots"] == rec["pivots"] and st["additions"] == rec["additions"]
    assert st["bars"] == rec["bars"] and st["zero_length"] == rec["zero_length"]
