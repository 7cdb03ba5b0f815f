"""The paper's multi-core CPU scheme (Section 3: OpenMP loops inside the
sequential column loop), a timing baseline beside the GPU.  It is written
apart from the oracle (dense one-byte coefficients instead of bitsets) and
must agree with it exactly at every thread count: barcode, per-vertex deaths,
E_eff, |D| and the number of column additions.  CPU only."""
import numpy as np
import pytest

import oracle
from paper_2203_02527_amd import synth

INF = oracle.INF


def _clouds():
    rng = np.random.default_rng(11)
    return [
        ("n1", np.array([[3, -4]], np.int16)),
        ("n2", np.array([[0, 0, 0], [1, 2, 2]], np.int8)),
        ("identical", np.full((17, 3), 5, np.int16)),
        ("ties", rng.integers(0, 3, size=(90, 3)).astype(np.int16)),
        ("line_0_1_3_6_10", np.array([[0], [1], [3], [6], [10]], np.int8)),
        ("uniform_d3", synth.uniform_cloud(200, 3, seed=4)),
        ("mixture_d16", synth.mixture_cloud(300, 16, 4, 10.0, seed=5)),
        ("unit_square", synth.unit_square_cloud(257, seed=6)),
    ]


@pytest.mark.parametrize("name,x", _clouds())
@pytest.mark.parametrize("threads", [1, 2, 3])
def test_omp_matches_oracle(name, x, threads):
    ref = oracle.barcode(x)
    got = oracle.omp_barcode(x, threads)
    np.testing.assert_array_equal(got.canonical, ref.canonical)
    np.testing.assert_array_equal(got.death_by_vertex, ref.death_by_vertex)
    assert got.threads == threads
    assert (got.E, got.E_eff, got.distinct) == (ref.E, ref.E_eff, ref.distinct)
    assert got.additions == ref.additions
    assert got.pivots == x.shape[0] - 1


def test_omp_literal_mode_matches_early_exit():
    # Reducing every column (no stop at the (N-1)-th pivot) must not change
    # the barcode: every later column reduces to zero.
    x = synth.uniform_cloud(60, 3, seed=8)
    lit = oracle.omp_barcode(x, 2, early_exit=False)
    ee = oracle.omp_barcode(x, 2, early_exit=True)
    ref = oracle.barcode(x, early_exit=False)
    np.testing.assert_array_equal(lit.canonical, ee.canonical)
    assert lit.additions == ref.additions >= ee.additions
    assert lit.E_eff == ee.E_eff


def test_omp_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.omp_barcode(np.zeros((4, 2), np.int16), 0)
