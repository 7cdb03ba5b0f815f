"""Pins for the H1 part of the CPU oracle (the edge-by-triangle boundary
matrix).  Each pin comes from outside the oracle: persistent Betti numbers
computed from ranks of explicit boundary matrices over F2 (independent of any
column order), hand-derived closed forms, the topology of the complete
2-skeleton, and invariance under relabelling the points.  CPU only."""
import numpy as np
import pytest

import oracle


def _f2_rank(m):
    """Rank over F2 of a 0/1 matrix (plain Gaussian elimination)."""
    a = (np.asarray(m, dtype=np.uint8) & 1).copy()
    rows, cols = a.shape
    r = 0
    for c in range(cols):
        if r == rows:
            break
        piv = np.nonzero(a[r:, c])[0]
        if piv.size == 0:
            continue
        p = r + piv[0]
        if p != r:
            a[[r, p]] = a[[p, r]]
        hit = np.nonzero(a[:, c])[0]
        hit = hit[hit != r]
        a[hit] ^= a[r]
        r += 1
    return r


def _brute_h1(x):
    """H1 bars from persistent Betti numbers, written from the definitions.

    Grades: 1-based index of an edge's squared distance among the distinct
    ones; a triangle's grade is the largest of its edges'.  With K_b the
    complex of grade <= b, beta(b, c) = dim of the image of H1(K_b) in
    H1(K_c) = dim Z1(K_b) - dim(B1(K_c) restricted to edges of K_b), and
    dim(B1(K_c) on K_b edges) = rank d2(K_c) - rank(d2(K_c) rows of edges
    outside K_b).  The number of bars [b, e) is the inclusion-exclusion
    beta(b, e-1) - beta(b-1, e-1) - beta(b, e) + beta(b-1, e)."""
    x = np.asarray(x, dtype=np.int64)
    n = x.shape[0]
    pairs = [(i, j) for j in range(n) for i in range(j)]
    delta = np.array([int(((x[i] - x[j]) ** 2).sum()) for i, j in pairs], dtype=np.int64)
    D = np.unique(delta)
    eg = np.searchsorted(D, delta) + 1
    idx = {p: k for k, p in enumerate(pairs)}
    tris = [(a, b, c) for a in range(n) for b in range(a + 1, n) for c in range(b + 1, n)]
    d1 = np.zeros((n, len(pairs)), np.uint8)
    for k, (i, j) in enumerate(pairs):
        d1[i, k] = d1[j, k] = 1
    d2 = np.zeros((len(pairs), len(tris)), np.uint8)
    tg = np.zeros(len(tris), np.int64)
    for t, (a, b, c) in enumerate(tris):
        es = [idx[(a, b)], idx[(a, c)], idx[(b, c)]]
        d2[es, t] = 1
        tg[t] = eg[es].max()
    G = len(D)

    def beta(b, c):
        if b <= 0:
            return 0
        eb = eg <= b
        z = int(eb.sum()) - _f2_rank(d1[:, eb])
        bc = d2[:, tg <= c]
        if bc.shape[1] == 0:
            return z
        return z - (_f2_rank(bc) - _f2_rank(bc[~eb, :]))

    B = {(b, c): beta(b, c) for b in range(0, G + 1) for c in range(b, G + 1)}
    bars = []
    for b in range(1, G + 1):
        for e in range(b + 1, G + 1):
            mu = (B[(b, e - 1)] - B.get((b - 1, e - 1), 0) - B[(b, e)]
                  + B.get((b - 1, e), 0))
            assert mu >= 0
            bars += [(b, e)] * mu
        assert B[(b, G)] == 0 or b < G  # nothing survives the full complex
    assert B[(G, G)] == 0
    return np.array(sorted(bars), dtype=np.uint32).reshape(-1, 2)


def _tiny_clouds():
    rng = np.random.default_rng(21)
    out = []
    for k in range(24):
        n = int(rng.integers(3, 9))
        d = int(rng.integers(1, 4))
        hi = int(rng.choice([1, 2, 6, 40]))
        out.append(rng.integers(-hi, hi + 1, size=(n, d)).astype(np.int16))
    return out


@pytest.mark.parametrize("k", range(24))
def test_h1_matches_persistent_betti_numbers(k):
    x = _tiny_clouds()[k]
    res = oracle.h1_barcode(x)
    np.testing.assert_array_equal(res.bars, _brute_h1(x))


def test_h1_square_closed_form():
    # Unit square corners: four sides at delta 1 (grade 1) close one cycle,
    # which the diagonals (delta 2, grade 2) fill: the single bar [1, 2).
    sq = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.int8)
    res = oracle.h1_barcode(sq)
    np.testing.assert_array_equal(res.bars, [[1, 2]])
    assert res.pivots == 6 - 4 + 1 and res.zero_length == 2


def test_h1_collinear_points_have_no_bars():
    # Points on a line: every Vietoris-Rips complex is a union of contractible
    # interval-graph clique complexes, so H1 is zero at every grade.
    x = np.array([[0], [1], [3], [6], [10], [15], [21], [22]], np.int8)
    res = oracle.h1_barcode(x)
    assert res.bars.shape == (0, 2)
    assert res.pivots == res.zero_length == 28 - 8 + 1


@pytest.mark.parametrize("seed", range(4))
def test_h1_pair_count_and_invariance(seed):
    rng = np.random.default_rng(seed)
    n = 30
    x = rng.integers(-20, 21, size=(n, 3)).astype(np.int16)
    res = oracle.h1_barcode(x)
    E = n * (n - 1) // 2
    assert res.pivots == E - n + 1  # the complete 2-skeleton has no H1
    assert res.bars.shape[0] + res.zero_length == res.pivots
    assert (res.bars[:, 0] < res.bars[:, 1]).all()
    perm = rng.permutation(n)
    np.testing.assert_array_equal(oracle.h1_barcode(x[perm]).bars, res.bars)
    np.testing.assert_array_equal(oracle.h1_barcode(-x).bars, res.bars)
    lit = oracle.h1_barcode(x, early_exit=False)
    np.testing.assert_array_equal(lit.bars, res.bars)
    np.testing.assert_array_equal(lit.tri_of_edge, res.tri_of_edge)
    assert lit.additions >= res.additions and lit.columns == res.T


# ---- pairing and addition count, pinned apart from the oracle ----

from tests import checks  # noqa: E402


def _pin_clouds():
    """The tiny clouds above, eight with heavy ties (N up to 9) and eight with
    N = 10 to 16, where more pairs are not a triangle's own latest edge."""
    rng = np.random.default_rng(77)
    out = list(_tiny_clouds())
    for k in range(8):
        n = int(rng.integers(5, 10))
        out.append(rng.integers(0, 3, size=(n, 2)).astype(np.int8))
    for k in range(8):
        n = int(rng.integers(10, 17))
        hi = int(rng.choice([2, 40]))
        out.append(rng.integers(-hi, hi + 1, size=(n, 2)).astype(np.int16))
    return out


@pytest.mark.parametrize("k", range(40))
def test_h1_pairing_matches_pairing_lemma(k):
    # Which triangle each edge pairs with, from ranks of submatrices of the
    # boundary matrix alone: no column reduction is performed.
    x = _pin_clouds()[k]
    res = oracle.h1_barcode(x)
    np.testing.assert_array_equal(res.tri_of_edge, checks.h1_pairing_by_ranks(x))


@pytest.mark.parametrize("k", range(40))
def test_h1_additions_match_set_reduction(k):
    x = _pin_clouds()[k]
    for early in (True, False):
        res = oracle.h1_barcode(x, early_exit=early)
        ref = checks.h1_reduction_sets(x, early_exit=early)
        assert res.additions == ref["additions"]
        np.testing.assert_array_equal(res.tri_of_edge, ref["tri_of_edge"])
        assert res.pivots == ref["pivots"]


def test_h1_pins_catch_planted_mistakes(tmp_path):
    # Triangles of one latest edge taken in the wrong order (third vertex
    # descending): the pairing-lemma pin must fail on some cloud.  An uncounted clearing addition must fail the
    # set-reduction pin.  (Both mistakes leave the bars unchanged.)
    clouds = _pin_clouds()
    order = oracle.build_planted("PH0O_PLANT_H1_ORDER", str(tmp_path))
    by_pairing = by_count = 0
    for x in clouds:
        got = oracle.h1_barcode(x, lib=order)
        np.testing.assert_array_equal(got.bars, oracle.h1_barcode(x).bars)  # bars blind to it
        by_pairing += not np.array_equal(got.tri_of_edge, checks.h1_pairing_by_ranks(x))
        by_count += got.additions != checks.h1_reduction_sets(x)["additions"]
    assert by_pairing >= 2 and by_count >= 10
    count = oracle.build_planted("PH0O_PLANT_H1_COUNT", str(tmp_path))
    caught = 0
    for x in clouds:
        got = oracle.h1_barcode(x, lib=count).additions
        caught += got != checks.h1_reduction_sets(x)["additions"]
    assert caught >= 10
