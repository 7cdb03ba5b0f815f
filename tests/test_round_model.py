"""CPU models of the GPU reductions' round schemes, checked against the
oracle.  They restate, in plain Python on small clouds, the rules the HIP
kernels apply in parallel -- which survivors of a round may commit, what a
survivor keeps between rounds -- so that the rules themselves (not only the
kernels' results) are tested for reproducing the sequential left-to-right
reduction exactly: the same stored columns and the same addition counts.
CPU only; they share no code with the kernels."""
import numpy as np
import pytest

import oracle


def _sorted_pairs(x):
    x = np.asarray(x, dtype=np.int64)
    n = x.shape[0]
    ed = []
    for j in range(1, n):
        for i in range(j):
            ed.append((int(((x[i] - x[j]) ** 2).sum()), j, i))
    ed.sort()
    return ed


def h0_rounds(x, width, growth=1):
    """H0: a window of `width` sorted columns is walked against the table as
    committed at the start of the round; a survivor stops on a free row.
    Survivors commit if they precede the first survivor whose low repeats an
    earlier survivor's, or if no earlier survivor has their low r or has r as
    the root of its other row; the rest stay.  The window widens up to
    `growth` times while rounds leave almost nothing active."""
    ed = _sorted_pairs(x)
    n = len(x)
    part = [-1] * n
    killer = [-1] * n
    state = {}  # column -> (a, r, additions so far)
    done = {}   # finished column -> its additions
    F, w, pivots = 0, width, 0
    while pivots < n - 1:
        end = min(len(ed), F + w)
        surv = []
        for p in range(F, end):
            if p not in state:
                state[p] = (ed[p][2], ed[p][1], 0)
            a, r, s = state[p]
            if a < 0:
                continue  # final
            zero = False
            while part[r] >= 0:
                y = part[r]
                s += 1
                if y == a:
                    zero = True
                    break
                a, r = min(a, y), max(a, y)
            if zero:
                state[p] = (-1, -1, s)
                done[p] = s
                continue
            v = a
            while part[v] >= 0:
                v = part[v]
            state[p] = (a, r, s)
            surv.append((p, a, r, v))
        first_on = {}
        for p, a, r, v in surv:
            first_on.setdefault(r, p)
        fd = min([p for p, a, r, v in surv if first_on[r] != p], default=1 << 60)
        touch = {}
        for p, a, r, v in surv:
            touch[r] = min(touch.get(r, 1 << 60), p)
            touch[v] = min(touch.get(v, 1 << 60), p)
        stay = 0
        for p, a, r, v in surv:
            if p < fd or (first_on[r] == p and touch[r] == p):
                part[r] = a
                killer[r] = p
                done[p] = state[p][2]
                state[p] = (-1, -1, 0)
                pivots += 1
            else:
                stay += 1
        nf = F
        while nf < end and (nf in state and state[nf][0] < 0):
            nf += 1
        F = nf
        if stay < w / 256:
            w = min(2 * w, growth * width)
        elif stay > w / 16:
            w = max(width, w // 2)
    # Columns before the last pivot that are still open finish as zeros;
    # the sequential count covers the columns up to the last pivot only.
    last = max(killer)
    for p in range(last + 1):
        if p in state and state[p][0] >= 0:
            a, r, s = state[p]
            while part[r] >= 0:
                y = part[r]
                s += 1
                if y == a:
                    break
                a, r = min(a, y), max(a, y)
            done[p] = s
    adds = sum(v for p, v in done.items() if p <= last)
    return part, killer, adds


def _tri_order(ed, n):
    pos = {}
    for q, (_, j, i) in enumerate(ed):
        pos[(i, j)] = pos[(j, i)] = q
    tri = []
    for q, (_, j, i) in enumerate(ed):
        for k in range(n):
            if k != i and k != j and pos[(i, k)] < q and pos[(j, k)] < q:
                tri.append((q, pos[(i, k)], pos[(j, k)]))
    return tri


def h1_rounds(x):
    """H1: emergent pairs (the first triangle of each edge with that edge)
    are stored first; every other triangle is walked; a zero column is
    final; survivors before the first survivor that is not the smallest on
    its row commit; survivors whose row was just taken continue from their
    kept column; the others keep their walk."""
    ed = _sorted_pairs(x)
    n = len(x)
    tri = _tri_order(ed, n)
    owner, rows, first = {}, {}, {}
    for t, (q, e0, e1) in enumerate(tri):
        if q not in first:
            first[q] = t
            owner[q] = t
            rows[q] = {e0, e1, q}
    adds = 0

    def reduce(col, s):
        while col:
            low = max(col)
            if low not in owner:
                return low, col, s
            col = col ^ rows[low]
            s += 1
        return -1, col, s

    live = {}  # t -> (low, column, additions)
    for t, (q, e0, e1) in enumerate(tri):
        if first[q] == t:
            continue
        low, col, s = reduce({e0, e1, q}, 0)
        if low < 0:
            adds += s
        else:
            live[t] = (low, col, s)
    while live:
        minc = {}
        for t, (low, _, _) in live.items():
            minc[low] = min(minc.get(low, 1 << 60), t)
        fd = min([t for t, (low, _, _) in live.items() if minc[low] != t], default=1 << 60)
        for t in sorted(t for t in live if t < fd):
            low, col, s = live.pop(t)
            owner[low] = t
            rows[low] = col
            adds += s
        for t in [t for t, (low, _, _) in live.items() if low in owner]:
            low, col, s = live.pop(t)
            low, col, s = reduce(col, s)
            if low < 0:
                adds += s
            else:
                live[t] = (low, col, s)
    return {q: t for q, t in owner.items()}, adds


def _clouds(count, seed):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        n = int(rng.integers(3, 26))
        d = int(rng.integers(1, 4))
        hi = int(rng.choice([1, 3, 50]))
        yield rng.integers(-hi, hi + 1, size=(n, d)).astype(np.int16)


@pytest.mark.parametrize("width,growth", [(1, 1), (3, 4), (16, 1), (64, 4), (1 << 20, 1)])
def test_h0_round_rules_reproduce_the_sequential_reduction(width, growth):
    for x in _clouds(12, width):
        ref = oracle.barcode(x)
        part, killer, adds = h0_rounds(x, width, growth)
        n = x.shape[0]
        np.testing.assert_array_equal(np.array(part, np.int32), ref.partner)
        np.testing.assert_array_equal(np.array(killer, np.int64), ref.killer_pos)
        assert adds == ref.additions


def test_h1_round_rules_reproduce_the_sequential_reduction():
    for x in _clouds(16, 99):
        ref = oracle.h1_barcode(x, early_exit=False)
        owner, adds = h1_rounds(x)
        got = np.full(ref.tri_of_edge.size, -1, np.int64)
        for q, t in owner.items():
            got[q] = t
        np.testing.assert_array_equal(got, ref.tri_of_edge)
        assert adds == ref.additions


def test_first_repeat_from_returning_minima():
    """The round kernel finds the first survivor whose low repeats an earlier
    survivor's low without a pass of its own: each survivor lowers the
    per-row minimum with an atomic that returns the previous value, and
    when that value is another survivor of the same round, the larger of the
    two positions is a candidate.  Whatever order the atomics land in, the
    smallest candidate is the second-smallest survivor of some row and no
    candidate is smaller -- exactly the sequential definition."""
    rng = np.random.default_rng(11)
    for _ in range(400):
        m = int(rng.integers(1, 40))
        pos = rng.choice(10_000, size=m, replace=False)
        low = rng.integers(0, max(1, m // 3 + 1), size=m)
        # the definition: smallest position whose low already occurred earlier
        want = None
        seen = set()
        for p, r in sorted(zip(pos.tolist(), low.tolist())):
            if r in seen and want is None:
                want = p
            seen.add(r)
        for _ in range(5):
            cur = {}
            cand = None
            for k in rng.permutation(m):
                p, r = int(pos[k]), int(low[k])
                old = cur.get(r)
                if old is not None:
                    hi = max(old, p)
                    cand = hi if cand is None else min(cand, hi)
                cur[r] = p if old is None else min(old, p)
            assert cand == want
