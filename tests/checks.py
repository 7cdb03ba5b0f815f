"""Independent checkers for the H0 barcode, used to pin the oracle and the GPU.

None of these share code with the oracle (oracle/) or the GPU library.  They
reach the same results by other routes:

* ``sqdist_colex``      -- scipy's pdist (squared Euclidean, exact in float64
                           for these integer ranges), rearranged to colex order.
* ``sorted_order``      -- numpy's lexsort on (delta, j, i).
* ``kruskal_minlabel``  -- Kruskal's algorithm with a union-find that tracks
                           each component's minimum vertex: an edge joining two
                           components kills the larger of the two minima.  Over
                           F2 a column reduces to zero exactly when its edge
                           closes a cycle with earlier edges (graphic matroid),
                           so the death edges are Kruskal's spanning-tree edges.
* ``mst_grades_scipy``  -- scipy's minimum spanning tree; its weights, mapped
                           to 1-based indices in D, are the finite deaths.
* ``betti0_brute``      -- number of connected components of the graph of
                           edges with grade <= b, by breadth-first search.
* ``sparse_pair_walk``  -- the column reduction on 2-sparse columns kept as
                           index pairs: adding the stored column {c, r} to
                           {a, r} gives {a, c} (empty when a == c).
"""
from __future__ import annotations

from collections import deque

import numpy as np
from scipy.sparse.csgraph import minimum_spanning_tree
from scipy.spatial.distance import pdist

INF = 0xFFFFFFFF


def sqdist_colex(points: np.ndarray) -> np.ndarray:
    """Squared distances of all pairs i < j at index j(j-1)/2 + i."""
    n = points.shape[0]
    if n < 2:
        return np.zeros(0, np.int64)
    dd = pdist(points.astype(np.float64), metric="sqeuclidean")
    assert dd.max() < 2.0 ** 53
    i, j = np.triu_indices(n, 1)
    out = np.empty(dd.size, np.int64)
    out[j * (j - 1) // 2 + i] = dd.astype(np.int64)
    return out


def colex_pairs(n: int) -> tuple[np.ndarray, np.ndarray]:
    """(i, j) of every edge in colex order (j ascending, then i)."""
    j = np.repeat(np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64))
    start = j * (j - 1) // 2
    i = np.arange(j.size, dtype=np.int64) - start
    return i, j


def sorted_order(points: np.ndarray):
    """(delta, i, j, grade) of all edges sorted by (delta, j, i); grade 1-based."""
    n = points.shape[0]
    delta = sqdist_colex(points)
    i, j = colex_pairs(n)
    order = np.lexsort((i, j, delta))
    ds = delta[order]
    _, inv = np.unique(ds, return_inverse=True)
    return ds, i[order], j[order], (inv + 1).astype(np.uint32)


def kruskal_minlabel(points: np.ndarray, tie_perm_seed: int | None = None):
    """Per-vertex deaths by Kruskal + min-label union-find.

    Returns (vertex_deaths uint32[n], killer position int64[n]).  With
    tie_perm_seed set, edges of equal distance are visited in a random order
    (the canonical barcode must not change; the per-vertex one may).
    """
    n = points.shape[0]
    ds, ii, jj, gr = sorted_order(points)
    order = np.arange(ds.size)
    if tie_perm_seed is not None:
        rng = np.random.default_rng(tie_perm_seed)
        order = np.lexsort((rng.random(ds.size), ds))
    parent = list(range(n))
    minv = list(range(n))

    def find(v):
        while parent[v] != v:
            parent[v] = parent[parent[v]]
            v = parent[v]
        return v

    death = np.full(n, INF, np.uint32)
    killer = np.full(n, -1, np.int64)
    joined = 0
    for p in order:
        if joined == n - 1:
            break
        a, b = find(int(ii[p])), find(int(jj[p]))
        if a == b:
            continue
        hi = max(minv[a], minv[b])
        death[hi] = gr[p]
        killer[hi] = p
        parent[a] = b
        minv[b] = min(minv[a], minv[b])
        joined += 1
    return death, killer


def mst_grades_scipy(points: np.ndarray) -> np.ndarray:
    """Sorted finite deaths from scipy's minimum spanning tree weights."""
    n = points.shape[0]
    if n < 2:
        return np.zeros(0, np.uint32)
    delta = sqdist_colex(points)
    D = np.unique(delta)
    i, j = colex_pairs(n)
    w = np.zeros((n, n))
    w[i, j] = delta + 1.0  # scipy drops zero weights; shift keeps the order
    mst = minimum_spanning_tree(w).toarray()
    weights = np.sort(mst[mst > 0].astype(np.int64) - 1)
    assert weights.size == n - 1
    return (np.searchsorted(D, weights) + 1).astype(np.uint32)


def betti0_brute(points: np.ndarray):
    """Canonical deaths from component counts of the grade-b subgraphs."""
    n = points.shape[0]
    ds, ii, jj, gr = sorted_order(points)
    nd = int(gr.max()) if gr.size else 0

    def components(b):
        adj = [[] for _ in range(n)]
        for k in range(ds.size):
            if gr[k] <= b:
                adj[ii[k]].append(jj[k])
                adj[jj[k]].append(ii[k])
        seen = [False] * n
        c = 0
        for s in range(n):
            if seen[s]:
                continue
            c += 1
            seen[s] = True
            q = deque([s])
            while q:
                u = q.popleft()
                for v in adj[u]:
                    if not seen[v]:
                        seen[v] = True
                        q.append(v)
        return c

    deaths = []
    prev = components(0) if nd else n
    assert prev == n
    for b in range(1, nd + 1):
        cur = components(b)
        deaths += [b] * (prev - cur)
        prev = cur
    assert prev == 1
    return np.array(deaths + [INF], dtype=np.uint32)


def sparse_pair_walk(points: np.ndarray, early_exit: bool = True):
    """Column reduction with columns kept as index pairs.

    Returns dict(partner, vertex_deaths, additions, E_eff, killer).
    """
    n = points.shape[0]
    ds, ii, jj, gr = sorted_order(points)
    partner = np.full(n, -1, np.int64)
    death = np.full(n, INF, np.uint32)
    killer = np.full(n, -1, np.int64)
    adds = 0
    pivots = 0
    e_eff = 0
    for p in range(ds.size):
        if early_exit and pivots == n - 1:
            break
        a, r = int(ii[p]), int(jj[p])
        zero = False
        while partner[r] >= 0:
            c = int(partner[r])
            adds += 1
            if c == a:
                zero = True
                break
            a, r = min(a, c), max(a, c)
        if not zero:
            assert pivots < n - 1
            partner[r] = a
            death[r] = gr[p]
            killer[r] = p
            pivots += 1
            e_eff = p + 1
    return dict(partner=partner, vertex_deaths=death, additions=adds, E_eff=e_eff,
                killer=killer)


# ---- H1 (edge-by-triangle) checks ----
#
# Both are written apart from the oracle.  ``h1_pairing_by_ranks`` reads the
# pairing off ranks of submatrices of the boundary matrix (the pairing lemma
# of persistence: row e is the low of reduced column t exactly when
# r(>=e, <=t) - r(>=e, <t) - r(>e, <=t) + r(>e, <t) = 1, r = F2 rank of the
# rows and columns named), so it fixes which triangle each edge pairs with
# without performing any reduction.  ``h1_reduction_sets`` repeats the left to
# right reduction with each column kept as a Python set of edge rows, for the
# number of column additions.


def h1_boundary(points: np.ndarray):
    """Edge grades in sorted (delta, j, i) order and the triangle columns.

    Triangles are ordered by (sorted position of their latest edge, the vertex
    not on that edge); each column is the set of its three edge positions.
    Returns (grades uint32[E], list of (latest, third, frozenset))."""
    n = points.shape[0]
    ds, ii, jj, gr = sorted_order(points)
    pos = {}
    for q in range(ds.size):
        pos[(int(ii[q]), int(jj[q]))] = q
    cols = []
    for a in range(n):
        for b in range(a + 1, n):
            for c in range(b + 1, n):
                sides = {(a, b): c, (a, c): b, (b, c): a}
                q = {pos[s]: v for s, v in sides.items()}
                latest = max(q)
                cols.append((latest, q[latest], frozenset(q)))
    cols.sort(key=lambda t: (t[0], t[1]))
    return gr, cols


def _rank_profile(masks, lo_row):
    """F2 ranks of the first k columns restricted to rows >= lo_row, k = 0..T.

    Columns are int bitmasks over edge rows; elimination keys on the lowest
    set bit (any pivot rule gives the same rank)."""
    keep = ~((1 << lo_row) - 1)
    basis = {}
    out = [0]
    r = 0
    for m in masks:
        v = m & keep
        while v:
            lb = v & -v
            if lb in basis:
                v ^= basis[lb]
            else:
                basis[lb] = v
                r += 1
                break
        out.append(r)
    return out


def h1_pairing_by_ranks(points: np.ndarray) -> np.ndarray:
    """tri_of_edge[E]: the triangle index (in triangle order) paired with the
    edge at each sorted position, -1 if none, from the pairing lemma."""
    gr, cols = h1_boundary(points)
    E = gr.size
    masks = [sum(1 << e for e in c[2]) for c in cols]
    prof = [_rank_profile(masks, lo) for lo in range(E + 1)]  # prof[e][t + 1] = r(>=e, <=t)
    out = np.full(E, -1, np.int64)
    for e in range(E):
        for t in range(len(cols)):
            mu = prof[e][t + 1] - prof[e][t] - prof[e + 1][t + 1] + prof[e + 1][t]
            assert mu in (0, 1)
            if mu == 1:
                assert out[e] == -1
                out[e] = t
    return out


def h1_reduction_sets(points: np.ndarray, early_exit: bool = True):
    """Left to right reduction of the triangle columns kept as sets of edge
    rows (low = largest row).  Returns dict(tri_of_edge, additions, pivots)."""
    n = points.shape[0]
    gr, cols = h1_boundary(points)
    E = gr.size
    want = E - (n - 1)
    stored = {}
    paired = np.full(E, -1, np.int64)
    adds = pivots = 0
    for t, (_, _, col) in enumerate(cols):
        if early_exit and pivots == want:
            break
        c = set(col)
        while c and max(c) in stored:
            c ^= stored[max(c)]
            adds += 1
        if c:
            stored[max(c)] = c
            paired[max(c)] = t
            pivots += 1
    return dict(tri_of_edge=paired, additions=adds, pivots=pivots)
