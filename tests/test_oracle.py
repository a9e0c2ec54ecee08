"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these retypes the oracle's formulas: each compares it with a
printed value, a closed form, a library routine on an equivalent problem,
an invariant, or a brute force written independently in Python.
"""
import math
import os

import numpy as np
import pytest
import scipy.spatial.distance as ssd

import workloads
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ---------------------------------------------------------------- ranks ----

def test_sortperm_matches_paper_example(orc):
    """Section 4.5 prints sortperm([7,3,8,4,2]) = [5,2,4,1,3] (1-based)."""
    rows = dict((r[0], [int(x) for x in r[1:]]) for r in _golden_rows("sortperm_example.txt"))
    got = orc.sortperm(rows["v"])
    assert [int(x) + 1 for x in got] == rows["sortperm"]


@pytest.mark.parametrize("seed", range(6))
def test_edge_order_equals_stable_library_sort(orc, seed):
    """Ranks = stable sort on q, ties by pair index (lexsort on (q, i, j))."""
    c = workloads.lattice_cloud(seed, 20 + seed, side=3)  # many exact ties
    q = orc.sqdist(c.points)
    i, j = orc.pair_lists(c.n)
    ref = np.lexsort((j, i, q))
    assert np.array_equal(orc.sortperm(q), ref)
    assert np.array_equal(orc.sortperm(q), np.argsort(q, kind="stable"))


# ------------------------------------------------------------ distances ----

@pytest.mark.parametrize("dtype,lo,hi", [(np.int8, -128, 127), (np.int16, -3000, 3000), (np.int32, 0, 1023)])
def test_sqdist_three_ways(orc, dtype, lo, hi):
    """Direct sum, the Gram identity |x|^2+|y|^2-2<x,y>, and scipy agree."""
    rng = np.random.default_rng(7)
    pts = rng.integers(lo, hi + 1, (23, 5)).astype(dtype)
    q = orc.sqdist(pts)
    x = pts.astype(np.int64)
    g = x @ x.T
    nrm = np.diag(g)
    i, j = orc.pair_lists(len(pts))
    gram = nrm[i] + nrm[j] - 2 * g[i, j]
    assert np.array_equal(q, gram)
    sp = ssd.pdist(x.astype(np.float64), "sqeuclidean")
    assert np.array_equal(q, sp.astype(np.int64))
    bd = bf.sqdist_pairs(pts)
    assert [bd[(a, b)] for a, b in zip(i, j)] == list(q)


def test_sqdist_extreme_int8(orc):
    """-128 against 127 in every coordinate: q = d * 255^2 exactly."""
    d = 64
    pts = np.array([[-128] * d, [127] * d], np.int8)
    assert orc.sqdist(pts).tolist() == [d * 255 * 255]


# ------------------------------------------------------------ threshold ----

def test_num_kept_closed_forms(orc):
    """K = floor(num * E / den): 20% of C(1000,2) and 10% of C(4000,2)."""
    assert orc.num_kept(("fraction", 20, 100), np.zeros(499500, np.int64)) == 99900
    assert orc.num_kept(("fraction", 10, 100), np.zeros(7998000, np.int64)) == 799800
    assert orc.num_kept(("full", 0, 1), np.zeros(2016, np.int64)) == 2016
    assert orc.num_kept(("fraction", 1, 3), np.zeros(10, np.int64)) == 3  # floor(10/3)
    assert orc.num_kept(("count", 7, 1), np.zeros(10, np.int64)) == 7
    with pytest.raises(ValueError):
        orc.num_kept(("count", 11, 1), np.zeros(10, np.int64))
    with pytest.raises(ValueError):
        orc.num_kept(("fraction", 101, 100), np.zeros(10, np.int64))


def test_sqdist_threshold_is_strict(orc):
    """Edges join points closer than the threshold (Section 2.1): q < tau."""
    q = np.array([4, 1, 4, 9, 0, 4], np.int64)
    assert orc.num_kept(("sqdist", 4, 0), q) == 2
    assert orc.num_kept(("sqdist", 5, 0), q) == 5
    assert orc.num_kept(("sqdist", 0, 0), q) == 0


# ------------------------------------------------------------ triangles ----

def _K_of(thr):
    kind, num, den = thr

    def f(qs):
        E = len(qs)
        if kind == "full":
            return E
        if kind == "count":
            return num
        if kind == "fraction":
            return (num * E) // den
        return sum(1 for v in qs if v < num)

    return f


CASES = [
    workloads.uniform_cloud(1, 9, 2, thr=("full", 0, 1)),
    workloads.uniform_cloud(2, 11, 3, thr=("fraction", 40, 100)),
    workloads.lattice_cloud(3, 12, side=3, thr=("fraction", 50, 100)),   # duplicates and ties
    workloads.lattice_cloud(4, 10, side=2, thr=("count", 17, 1)),
    workloads.uniform_cloud(5, 12, 4, thr=("sqdist", 20000, 0)),
    workloads.uniform_cloud(6, 3, 1, thr=("full", 0, 1)),
    workloads.uniform_cloud(7, 2, 2, thr=("full", 0, 1)),
    workloads.uniform_cloud(8, 1, 2, thr=("full", 0, 1)),
    workloads.lattice_cloud(9, 8, side=1, thr=("fraction", 60, 100)),    # all points equal
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c.name + "_" + c.thr[0])
def test_filtration_matches_bruteforce(orc, case):
    kept, rank, tris, _ = bf.filtration(case.points, _K_of(case.thr))
    f = orc.build(case.points, case.thr)
    assert f.K == len(kept)
    assert list(zip(f.ei.tolist(), f.ej.tolist())) == kept
    assert [tuple(r) for r in f.tris.tolist()] == tris


@pytest.mark.parametrize("n", [3, 4, 10, 64])
def test_full_threshold_counts_are_binomials(orc, n):
    """At the infinite threshold every pair and triple is a simplex."""
    c = workloads.uniform_cloud(n, n, 2, dtype=np.int32, lo=0, hi=1023)
    f = orc.build(c.points, ("full", 0, 1))
    assert (f.K, f.T) == (math.comb(n, 2), math.comb(n, 3))


def test_plain64_counts(orc):
    f = orc.build(*_cloud_args(workloads.plain64()))
    assert f.counts == (64, 2016, 41664)


def _cloud_args(c):
    return c.points, c.thr


@pytest.mark.parametrize("row", _golden_rows("complex_sizes.txt"), ids=lambda r: r[0])
def test_paper_complex_sizes(orc, row):
    """Table 5's size of complex = n + C(n,2) + C(n,3) at the infinite threshold,
    to the paper's two significant figures; counts come from the oracle's own
    triangle test on a random cloud of that many points."""
    name, n, mant, expo = row[0], int(row[1]), float(row[2]), int(row[3])
    c = workloads.uniform_cloud(n, n, 3)
    f = orc.build(c.points, ("full", 0, 1), list_triangles=False)
    size = f.n + f.K + f.T
    assert round(size / 10 ** expo, 1) == mant


@pytest.mark.parametrize("seed,thr", [(11, ("fraction", 30, 100)), (12, ("fraction", 8, 100)), (13, ("count", 500, 1))])
def test_triangle_count_by_adjacency_cube(orc, seed, thr):
    """T = trace(A^3)/6 and, per vertex, (A^3)_vv / 2 triangles contain v."""
    c = workloads.uniform_cloud(seed, 120, 3, thr=thr)
    f = orc.build(c.points, c.thr)
    A = (f.R >= 0).astype(np.int64)
    A3 = A @ A @ A
    assert f.T == np.trace(A3) // 6
    per_vertex = np.zeros(f.n, np.int64)
    for col in (1, 2, 3):
        np.add.at(per_vertex, f.tris[:, col], 1)
    assert np.array_equal(per_vertex, np.diag(A3) // 2)


def test_triangles_per_value_partition(orc):
    c = workloads.noisy_circle(n=300)
    f = orc.build(c.points, c.thr)
    cnt = orc.triangles_per_value(f)
    assert cnt.sum() == f.T
    assert np.array_equal(cnt, np.bincount(f.tris[:, 0], minlength=f.K))
    for r in (0, f.K // 3, f.K - 1):
        rows = orc.triangles_of_value(f, r)
        assert np.array_equal(rows, f.tris[f.tris[:, 0] == r])


# ------------------------------------------------------------ reduction ----

def _pairs_in_total_order(f, p):
    """(birth, death) pairs and essential births as total-order indices."""
    order = bf.total_order(f.n, list(zip(f.ei.tolist(), f.ej.tolist())), [tuple(t) for t in f.tris.tolist()])
    pos = {s: i for i, s in enumerate(order)}
    vid = lambda v: pos[("v", (v,))]
    eid = lambda r: pos[("e", (int(f.ei[r]), int(f.ej[r])))]
    tid = lambda t: pos[("t", tuple(int(x) for x in f.tris[t, 1:]))]
    pairs = {0: [], 1: []}
    for r in np.nonzero(p.e_low >= 0)[0]:
        pairs[0].append((vid(int(p.e_low[r])), eid(r)))
    for t in np.nonzero(p.t_low >= 0)[0]:
        pairs[1].append((eid(int(p.t_low[t])), tid(t)))
    e0, e1, e2 = p.essential()
    ess = {0: [vid(v) for v in e0], 1: [eid(r) for r in e1], 2: [tid(t) for t in e2]}
    return len(order), pairs, ess


@pytest.mark.parametrize("case", [
    workloads.uniform_cloud(21, 6, 2, thr=("full", 0, 1)),
    workloads.uniform_cloud(22, 7, 2, thr=("fraction", 70, 100)),
    workloads.lattice_cloud(23, 7, side=3, thr=("fraction", 60, 100)),
    workloads.uniform_cloud(24, 6, 3, thr=("count", 9, 1)),
], ids=lambda c: c.name)
@pytest.mark.parametrize("method", ["homology", "cohomology"])
def test_reduction_matches_bruteforce_persistent_betti(orc, case, method):
    """Pairs reproduce every persistent Betti number rank(H_k(X_s) -> H_k(X_t))."""
    f = orc.build(case.points, case.thr)
    p = orc.reduce(f, method)
    N, pairs, ess = _pairs_in_total_order(f, p)
    _, beta = bf.persistent_betti(f.n, list(zip(f.ei.tolist(), f.ej.tolist())), [tuple(t) for t in f.tris.tolist()])
    got = bf.betti_from_pairs(N, pairs, ess)
    for k in (0, 1, 2):
        assert got[k] == beta[k], f"dimension {k}"


@pytest.mark.parametrize("case", [
    workloads.uniform_cloud(21, 6, 2, thr=("full", 0, 1)),
    workloads.uniform_cloud(22, 7, 2, thr=("fraction", 70, 100)),
    workloads.lattice_cloud(23, 7, side=3, thr=("fraction", 60, 100)),
    workloads.uniform_cloud(24, 6, 3, thr=("count", 9, 1)),
    workloads.uniform_cloud(25, 8, 2, thr=("fraction", 45, 100)),
], ids=lambda c: c.name)
def test_barcode_reproduces_persistent_betti_by_value(orc, case):
    """The barcode in filtration values (vertices -1, edge r at r, a triangle
    at its largest edge rank): for every pair of values s <= t, the bars of
    dimension k with birth <= s and death > t number rank(H_k(X_s) -> H_k(X_t)),
    X_s being every simplex of value <= s (brute force from F2 ranks).  A
    bar read backwards (birth after death) is never counted, so a swapped
    orientation fails; zero-length bars are absent and every bar is
    born strictly before it dies."""
    f = orc.build(case.points, case.thr)
    bars = orc.barcode(f, orc.reduce(f, "cohomology"))
    assert all(b < d for _, b, d in bars)
    kept = list(zip(f.ei.tolist(), f.ej.tolist()))
    tris = [tuple(t) for t in f.tris.tolist()]
    order, beta = bf.persistent_betti(f.n, kept, tris)
    # last total-order index of a simplex of value <= s
    value_of = {("e", e): r for r, e in enumerate(kept)}
    value_of.update({("t", tuple(t[1:])): t[0] for t in tris})
    last = {-1: f.n - 1}
    for p_, (kind, verts) in enumerate(order):
        if kind != "v":
            last[value_of[(kind, verts)]] = p_
    values = sorted(last)
    assert values == list(range(-1, f.K))
    for k in (0, 1, 2):
        for s in values:
            for t in values:
                if t < s:
                    continue
                alive = sum(1 for dim, b, d in bars if dim == k and b <= s and d > t)
                assert alive == beta[k][(last[s], last[t])], (k, s, t)


@pytest.mark.parametrize("seed,thr", [(31, ("fraction", 15, 100)), (32, ("full", 0, 1)), (33, ("fraction", 40, 100))])
def test_homology_and_cohomology_give_same_pivots(orc, seed, thr):
    """Section 2.2.2: the anti-transpose yields the same pivot pairs."""
    c = workloads.uniform_cloud(seed, 40, 3, thr=thr)
    f = orc.build(c.points, c.thr)
    a = orc.reduce(f, "homology", clear=False)
    b = orc.reduce(f, "homology", clear=True)
    h = orc.reduce(f, "cohomology")
    for x in (b, h):
        assert np.array_equal(a.e_low, x.e_low)
        assert np.array_equal(a.t_low, x.t_low)


@pytest.mark.parametrize("seed", [41, 42, 43])
def test_h0_deaths_are_kruskal_edges(orc, seed):
    c = workloads.uniform_cloud(seed, 150, 3, thr=("fraction", 5, 100))
    f = orc.build(c.points, c.thr)
    p = orc.reduce(f, "cohomology")
    deaths = np.nonzero(p.e_low >= 0)[0].tolist()
    assert deaths == bf.kruskal_deaths(f.n, list(zip(f.ei.tolist(), f.ej.tolist())))
    assert p.betti()[0] == f.n - len(deaths)


@pytest.mark.parametrize("seed,thr", [(51, ("fraction", 12, 100)), (52, ("fraction", 35, 100)), (53, ("sqdist", 900, 0))])
def test_euler_characteristic(orc, seed, thr):
    """n - K + T = beta0 - beta1 + beta2 (essential classes of the final complex)."""
    c = workloads.uniform_cloud(seed, 90, 2, thr=thr)
    f = orc.build(c.points, c.thr)
    b0, b1, b2 = orc.reduce(f, "cohomology").betti()
    assert f.n - f.K + f.T == b0 - b1 + b2


def test_full_threshold_betti(orc):
    """The 2-skeleton of a full simplex on n vertices: beta = (1, 0, C(n-1,3))."""
    f = orc.build(*_cloud_args(workloads.plain64()))
    assert orc.reduce(f, "cohomology").betti() == (1, 0, math.comb(63, 3))


def test_noisy_circle_has_one_dominant_h1_bar(orc):
    """A noisy circle at the 20th percentile: one essential H1 class, every
    finite H1 bar shorter than a tenth of the kept ranks."""
    c = workloads.noisy_circle(n=400)
    f = orc.build(c.points, c.thr)
    p = orc.reduce(f, "cohomology")
    assert p.betti()[1] == 1
    finite = [d - b for dim, b, d in orc.barcode(f, p) if dim == 1 and d != np.iinfo(np.int64).max]
    assert max(finite, default=0) < f.K // 10


# ---------------------------------------------------------------------------
# Dissimilarity-matrix input (the paper's Section 3: the input may be a
# symmetric distance matrix instead of points; its HIV example uses Hamming
# distances).


def _sq_matrix(points):
    p = points.astype(np.int64)
    return ((p[:, None, :] - p[None, :, :]) ** 2).sum(-1)


@pytest.mark.parametrize("case", [
    (workloads.uniform_cloud(91, 60, 3), ("fraction", 25, 100)),
    (workloads.lattice_cloud(92, 70, side=3, d=2), ("fraction", 40, 100)),  # many ties
    (workloads.uniform_cloud(93, 45, 5), ("sqdist", 20000, 0)),
    (workloads.uniform_cloud(94, 30, 2), ("full", 0, 1)),
])
def test_matrix_input_equals_points_input(orc, case):
    cloud, thr = case
    f = orc.build(cloud.points, thr)
    g = orc.build_matrix(_sq_matrix(cloud.points).astype(np.int32), thr)
    assert f.counts == g.counts
    for a, b in ((f.ei, g.ei), (f.ej, g.ej), (f.eq, g.eq), (f.tris, g.tris), (f.R, g.R)):
        assert np.array_equal(a, b)


def _hypercube_hamming(m):
    x = np.arange(1 << m)
    return np.array([[bin(a ^ b).count("1") for b in x] for a in x], np.int32)


@pytest.mark.parametrize("m", [3, 4, 5])
def test_hypercube_hamming_closed_forms(orc, m):
    n = 1 << m
    M = _hypercube_hamming(m)
    # distance < 2: the hypercube graph, m 2^(m-1) edges and, being
    # bipartite, no triangles
    f = orc.build_matrix(M, ("sqdist", 2, 0))
    assert f.counts == (n, m * (1 << (m - 1)), 0)
    assert set(f.eq.tolist()) == {1}
    # full threshold: every pair and triple
    f = orc.build_matrix(M, ("full", 0, 1))
    assert f.counts == (n, math.comb(n, 2), math.comb(n, 3))
    # distance < 3: each vertex has C(m,1) + C(m,2) neighbours; a triple is a
    # triangle when its three distances are at most 2 (brute force)
    f = orc.build_matrix(M, ("sqdist", 3, 0))
    assert f.K == n * (m + math.comb(m, 2)) // 2
    T = sum(1 for a in range(n) for b in range(a + 1, n) for c in range(b + 1, n)
            if M[a, b] <= 2 and M[a, c] <= 2 and M[b, c] <= 2)
    assert f.T == T


def test_matrix_ties_rank_by_pair_index(orc):
    n, frac = 14, ("fraction", 30, 100)
    M = np.ones((n, n), np.int32)
    f = orc.build_matrix(M, frac)
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    K = len(pairs) * 30 // 100  # the fraction threshold keeps floor(E num / den) edges
    assert f.K == K
    assert list(zip(f.ei.tolist(), f.ej.tolist())) == pairs[:K]
    rank = {p: r for r, p in enumerate(pairs[:K])}
    want = sorted((max(rank[(a, b)], rank[(a, c)], rank[(b, c)]), a, b, c)
                  for a in range(n) for b in range(a + 1, n) for c in range(b + 1, n)
                  if (a, b) in rank and (a, c) in rank and (b, c) in rank)
    assert [tuple(t) for t in f.tris.tolist()] == want


def test_matrix_input_rejects_negative_or_nonsquare(orc):
    with pytest.raises(ValueError):
        orc.build_matrix(-np.ones((5, 5), np.int32), ("full", 0, 1))
    with pytest.raises(ValueError):
        orc.build_matrix(np.ones((5, 4), np.int32), ("full", 0, 1))


# --- per-column ordering (Section 4.3) -------------------------------------

def test_column_order_matches_paper_sortperm_example(orc):
    """One column holding the Section 4.5 example: the slot of each entry is
    the inverse of the printed sortperm (the two are inverse permutations)."""
    rows = dict((r[0], [int(x) for x in r[1:]]) for r in _golden_rows("sortperm_example.txt"))
    perm = [p - 1 for p in rows["sortperm"]]
    inv = [0] * len(perm)
    for slot, e in enumerate(perm):
        inv[e] = slot
    v = rows["v"]
    assert list(orc.column_order([0, len(v)], v)) == inv


@pytest.mark.parametrize("seed", range(8))
def test_column_order_matches_bruteforce(orc, seed):
    """The definition by counting (smaller entries plus earlier equal
    entries), in pure Python, on ragged columns with empties and ties."""
    colptr, v = workloads.csc_columns(seed, ncols=40, mean_len=6, maxvalue=[1, 3, 9, 50][seed % 4])
    a = orc.column_order(colptr, v)
    assert list(a) == bf.column_order(colptr, [int(x) for x in v])


@pytest.mark.parametrize("seed", range(4))
def test_column_order_equals_stable_library_sort(orc, seed):
    """Per column, the inverse of numpy's stable argsort."""
    colptr, v = workloads.csc_columns(100 + seed, ncols=300, mean_len=40, maxvalue=[0, 5, 1000, 2**20][seed],
                                      long_cols=2, long_len=3000)
    z = orc.column_order(colptr, v)
    ref = np.empty_like(z)
    for j in range(len(colptr) - 1):
        a, b = colptr[j], colptr[j + 1]
        ref[a + np.argsort(v[a:b], kind="stable")] = np.arange(a, b)
    assert np.array_equal(z, ref)


def test_column_order_invariants(orc):
    """Each column's slots are a permutation of its own range; placing the
    values by z sorts every column; equal values keep their entry order."""
    colptr, v = workloads.csc_columns(7, ncols=500, mean_len=30, maxvalue=12)
    z = orc.column_order(colptr, v)
    out = np.empty_like(v)
    out[z] = v
    src = np.empty_like(z)
    src[z] = np.arange(len(z))
    for j in range(len(colptr) - 1):
        a, b = colptr[j], colptr[j + 1]
        assert np.array_equal(np.sort(z[a:b]), np.arange(a, b))
        assert np.all(np.diff(out[a:b]) >= 0)
        same = np.diff(out[a:b]) == 0
        assert np.all(np.diff(src[a:b])[same] > 0)


def test_column_order_special_cases(orc):
    """Empty array, empty columns only, one entry, constant columns (identity),
    and columns already sorted (identity) or strictly descending (reversal)."""
    assert len(orc.column_order([0, 0, 0], [])) == 0
    assert list(orc.column_order([0, 1], [5])) == [0]
    assert list(orc.column_order([0, 0, 4, 4], [3, 3, 3, 3])) == [0, 1, 2, 3]
    assert list(orc.column_order([0, 3, 6], [1, 2, 3, 9, 8, 7])) == [0, 1, 2, 5, 4, 3]
    assert list(orc.column_order([0, 4], [-5, 2**31 - 1, -2**31, 0])) == [1, 3, 0, 2]
    with pytest.raises(ValueError):
        orc.column_order([0, 3], [1, 2])


def test_reductions_without_triangles(orc):
    """Up to dimension 1 the complex is a graph: both reductions pair the
    spanning-forest edges with vertices and leave every other edge unpaired."""
    c = workloads.noisy_circle(seed=30, n=150)
    f1 = orc.build(c.points, c.thr, maxdim=1)
    f2 = orc.build(c.points, c.thr)
    for m in ("homology", "cohomology"):
        p1, p2 = orc.reduce(f1, m), orc.reduce(f2, m)
        assert np.array_equal(p1.e_low, p2.e_low)
        assert len(p1.t_low) == 0


@pytest.mark.parametrize("seed", range(4))
def test_dim0_pairs_follow_elder_rule(orc, seed):
    """With vertices ordered by index, the column reduction pairs edge r with
    the younger of the two components it joins, named by its smallest vertex
    (a union-find that keeps each component's smallest vertex as its root)."""
    c = workloads.noisy_circle(seed=50 + seed, n=120)
    f = orc.build(c.points, [("fraction", 8, 100), ("count", 90, 1), ("full", 0, 1), ("sqdist", 300, 0)][seed])
    root = list(range(f.n))

    def find(x):
        while root[x] != x:
            x = root[x]
        return x

    want = np.full(f.K, -1)
    for r, (a, b) in enumerate(zip(f.ei, f.ej)):
        ra, rb = find(a), find(b)
        if ra != rb:
            want[r] = max(ra, rb)
            root[max(ra, rb)] = min(ra, rb)
    for m in ("homology", "cohomology"):
        assert np.array_equal(orc.reduce(f, m).e_low, want)


# --- F2 sparse product and sum (Section 4.6) --------------------------------

def _f2(seed, m, n, L, dup=0.2):
    return workloads.f2_csc(seed, m, n, L, dup=dup)


@pytest.mark.parametrize("seed", range(5))
def test_blockprodsum_dense_equals_columnwise_and_scipy(orc, seed):
    import scipy.sparse as sp

    m, k, n = [(30, 20, 25), (64, 64, 64), (97, 13, 40), (5, 50, 7), (200, 150, 120)][seed]
    C, E, D = _f2(seed, m, k, 3), _f2(seed + 10, k, n, 2), _f2(seed + 20, m, n, 2)
    cp, rw = orc.blockprodsum(m, C, E, D)
    for j in range(n):
        assert np.array_equal(rw[cp[j]:cp[j + 1]], orc.blockprodsum_column(m, C, E, D, j))

    def mat(x, rows):
        c, r = x
        return sp.csc_matrix((np.ones(len(r), np.int64), r.astype(np.int64), c), shape=(rows, len(c) - 1))

    S = (mat(D, m) + mat(C, m) @ mat(E, k)).toarray() % 2
    cps, rws = orc._csc_of_dense(S)
    assert np.array_equal(cp, cps) and np.array_equal(rw, rws)


def test_blockprodsum_special_cases(orc):
    m, n = 40, 30
    C, D = _f2(1, m, n, 4, dup=0), _f2(2, m, n, 3, dup=0)
    eye = (np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32))
    zero = (np.zeros(n + 1, np.int64), np.zeros(0, np.int32))
    # E = I: S = D + C
    cp, rw = orc.blockprodsum(m, C, eye, D)
    want = (orc._dense_f2(D[0], D[1].astype(np.int64), m) + orc._dense_f2(C[0], C[1].astype(np.int64), m)) % 2
    assert np.array_equal(orc._dense_f2(cp, rw, m), want)
    # E = 0: S = D;  D = 0 and C = I: S = E
    cp, rw = orc.blockprodsum(m, C, zero, D)
    assert np.array_equal(orc._dense_f2(cp, rw, m), orc._dense_f2(D[0], D[1].astype(np.int64), m))
    E = _f2(3, n, 25, 3)
    cp, rw = orc.blockprodsum(n, eye, E, (np.zeros(26, np.int64), np.zeros(0, np.int32)))
    assert np.array_equal(orc._dense_f2(cp, rw, n), orc._dense_f2(E[0], E[1].astype(np.int64), n))


def test_blockprodsum_is_linear(orc):
    """S(C, E1 + E2, D1 + D2) = S(C, E1, D1) + S(C, E2, D2) over F2."""
    m, k, n = 50, 40, 30
    C = _f2(4, m, k, 5)
    E1, E2, D1, D2 = _f2(5, k, n, 3), _f2(6, k, n, 3), _f2(7, m, n, 2), _f2(8, m, n, 2)

    def add(A, B, rows):
        return orc._csc_of_dense((orc._dense_f2(A[0], np.asarray(A[1], np.int64), rows)
                                  + orc._dense_f2(B[0], np.asarray(B[1], np.int64), rows)) % 2)

    lhs = orc.blockprodsum(m, C, add(E1, E2, k), add(D1, D2, m))
    s1, s2 = orc.blockprodsum(m, C, E1, D1), orc.blockprodsum(m, C, E2, D2)
    rhs = add(s1, s2, m)
    assert np.array_equal(lhs[0], rhs[0]) and np.array_equal(lhs[1], rhs[1])


@pytest.mark.parametrize("workers", [1, 2, 3, 4, 7])
def test_blockprodsum_by_workers_equals_whole(orc, workers):
    """The paper's partition by columns, with the column pointers shifted
    block after block, gives the whole product."""
    m, k, n = 60, 45, 33
    C, E, D = _f2(9, m, k, 4), _f2(10, k, n, 3), _f2(11, m, n, 2)
    a = orc.blockprodsum(m, C, E, D)
    b = orc.blockprodsum_by_workers(m, C, E, D, workers)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("case", range(4))
def test_apparent_pairs_are_persistence_pairs(orc, case):
    """The first triangle of each value (the oldest cofacet of that value's
    edge, which is the triangle's youngest facet) is always paired with that
    edge by the column algorithm, in both reductions."""
    c, thr = [(workloads.noisy_circle(seed=80, n=200), ("fraction", 20, 100)),
              (workloads.lattice_cloud(4, 60, side=3), ("fraction", 40, 100)),
              (workloads.plain64(), ("full", 0, 1)),
              (workloads.uniform_cloud(6, 100, 3), ("sqdist", 4000, 0))][case]
    f = orc.build(c.points, thr)
    v = f.tris[:, 0]
    first = np.nonzero(np.r_[True, v[1:] != v[:-1]])[0] if f.T else np.zeros(0, np.int64)
    for m in ("homology", "cohomology"):
        t_low = orc.reduce(f, m).t_low
        assert np.array_equal(t_low[first], v[first])


# --- tetrahedra counts (dimension 3) ----------------------------------------

@pytest.mark.parametrize("case", range(len(CASES)), ids=[c.name for c in CASES])
def test_tetra_counts_match_bruteforce(orc, case):
    c = CASES[case]
    f = orc.build(c.points, c.thr, list_triangles=False)
    assert list(orc.tetra_counts(f)) == bf.tetra_counts(c.points, _K_of(c.thr))


@pytest.mark.parametrize("n", [4, 5, 17, 40])
def test_tetra_counts_full_threshold_closed_form(orc, n):
    """Every 4-subset is a tetrahedron, counted at its largest edge once."""
    c = workloads.uniform_cloud(20 + n, n, 3)
    f = orc.build(c.points, ("full", 0, 1), list_triangles=False)
    assert int(orc.tetra_counts(f).sum()) == math.comb(n, 4)


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c.name for c in CASES])
def test_tetra_list_matches_bruteforce(orc, case):
    """The listed tetrahedra are exactly the 4-subsets with six kept edges,
    valued at their largest edge, in (value, vertices) order."""
    import itertools

    c = CASES[case]
    f = orc.build(c.points, c.thr, list_triangles=False)
    got = orc.tetra_list(f)
    kept, rank, _, _ = bf.filtration(c.points, _K_of(c.thr))
    want = []
    for quad in itertools.combinations(range(len(c.points)), 4):
        rs = [rank.get(e) for e in itertools.combinations(quad, 2)]
        if all(x is not None for x in rs):
            want.append((max(rs),) + quad)
    assert [tuple(r) for r in got] == sorted(want)
    assert np.array_equal(np.bincount(got[:, 0], minlength=f.K)[: f.K] if len(got) else np.zeros(f.K, int),
                          orc.tetra_counts(f))


# --- the oracle on several host threads ------------------------------------

@pytest.mark.parametrize("case", [
    workloads.noisy_circle(seed=61, n=300),
    workloads.lattice_cloud(62, 90, side=4, thr=("fraction", 30, 100)),  # ties
    workloads.uniform_cloud(63, 70, 4, thr=("full", 0, 1)),
    workloads.uniform_cloud(64, 120, 16, thr=("sqdist", 60000, 0)),
    workloads.uniform_cloud(65, 3, 2, thr=("full", 0, 1)),
    workloads.uniform_cloud(66, 2, 2, thr=("full", 0, 1)),
], ids=lambda c: c.name)
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_threaded_build_equals_plain_build(orc, case, threads):
    """Distances split by rows and triangles split by values give exactly
    the single-threaded triple loop's sorted list, whatever the thread count."""
    f = orc.build(case.points, case.thr)
    g = orc.build_mt(case.points, case.thr, threads)
    assert np.array_equal(f.q, g.q)
    assert (f.K, f.T) == (g.K, g.T)
    assert np.array_equal(f.tris.reshape(-1, 4), g.tris.reshape(-1, 4))


def test_triangles_by_value_ranges_concatenate(orc):
    """Listing values [0, a), [a, b), [b, K) separately and concatenating
    gives the whole list; an empty range gives nothing."""
    c = workloads.noisy_circle(seed=67, n=250)
    f = orc.build(c.points, c.thr)
    a, b = f.K // 3, 2 * f.K // 3
    parts = [orc.triangles_by_value(f, 0, a, 2), orc.triangles_by_value(f, a, b, 5),
             orc.triangles_by_value(f, b, f.K, 1)]
    assert np.array_equal(np.concatenate(parts), f.tris)
    assert len(orc.triangles_by_value(f, a, a, 4)) == 0
    assert all((p[:, 0] >= lo).all() and (p[:, 0] < hi).all() for p, lo, hi in zip(parts, (0, a, b), (a, b, f.K)))
    with pytest.raises(ValueError):
        orc.triangles_by_value(f, 0, f.K + 1)


# --- pairs of dimension 2 (triangles with tetrahedra) ------------------------

def _pairs3_in_total_order(f, p, tets):
    """(birth, death) pairs of dimensions 0..2 and essential births of
    dimensions 0..3 as total-order indices, tetrahedra included."""
    order = bf.total_order(f.n, list(zip(f.ei.tolist(), f.ej.tolist())), [tuple(t) for t in f.tris.tolist()],
                           [tuple(q) for q in tets.tolist()])
    pos = {s: i for i, s in enumerate(order)}
    vid = lambda v: pos[("v", (v,))]
    eid = lambda r: pos[("e", (int(f.ei[r]), int(f.ej[r])))]
    tid = lambda t: pos[("t", tuple(int(x) for x in f.tris[t, 1:]))]
    qid = lambda s: pos[("q", tuple(int(x) for x in tets[s, 1:]))]
    pairs = {0: [], 1: [], 2: []}
    for r in np.nonzero(p.e_low >= 0)[0]:
        pairs[0].append((vid(int(p.e_low[r])), eid(r)))
    for t in np.nonzero(p.t_low >= 0)[0]:
        pairs[1].append((eid(int(p.t_low[t])), tid(t)))
    for s in np.nonzero(p.q_low >= 0)[0]:
        pairs[2].append((tid(int(p.q_low[s])), qid(s)))
    e0, e1, e2, e3 = p.essential()
    ess = {0: [vid(v) for v in e0], 1: [eid(r) for r in e1], 2: [tid(t) for t in e2], 3: [qid(s) for s in e3]}
    return len(order), pairs, ess


DIM2_TINY = [
    workloads.uniform_cloud(121, 6, 3, thr=("full", 0, 1)),
    workloads.uniform_cloud(122, 7, 3, thr=("fraction", 75, 100)),
    workloads.lattice_cloud(123, 7, side=3, thr=("fraction", 65, 100)),
    workloads.uniform_cloud(124, 7, 2, thr=("count", 16, 1)),
]


@pytest.mark.parametrize("case", DIM2_TINY, ids=lambda c: c.name)
@pytest.mark.parametrize("method", ["homology", "cohomology"])
def test_dim2_pairs_match_bruteforce_persistent_betti(orc, case, method):
    """With the tetrahedra, the pairs of every dimension reproduce every
    persistent Betti number rank(H_k(X_s) -> H_k(X_t)), k = 0..3, brute
    force from F2 ranks of the boundary matrices."""
    f = orc.build(case.points, case.thr)
    tets = orc.tetra_list(f)
    assert len(tets) > 0
    p = orc.with_dim2(f, orc.reduce(f, method), tets, method)
    N, pairs, ess = _pairs3_in_total_order(f, p, tets)
    _, beta = bf.persistent_betti(f.n, list(zip(f.ei.tolist(), f.ej.tolist())), [tuple(t) for t in f.tris.tolist()],
                                  [tuple(q) for q in tets.tolist()])
    got = bf.betti_from_pairs(N, pairs, ess, dims=(0, 1, 2, 3))
    for k in (0, 1, 2, 3):
        assert got[k] == beta[k], f"dimension {k}"


@pytest.mark.parametrize("seed,n,thr", [(131, 30, ("fraction", 30, 100)), (132, 24, ("full", 0, 1)),
                                        (133, 40, ("fraction", 15, 100)), (134, 36, ("sqdist", 2500, 0))])
def test_dim2_homology_and_cohomology_give_same_pairs(orc, seed, n, thr):
    """Section 2.2.2 one dimension up: the tetrahedra's boundary block and
    the triangles' coboundaries with clearing pair the same simplices."""
    c = workloads.uniform_cloud(seed, n, 3, thr=thr)
    f = orc.build(c.points, c.thr)
    tets = orc.tetra_list(f)
    h = orc.reduce_dim2(f, tets, "homology")
    co = orc.reduce_dim2(f, tets, "cohomology", orc.reduce(f, "cohomology").t_low)
    assert np.array_equal(h, co)
    # a triangle pairs at most once, never with an older tetrahedron (its
    # column's low is a row above the column), and a triangle paired with an
    # edge is never paired with a tetrahedron
    paired = h[h >= 0]
    assert len(set(paired.tolist())) == len(paired)
    assert all(f.tris[h[s], 0] <= tets[s, 0] for s in np.nonzero(h >= 0)[0])
    t_low = orc.reduce(f, "homology").t_low
    assert not np.any(t_low[paired] >= 0)


@pytest.mark.parametrize("seed,thr", [(141, ("fraction", 12, 100)), (142, ("fraction", 35, 100)),
                                      (143, ("sqdist", 900, 0))])
def test_euler_characteristic_dim3(orc, seed, thr):
    """n - K + T - T3 = beta0 - beta1 + beta2 - beta3 of the 3-skeleton."""
    c = workloads.uniform_cloud(seed, 45, 2, thr=thr)
    f = orc.build(c.points, c.thr)
    tets = orc.tetra_list(f)
    b = orc.with_dim2(f, orc.reduce(f, "cohomology"), tets).betti()
    assert f.n - f.K + f.T - len(tets) == b[0] - b[1] + b[2] - b[3]


@pytest.mark.parametrize("n", [5, 9, 14])
def test_full_simplex_dim3_betti(orc, n):
    """The 3-skeleton of a full simplex on n vertices: beta = (1, 0, 0,
    C(n-1, 4)) (it is 2-connected; its cycles of dimension 3 are the
    boundaries of the C(n-1, 4) 4-simplices through one vertex)."""
    c = workloads.uniform_cloud(150 + n, n, 3)
    f = orc.build(c.points, ("full", 0, 1))
    tets = orc.tetra_list(f)
    assert len(tets) == math.comb(n, 4)
    assert orc.with_dim2(f, orc.reduce(f, "cohomology"), tets).betti() == (1, 0, 0, math.comb(n - 1, 4))


@pytest.mark.parametrize("case", DIM2_TINY[1:], ids=lambda c: c.name)
def test_dim2_barcode_reproduces_persistent_betti_by_value(orc, case):
    """The barcode with the tetrahedra, in filtration values: for every pair
    of values s <= t the bars of dimension k (k = 0..3) with birth <= s and
    death > t number rank(H_k(X_s) -> H_k(X_t)), X_s the simplices of value
    <= s; no bar is born after it dies."""
    f = orc.build(case.points, case.thr)
    tets = orc.tetra_list(f)
    bars = orc.barcode(f, orc.with_dim2(f, orc.reduce(f, "cohomology"), tets), tets)
    assert all(b < d for _, b, d in bars)
    kept = list(zip(f.ei.tolist(), f.ej.tolist()))
    tris = [tuple(t) for t in f.tris.tolist()]
    order, beta = bf.persistent_betti(f.n, kept, tris, [tuple(q) for q in tets.tolist()])
    value_of = {("e", e): r for r, e in enumerate(kept)}
    value_of.update({("t", tuple(t[1:])): t[0] for t in tris})
    value_of.update({("q", tuple(q[1:])): q[0] for q in tets.tolist()})
    last = {-1: f.n - 1}
    for p_, (kind, verts) in enumerate(order):
        if kind != "v":
            last[value_of[(kind, verts)]] = p_
    for k in (0, 1, 2, 3):
        for s in sorted(last):
            for t in sorted(last):
                if t >= s:
                    alive = sum(1 for dim, b, d in bars if dim == k and b <= s and d > t)
                    assert alive == beta[k][(last[s], last[t])], (k, s, t)
