"""All persistence pairs of dimension 1 (vr_pairs_dim1) and the barcode
(vr_barcode) on the device against the oracle's column reduction,
bit-exact; at the 4000-point mixture, against properties that hold at any
size (the Euler characteristic, the H0 pairs, the order of the pairs)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

INF = np.iinfo(np.int64).max


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1809_04424_amd as vr

    vr.lib()
    yield


def _device_pairs(r):
    import torch

    import paper_1809_04424_amd as vr

    e_low, _ = vr.pairs_dim0(r)
    toe = vr.pairs_dim1(r, e_low)
    bars, ess2 = vr.barcode(r, e_low, toe)
    torch.cuda.synchronize()
    return (e_low.cpu().numpy().astype(np.int64), toe.cpu().numpy().astype(np.int64),
            bars.cpu().numpy(), ess2)


def _oracle_tri_of_edge(p, K):
    want = np.full(K, -1, np.int64)
    for t in np.nonzero(p.t_low >= 0)[0]:
        want[p.t_low[t]] = t
    return want


def _check(orc, points, thr, label, maxdim=2):
    import torch

    import paper_1809_04424_amd as vr

    print(f"[gpu] pairs_dim1 {label} n={len(points)} thr={thr}", flush=True)
    f = orc.build(points, thr, maxdim=maxdim)
    p = orc.reduce(f, "cohomology")
    r = vr.build(torch.from_numpy(np.ascontiguousarray(points)).to("cuda:0"), thr, maxdim=maxdim)
    e_low, toe, bars, ess2 = _device_pairs(r)
    r.free()
    assert np.array_equal(e_low, p.e_low)
    assert np.array_equal(toe, _oracle_tri_of_edge(p, f.K))
    # the barcode, dimensions 0 and 1 listed, dimension 2 counted
    want = orc.barcode(f, p)
    got = sorted(tuple(int(x) for x in b) for b in bars) + [(2, None, INF)] * ess2
    assert sorted((d, b, e) for d, b, e in want if d < 2) == got[: len(got) - ess2]
    assert sum(1 for d, _, _ in want if d == 2) == ess2
    return f, p


CASES = [
    ("circle150_p10", lambda: workloads.noisy_circle(seed=40, n=150).points, ("fraction", 10, 100)),
    ("circle300_sparse", lambda: workloads.noisy_circle(seed=41, n=300).points, ("count", 250, 1)),
    ("lattice_ties", lambda: workloads.lattice_cloud(3, 90, side=3).points, ("fraction", 30, 100)),
    ("uniform_d16", lambda: workloads.uniform_cloud(42, 260, 16).points, ("fraction", 5, 100)),
    ("plain64_full", lambda: workloads.plain64().points, ("full", 0, 1)),
    ("n65", lambda: workloads.uniform_cloud(43, 65, 3).points, ("fraction", 50, 100)),
    ("n128_sqdist", lambda: workloads.uniform_cloud(44, 128, 2).points, ("sqdist", 900, 0)),
    ("uniform_d3_p30", lambda: workloads.uniform_cloud(48, 200, 3).points, ("fraction", 30, 100)),
    ("torus300", lambda: workloads.batched(seed=4, clouds=3, nmin=300, nmax=300)[2].points,
     ("fraction", 12, 100)),
    ("mixture_d64_600", lambda: workloads.mixture(seed=49, n=600).points, ("fraction", 10, 100)),
    # an edge column with 4202 cofacets, more than the 4096 a work-group's
    # LDS holds: reduced from a base in device memory
    ("hub_cycle_m4200", lambda: workloads.hub_cycle(), ("sqdist", 6000, 0)),
    ("hub_cycle_m4200_denser", lambda: workloads.hub_cycle(), ("sqdist", 6500, 0)),
    # the largest point count: every vertex's edge lists built from rows of
    # 8192 ranks (eight per thread)
    ("n8192_sparse", lambda: workloads.uniform_cloud(77, 8192, 2, dtype=np.int32, lo=0, hi=6000).points,
     ("count", 200000, 1)),
]


@pytest.mark.parametrize("name,gen,thr", CASES, ids=[c[0] for c in CASES])
def test_pairs_dim1_and_barcode(orc, name, gen, thr):
    _check(orc, gen(), thr, name)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_pairs_dim1_tiny(orc, n):
    pts = np.array([[0, 0], [3, 0], [0, 4], [5, 5]][:n], np.int32)
    _check(orc, pts, ("full", 0, 1), f"tiny{n}")


def test_pairs_dim1_without_triangles(orc):
    """Built up to dimension 1: no triangle, so no edge dies."""
    f, p = _check(orc, workloads.noisy_circle(seed=50, n=200).points, ("fraction", 20, 100), "maxdim1", maxdim=1)
    assert f.T == 0


def test_noisy_circle_one_class(orc):
    """circle1000 at its 20th-percentile threshold: the oracle's pairs, and
    exactly one class of dimension 1 that never dies."""
    f, p = _check(orc, workloads.noisy_circle().points, ("fraction", 20, 100), "circle1000")
    assert p.betti()[1] == 1


def test_pairs_dim1_of_batch_items(orc):
    import torch

    import paper_1809_04424_amd as vr

    clouds = [workloads.noisy_circle(seed=70 + i, n=n).points for i, n in enumerate((40, 150, 3, 260))]
    thr = ("fraction", 15, 100)
    b = vr.build_batch([torch.from_numpy(p).to("cuda:0") for p in clouds], thr)
    for pts, item in zip(clouds, b):
        print(f"[gpu] pairs_dim1 batch item n={len(pts)}", flush=True)
        e_low, toe, bars, ess2 = _device_pairs(item)
        f = orc.build(pts, thr)
        p = orc.reduce(f, "cohomology")
        assert np.array_equal(e_low, p.e_low)
        assert np.array_equal(toe, _oracle_tri_of_edge(p, f.K))
    b.free()


@pytest.mark.parametrize("n,thr", [(120, ("fraction", 20, 100)), (300, ("fraction", 6, 100))])
def test_pairs_dim1_of_a_matrix_build(orc, n, thr):
    """The pairs and barcode of a build from a Hamming dissimilarity matrix
    (ties everywhere: the edge order falls back to (i, j)) equal the
    oracle's."""
    import torch

    import paper_1809_04424_amd as vr

    M = workloads.hamming_matrix(90 + n, n)
    print(f"[gpu] pairs_dim1 hamming matrix n={n} thr={thr}", flush=True)
    r = vr.build_matrix(torch.from_numpy(M).to("cuda:0"), thr)
    e_low, toe, bars, ess2 = _device_pairs(r)
    f = orc.build_matrix(M, thr)
    p = orc.reduce(f, "cohomology")
    assert np.array_equal(e_low, p.e_low)
    assert np.array_equal(toe, _oracle_tri_of_edge(p, f.K))
    want = orc.barcode(f, p)
    assert sorted(tuple(int(x) for x in b) for b in bars) == sorted(b for b in want if b[0] < 2)
    assert ess2 == sum(1 for b in want if b[0] == 2)
    r.free()


def test_mixture4000_reduction_properties(orc):
    """The 4000-point mixture (94 million triangles, beyond the oracle's
    reduction): H0 pairs equal the oracle's spanning-forest edges, every
    dimension-1 pair joins an edge to a cofacet of no smaller value with
    each triangle used once, apparent pairs are the first triangle of each
    value, and the Euler characteristic n - K + T equals the alternating sum
    of the classes that never die."""
    import torch

    import paper_1809_04424_amd as vr

    c = workloads.mixture()
    print("[gpu] pairs_dim1 mixture4000", flush=True)
    f = orc.build_mt(c.points, c.thr, 16, list_triangles=False)
    r = vr.build(torch.from_numpy(c.points).to("cuda:0"), c.thr)
    e_low, toe, bars, ess2 = _device_pairs(r)
    keys = r.tri_key().cpu().numpy().view(np.uint64)
    ij = r.edge_ij().cpu().numpy().astype(np.int64)
    n, K, T = r.counts
    r.free()
    # dimension 0: Kruskal's forest (union-find over the edges in rank order)
    parent = np.arange(n)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    forest = np.zeros(K, bool)
    for e in range(K):
        a, b = find(ij[e, 0]), find(ij[e, 1])
        if a != b:
            parent[max(a, b)] = min(a, b)
            forest[e] = True
    assert np.array_equal(e_low >= 0, forest)
    # dimension 1: no forest edge is paired with a triangle, each triangle is
    # paired at most once, and never with an edge younger than itself (the
    # pivot of a reduced column comes from a sum of coboundaries, so it need
    # not contain the edge)
    paired = np.nonzero(toe >= 0)[0]
    assert not np.any(forest[paired])
    t = toe[paired]
    assert len(np.unique(t)) == len(t)
    v = (keys[t] >> np.uint64(39)).astype(np.int64)
    assert np.all(v >= paired)
    # apparent pairs: edges with triangles of their own value take the first
    # of them, which contains the edge
    vals = (keys >> np.uint64(39)).astype(np.int64)
    first = np.nonzero(np.r_[True, vals[1:] != vals[:-1]])[0]
    assert np.array_equal(toe[vals[first]], first)
    kt = keys[first]
    x = np.stack([(kt >> np.uint64(26)) & np.uint64(0x1FFF), (kt >> np.uint64(13)) & np.uint64(0x1FFF),
                  kt & np.uint64(0x1FFF)], 1).astype(np.int64)
    a, b = ij[vals[first], 0], ij[vals[first], 1]
    assert np.all(((x == a[:, None]).sum(1) == 1) & ((x == b[:, None]).sum(1) == 1))
    assert np.all(v[np.isin(paired, vals[first], invert=True)] > paired[np.isin(paired, vals[first], invert=True)])
    # Euler characteristic
    b0 = int(np.sum(bars[:n, 2] == INF))
    dim1 = bars[n:]
    b1 = int(np.sum(dim1[:, 2] == INF))
    assert n - K + T == b0 - b1 + ess2
    assert T == f.T and K == f.K
    print(f"[gpu] mixture4000: {len(paired)} pairs of dimension 1, {len(paired) - len(first)} not apparent, "
          f"betti {b0} {b1} {ess2}", flush=True)
