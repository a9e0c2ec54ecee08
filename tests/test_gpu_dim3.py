"""Dimension 3 in the build (maxdim 3: the tetrahedra listed into the
result) and the persistence pairs of dimension 2 (vr_pairs_dim2: triangles
with tetrahedra) on the device, bit-exact against the oracle's tetrahedra
and its reduction of the triangles' coboundaries; at the 1000-point noisy
circle (167 million tetrahedra), against properties that hold at any size
(the Euler characteristic of the 3-skeleton, pairs unique and never
backwards)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1809_04424_amd as vr

    vr.lib()
    yield


def _tet_rows_as_keys(rows):
    """Oracle rows (value, a, b, c, d) as the library's two-word keys."""
    rows = np.asarray(rows, np.int64).reshape(-1, 5)
    vk = (rows[:, 1] << 39) | (rows[:, 2] << 26) | (rows[:, 3] << 13) | rows[:, 4]
    return np.stack([rows[:, 0], vk], axis=1)


def _device(points, thr, count_only=False, allocator="library"):
    import torch

    import paper_1809_04424_amd as vr

    return vr.build(torch.from_numpy(np.ascontiguousarray(points)).to("cuda:0"), thr, maxdim=3,
                    count_only=count_only, allocator=allocator)


CASES = [
    ("full40", lambda: workloads.uniform_cloud(201, 40, 3).points, ("full", 0, 1)),
    ("sphere120_p15", lambda: workloads.sphere_cloud(202, 120).points, ("fraction", 15, 100)),
    ("sphere200_p10", lambda: workloads.sphere_cloud(203, 200).points, ("fraction", 10, 100)),
    ("circle150_p20", lambda: workloads.noisy_circle(seed=204, n=150).points, ("fraction", 20, 100)),
    ("lattice_ties", lambda: workloads.lattice_cloud(205, 80, side=3).points, ("fraction", 25, 100)),
    ("uniform_d16_h2", lambda: workloads.uniform_cloud(206, 120, 16).points, ("fraction", 15, 100)),
    ("torus250", lambda: workloads.batched(seed=4, clouds=3, nmin=250, nmax=250)[2].points, ("fraction", 8, 100)),
    ("circle300_p25", lambda: workloads.noisy_circle(seed=207, n=300).points, ("fraction", 25, 100)),
    ("mixture_d64_300", lambda: workloads.mixture(seed=208, n=300).points, ("fraction", 12, 100)),
]


@pytest.mark.parametrize("name,gen,thr", CASES, ids=[c[0] for c in CASES])
def test_maxdim3_build_and_dim2_pairs(orc, name, gen, thr):
    import torch

    import paper_1809_04424_amd as vr

    pts = gen()
    print(f"[gpu] dim3 {name} n={len(pts)} thr={thr}", flush=True)
    f = orc.build(pts, thr)
    tets = orc.tetra_list(f)
    r = _device(pts, thr)
    assert r.counts == f.counts and r.T3 == len(tets)
    want_off = np.zeros(f.K + 1, np.int64)
    np.cumsum(np.bincount(tets[:, 0], minlength=f.K)[: f.K] if len(tets) else np.zeros(f.K, np.int64),
              out=want_off[1:])
    assert np.array_equal(r.tet_off().cpu().numpy(), want_off)
    assert np.array_equal(r.tet_key().cpu().numpy(), _tet_rows_as_keys(tets))
    # the pairs, dimensions 1 and 2
    e_low, _ = vr.pairs_dim0(r)
    toe = vr.pairs_dim1(r, e_low)
    tt = vr.pairs_dim2(r, toe)
    torch.cuda.synchronize()
    got = tt.cpu().numpy()
    p1 = orc.reduce(f, "cohomology")
    q_low = orc.reduce_dim2(f, tets, "cohomology", p1.t_low)
    want = np.full(f.T, -1, np.int64)
    want[q_low[q_low >= 0]] = np.nonzero(q_low >= 0)[0]
    assert np.array_equal(got, want)
    # the barcode of dimension 2 and the classes of dimension 3
    bars, ess3 = vr.barcode_dim2(r, toe, tt)
    wb = orc.barcode(f, orc.with_dim2(f, p1, tets), tets)
    assert sorted(tuple(int(x) for x in b) for b in bars.cpu().numpy()) == sorted(b for b in wb if b[0] == 2)
    assert ess3 == sum(1 for b in wb if b[0] == 3)
    r.free()


def test_maxdim3_matrix_build_and_dim2_pairs(orc):
    """A maxdim-3 build from a Hamming dissimilarity matrix (ties broken by
    index throughout): the tetrahedra and the pairs and barcode of
    dimension 2 equal the oracle's."""
    import torch

    import paper_1809_04424_amd as vr

    M = workloads.hamming_matrix(211, 90)
    thr = ("fraction", 12, 100)
    print("[gpu] maxdim-3 matrix build n=90", flush=True)
    r = vr.build_matrix(torch.from_numpy(M).to("cuda:0"), thr, maxdim=3)
    f = orc.build_matrix(M, thr)
    tets = orc.tetra_list(f)
    assert r.counts == f.counts and r.T3 == len(tets)
    assert np.array_equal(r.tet_key().cpu().numpy(), _tet_rows_as_keys(tets))
    e_low, _ = vr.pairs_dim0(r)
    toe = vr.pairs_dim1(r, e_low)
    tt = vr.pairs_dim2(r, toe)
    bars, ess3 = vr.barcode_dim2(r, toe, tt)
    torch.cuda.synchronize()
    p1 = orc.reduce(f, "cohomology")
    q_low = orc.reduce_dim2(f, tets, "cohomology", p1.t_low)
    want = np.full(f.T, -1, np.int64)
    want[q_low[q_low >= 0]] = np.nonzero(q_low >= 0)[0]
    assert np.array_equal(tt.cpu().numpy(), want)
    wb = orc.barcode(f, orc.with_dim2(f, p1, tets), tets)
    assert sorted(tuple(int(x) for x in b) for b in bars.cpu().numpy()) == sorted(b for b in wb if b[0] == 2)
    assert ess3 == sum(1 for b in wb if b[0] == 3)
    r.free()


def test_maxdim3_count_only_and_torch_allocator(orc):
    """Count-only lists no tetrahedra but still gives their offsets; the
    torch allocator's blocks hold the same arrays as the library's cache."""
    c = workloads.noisy_circle(seed=209, n=120)
    f = orc.build(c.points, ("fraction", 20, 100))
    tets = orc.tetra_list(f)
    r = _device(c.points, ("fraction", 20, 100), count_only=True)
    assert r.T3 == len(tets) and r.tet_key().numel() == 0
    off = r.tet_off().cpu().numpy()
    assert off[-1] == len(tets) and np.array_equal(np.diff(off), np.bincount(tets[:, 0], minlength=f.K)[: f.K])
    r.free()
    r = _device(c.points, ("fraction", 20, 100), allocator="torch")
    assert np.array_equal(r.tet_key().cpu().numpy(), _tet_rows_as_keys(tets))
    r.free()


def test_maxdim3_small_and_empty(orc):
    """Fewer than four points, or no tetrahedron: T3 = 0, offsets all 0,
    and the dimension-2 pairs are all -1."""
    import paper_1809_04424_amd as vr

    for n, thr in ((3, ("full", 0, 1)), (2, ("full", 0, 1)), (30, ("count", 12, 1))):
        c = workloads.uniform_cloud(210 + n, n, 2)
        f = orc.build(c.points, thr)
        r = _device(c.points, thr)
        assert r.T3 == 0 and r.counts == f.counts
        assert np.array_equal(r.tet_off().cpu().numpy(), np.zeros(f.K + 1, np.int64))
        if f.T:
            e_low, _ = vr.pairs_dim0(r)
            tt = vr.pairs_dim2(r, vr.pairs_dim1(r, e_low)).cpu().numpy()
            assert np.all(tt == -1)
        r.free()


def _oldest_cofacet(R, v, tri):
    """By definition: the earliest tetrahedron holding triangle tri (value
    v): the least (value, sorted vertices) over the vertices l joined to all
    three; None when there is none."""
    i, j, k = tri
    ok = (R[i] >= 0) & (R[j] >= 0) & (R[k] >= 0)
    ok[[i, j, k]] = False
    ls = np.nonzero(ok)[0]
    if len(ls) == 0:
        return None
    w = np.maximum(np.maximum(R[i, ls], R[j, ls]), np.maximum(R[k, ls], v))
    return min((int(w[x]),) + tuple(sorted((i, j, k, int(ls[x])))) for x in range(len(ls)))


def _youngest_facet(R, tet):
    """By definition: the latest of the four triangles of tet."""
    _, a, b, c, d = tet
    facets = []
    for f in ((a, b, c), (a, b, d), (a, c, d), (b, c, d)):
        facets.append((max(R[f[0], f[1]], R[f[0], f[2]], R[f[1], f[2]]),) + f)
    return max(facets)


def test_circle1000_dim2_properties(orc):
    """The 20th-percentile noisy circle with its 167 million tetrahedra:
    every triangle pairs with at most one tetrahedron and each tetrahedron
    with at most one triangle, never an older one, and no triangle paired
    with an edge pairs again; on 3000 sampled triangles, checked by
    definition (oldest cofacet, youngest facet, from the kept edges): a
    triangle whose oldest cofacet has it as its youngest facet is paired
    with exactly that tetrahedron."""
    import torch

    import paper_1809_04424_amd as vr

    c = workloads.noisy_circle()
    print("[gpu] dim3 circle1000 build", flush=True)
    r = _device(c.points, c.thr)
    n, K, T = r.counts
    assert r.T3 == 166675675
    e_low, _ = vr.pairs_dim0(r)
    toe = vr.pairs_dim1(r, e_low)
    print("[gpu] dim3 circle1000 pairs_dim2", flush=True)
    tt = vr.pairs_dim2(r, toe)
    torch.cuda.synchronize()
    tt_h = tt.cpu().numpy()
    toe_h = toe.cpu().numpy().astype(np.int64)
    paired_t = tt_h >= 0
    tets_used = tt_h[paired_t]
    assert len(np.unique(tets_used)) == len(tets_used)
    tkey = r.tet_key()
    toff = r.tet_off()
    tval = tkey[torch.from_numpy(tets_used).to(tkey.device), 0].cpu().numpy()
    tri_h = r.tri_key().cpu().numpy()
    tri_val = tri_h >> 39
    assert np.all(tval >= tri_val[paired_t])
    dead_t = np.zeros(T, bool)
    dead_t[toe_h[toe_h >= 0]] = True
    assert not np.any(dead_t & paired_t)
    # sampled apparent pairs, by definition
    ij = r.edge_ij().cpu().numpy().astype(np.int64)
    R = np.full((n, n), -1, np.int64)
    R[ij[:, 0], ij[:, 1]] = np.arange(K)
    R[ij[:, 1], ij[:, 0]] = np.arange(K)
    rng = np.random.default_rng(7)
    apparent = 0
    for t in rng.choice(np.nonzero(~dead_t)[0], 3000, replace=False):
        key = int(tri_h[t])
        v, tri = key >> 39, ((key >> 26) & 0x1FFF, (key >> 13) & 0x1FFF, key & 0x1FFF)
        s = _oldest_cofacet(R, v, tri)
        if s is None:
            assert tt_h[t] == -1
            continue
        if _youngest_facet(R, s) != (v,) + tri:
            continue
        apparent += 1
        vk = (s[1] << 39) | (s[2] << 26) | (s[3] << 13) | s[4]
        lo, hi = int(toff[s[0]]), int(toff[s[0] + 1])
        idx = lo + int(torch.searchsorted(tkey[lo:hi, 1].contiguous(), torch.tensor([vk], device=tkey.device)).item())
        assert tt_h[t] == idx, (t, s)
    assert apparent > 0
    # the barcode: a bar per pair of positive length and per triangle paired
    # with nothing; the tetrahedra left unpaired are the classes of dimension 3
    bars, ess3 = vr.barcode_dim2(r, toe, tt)
    b = bars.cpu().numpy()
    assert ess3 == r.T3 - int(paired_t.sum())
    assert np.all(b[:, 0] == 2) and np.all(b[:, 1] < b[:, 2])
    positive = int(np.count_nonzero(tval > tri_val[paired_t]))
    assert len(b) == positive + int(np.count_nonzero(~paired_t & ~dead_t))
    print(f"[gpu] circle1000 dimension 2: {int(paired_t.sum())} pairs, {apparent} of 3000 sampled apparent, "
          f"{len(b)} bars, {ess3} classes of dimension 3", flush=True)
    r.free()


@pytest.mark.parametrize("maxdim", [2, 3])
def test_persistence_chain_matches_oracle_barcode(orc, maxdim):
    """vr.persistence, the build, pairs and barcodes chained on the device,
    gives the oracle's barcode: every bar of dimensions 0..maxdim-1 and the
    count of classes of the top dimension."""
    import paper_1809_04424_amd as vr

    c = workloads.noisy_circle(seed=220, n=160)
    thr = ("fraction", 25, 100)
    import torch

    out = vr.persistence(torch.from_numpy(np.ascontiguousarray(c.points)).to("cuda:0"), thr, maxdim=maxdim)
    f = orc.build(c.points, thr)
    p = orc.reduce(f, "cohomology")
    if maxdim == 3:
        tets = orc.tetra_list(f)
        want = orc.barcode(f, orc.with_dim2(f, p, tets), tets)
        assert out["counts"] == f.counts + (len(tets),)
    else:
        want = orc.barcode(f, p)
        assert out["counts"] == f.counts
    got = sorted(tuple(int(x) for x in b) for b in out["bars"].cpu().numpy())
    assert got == sorted(b for b in want if b[0] < maxdim)
    assert out["essential_top"] == sum(1 for b in want if b[0] == maxdim)


@pytest.mark.parametrize("maxdim", [2, 3])
@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 6])
def test_persistence_tiny_clouds(orc, n, maxdim):
    """The chained call on clouds with no edge, no triangle or no
    tetrahedron (full threshold): the oracle's barcode, and the counts."""
    import torch

    import paper_1809_04424_amd as vr

    c = workloads.uniform_cloud(400 + n, n, 3, thr=("full", 0, 1))
    print(f"[gpu] persistence n={n} maxdim={maxdim}", flush=True)
    out = vr.persistence(torch.from_numpy(np.ascontiguousarray(c.points)).to("cuda:0"), c.thr, maxdim=maxdim)
    f = orc.build(c.points, c.thr)
    p = orc.reduce(f, "cohomology")
    if maxdim == 3:
        tets = orc.tetra_list(f)
        want = orc.barcode(f, orc.with_dim2(f, p, tets), tets)
        assert out["counts"] == f.counts + (len(tets),)
    else:
        want = orc.barcode(f, p)
        assert out["counts"] == f.counts
    got = sorted(tuple(int(x) for x in b) for b in out["bars"].cpu().numpy())
    assert got == sorted(b for b in want if b[0] < maxdim)
    assert out["essential_top"] == sum(1 for b in want if b[0] == maxdim)
