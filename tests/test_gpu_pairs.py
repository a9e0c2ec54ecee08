"""Dimension-0 persistence pairs on the device (vr_pairs_dim0) against the
oracle's column reductions, bit-exact."""
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


def _gpu_pairs(points, thr):
    import torch

    import paper_1809_04424_amd as vr

    r = vr.build(torch.from_numpy(np.ascontiguousarray(points)).to("cuda:0"), thr)
    e_low, death = vr.pairs_dim0(r)
    torch.cuda.synchronize()
    out = e_low.cpu().numpy().astype(np.int64), death.cpu().numpy().astype(np.int64), r.counts
    r.free()
    return out


def _check(orc, points, thr, label):
    print(f"[gpu] pairs_dim0 {label} n={len(points)} thr={thr}", flush=True)
    f = orc.build(points, thr, maxdim=1)  # dimension 0 needs no triangles
    ref = orc.reduce(f, "cohomology").e_low
    e_low, death, counts = _gpu_pairs(points, thr)
    assert counts[0] == f.n and counts[1] == f.K
    assert np.array_equal(e_low, ref)
    # death is the inverse of e_low; the unpaired vertices are one per component
    want = np.full(f.n, -1, np.int64)
    for r in np.nonzero(ref >= 0)[0]:
        want[ref[r]] = r
    assert np.array_equal(death, want)
    assert death[0] == -1 if f.n else True


CASES = [
    ("circle150_p10", lambda: workloads.noisy_circle(seed=40, n=150).points, ("fraction", 10, 100)),
    ("circle300_sparse", lambda: workloads.noisy_circle(seed=41, n=300).points, ("count", 250, 1)),
    ("circle1000_p20", lambda: workloads.noisy_circle().points, ("fraction", 20, 100)),
    ("lattice_ties", lambda: workloads.lattice_cloud(3, 90, side=3).points, ("fraction", 30, 100)),
    ("mixture_d16", lambda: workloads.uniform_cloud(42, 260, 16).points, ("fraction", 5, 100)),
    ("plain64_full", lambda: workloads.plain64().points, ("full", 0, 1)),
    ("n65", lambda: workloads.uniform_cloud(43, 65, 3).points, ("fraction", 50, 100)),
    ("n128_sqdist", lambda: workloads.uniform_cloud(44, 128, 2).points, ("sqdist", 900, 0)),
    ("n2000", lambda: workloads.noisy_circle(seed=45, n=2000).points, ("fraction", 2, 100)),
]


@pytest.mark.parametrize("name,gen,thr", CASES, ids=[c[0] for c in CASES])
def test_pairs_dim0(orc, name, gen, thr):
    _check(orc, gen(), thr, name)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_pairs_dim0_tiny(orc, n):
    pts = np.array([[0, 0], [3, 0], [0, 4]][:n], np.int32)
    _check(orc, pts, ("full", 0, 1), f"tiny{n}")


def test_pairs_dim0_no_edges(orc):
    pts = workloads.uniform_cloud(46, 50, 3).points
    e_low, death, counts = _gpu_pairs(pts, ("count", 0, 1))
    assert counts[1] == 0 and len(e_low) == 0 and np.all(death == -1)


def test_pairs_dim0_largest_point_count(orc):
    """n = 8192, the largest point count (a 268 MB closure in 128 pivot
    blocks), at a sparse threshold that leaves several components."""
    import time

    import torch

    import paper_1809_04424_amd as vr

    c = workloads.uniform_cloud(47, 8192, 3)
    thr = ("fraction", 1, 1000)
    print("[gpu] pairs_dim0 n=8192", flush=True)
    f = orc.build(c.points, thr, maxdim=1)
    ref = orc.reduce(f, "cohomology").e_low
    r = vr.build(torch.from_numpy(c.points).to("cuda:0"), thr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e_low, death = vr.pairs_dim0(r)
    torch.cuda.synchronize()
    print(f"[gpu] pairs_dim0 n=8192 K={r.counts[1]}: {1e3 * (time.perf_counter() - t0):.1f} ms", flush=True)
    assert np.array_equal(e_low.cpu().numpy().astype(np.int64), ref)
    assert int((death.cpu().numpy() < 0).sum()) == f.n - int((ref >= 0).sum())
    r.free()


def test_pairs_dim0_of_batch_items_and_matrix_builds(orc):
    """Any result works: the clouds of a batch (pairs of both dimensions and
    tetrahedra), and a dissimilarity-matrix build."""
    import torch

    import paper_1809_04424_amd as vr

    clouds = [workloads.noisy_circle(seed=60 + i, n=n).points for i, n in enumerate((40, 150, 3, 260))]
    thr = ("fraction", 15, 100)
    b = vr.build_batch([torch.from_numpy(p).to("cuda:0") for p in clouds], thr)
    for p, item in zip(clouds, b):
        e_low, death = vr.pairs_dim0(item)
        tet = vr.tetra_counts(item)
        app = vr.pairs_dim1_apparent(item)
        torch.cuda.synchronize()
        f = orc.build(p, thr)
        assert np.array_equal(e_low.cpu().numpy().astype(np.int64), orc.reduce(f, "cohomology").e_low)
        assert np.array_equal(tet.cpu().numpy(), orc.tetra_counts(f))
        want = np.full(f.K, -1, np.int64)
        if f.T:
            v = f.tris[:, 0]
            first = np.nonzero(np.r_[True, v[1:] != v[:-1]])[0]
            want[v[first]] = first
        assert np.array_equal(app.cpu().numpy().astype(np.int64), want)
    b.free()
    M = workloads.hamming_matrix(61, 300)
    r = vr.build_matrix(torch.from_numpy(M).to("cuda:0"), ("fraction", 5, 100))
    e_low, _ = vr.pairs_dim0(r)
    torch.cuda.synchronize()
    f = orc.build_matrix(M, ("fraction", 5, 100), maxdim=1)
    assert np.array_equal(e_low.cpu().numpy().astype(np.int64), orc.reduce(f, "cohomology").e_low)
    r.free()


@pytest.mark.parametrize("name,gen,thr", CASES[:6], ids=[c[0] for c in CASES[:6]])
def test_pairs_dim1_apparent(orc, name, gen, thr):
    import torch

    import paper_1809_04424_amd as vr

    pts = gen()
    print(f"[gpu] pairs_dim1_apparent {name}", flush=True)
    f = orc.build(pts, thr)
    r = vr.build(torch.from_numpy(np.ascontiguousarray(pts)).to("cuda:0"), thr)
    got = vr.pairs_dim1_apparent(r).cpu().numpy().astype(np.int64)
    torch.cuda.synchronize()
    r.free()
    v = f.tris[:, 0]
    want = np.full(f.K, -1, np.int64)
    if f.T:
        first = np.nonzero(np.r_[True, v[1:] != v[:-1]])[0]
        want[v[first]] = first
    assert np.array_equal(got, want)
    if f.K <= 5000:  # each is a pair of the column reduction
        t_low = orc.reduce(f, "cohomology").t_low
        assert np.all(t_low[got[got >= 0]] == np.nonzero(got >= 0)[0])


def test_pairs_dim1_apparent_needs_keys():
    import torch

    import paper_1809_04424_amd as vr

    c = workloads.noisy_circle(seed=81, n=100)
    r = vr.build(torch.from_numpy(c.points).to("cuda:0"), c.thr, count_only=True)
    with pytest.raises(vr.VrError) as e:
        vr.pairs_dim1_apparent(r)
    assert e.value.code == vr.VR_EINVAL
    r.free()


TET_CASES = [
    ("circle150_p20", lambda: workloads.noisy_circle(seed=90, n=150).points, ("fraction", 20, 100)),
    ("lattice_ties", lambda: workloads.lattice_cloud(5, 80, side=3).points, ("fraction", 40, 100)),
    ("uniform_d4_sqdist", lambda: workloads.uniform_cloud(91, 120, 4).points, ("sqdist", 30000, 0)),
    ("plain64_full", lambda: workloads.plain64().points, ("full", 0, 1)),
    ("n3", lambda: workloads.uniform_cloud(92, 3, 2).points, ("full", 0, 1)),
    ("n4", lambda: workloads.uniform_cloud(93, 4, 2).points, ("full", 0, 1)),
    ("hub_pair_m300", lambda: workloads.hub_pair(), ("sqdist", 7000, 0)),
]


@pytest.mark.parametrize("name,gen,thr", TET_CASES, ids=[c[0] for c in TET_CASES])
def test_tetra_counts(orc, name, gen, thr):
    import torch

    import paper_1809_04424_amd as vr

    pts = gen()
    print(f"[gpu] tetra_counts {name}", flush=True)
    f = orc.build(pts, thr, list_triangles=False)
    r = vr.build(torch.from_numpy(np.ascontiguousarray(pts)).to("cuda:0"), thr)
    got = vr.tetra_counts(r).cpu().numpy()
    r.free()
    assert np.array_equal(got, orc.tetra_counts(f))


@pytest.mark.parametrize("n", [100, 300])
def test_tetra_counts_full_threshold(n):
    """Every 4-subset once: the counts sum to C(n, 4)."""
    import math

    import torch

    import paper_1809_04424_amd as vr

    c = workloads.uniform_cloud(94 + n, n, 3)
    r = vr.build(torch.from_numpy(c.points).to("cuda:0"), ("full", 0, 1))
    got = vr.tetra_counts(r)
    assert int(got.sum().item()) == math.comb(n, 4)
    assert int(got[:3].sum().item()) == 0  # the first three edges close no tetrahedron
    r.free()


LIST_CASES = [
    ("circle120_p20", lambda: workloads.noisy_circle(seed=95, n=120).points, ("fraction", 20, 100)),
    ("lattice_ties", lambda: workloads.lattice_cloud(6, 50, side=3).points, ("fraction", 40, 100)),
    ("uniform_full40", lambda: workloads.uniform_cloud(96, 40, 3).points, ("full", 0, 1)),
    ("uniform_sqdist", lambda: workloads.uniform_cloud(97, 90, 4).points, ("sqdist", 25000, 0)),
    ("n4", lambda: workloads.uniform_cloud(98, 4, 2).points, ("full", 0, 1)),
    ("n3", lambda: workloads.uniform_cloud(99, 3, 2).points, ("full", 0, 1)),
    # the hub edge has 300 common older neighbours: several 256-vertex chunks
    # per row scan, rows of up to 299 later neighbours, 44850 pairs of them
    ("hub_pair_m300", lambda: workloads.hub_pair(), ("sqdist", 7000, 0)),
]


@pytest.mark.parametrize("name,gen,thr", LIST_CASES, ids=[c[0] for c in LIST_CASES])
def test_tetrahedra_listed_in_order(orc, name, gen, thr):
    import torch

    import paper_1809_04424_amd as vr

    pts = gen()
    print(f"[gpu] tetrahedra {name}", flush=True)
    f = orc.build(pts, thr, list_triangles=False)
    r = vr.build(torch.from_numpy(np.ascontiguousarray(pts)).to("cuda:0"), thr)
    off, keys = vr.tetrahedra(r)
    off, keys = off.cpu().numpy(), keys.cpu().numpy().view(np.uint64)
    r.free()
    want = orc.tetra_list(f)
    counts = orc.tetra_counts(f)
    assert np.array_equal(off, np.r_[0, np.cumsum(counts)])
    assert len(keys) == len(want)
    if len(want):
        m = np.uint64(0x1FFF)
        got = np.stack([keys[:, 0], keys[:, 1] >> np.uint64(39), (keys[:, 1] >> np.uint64(26)) & m,
                        (keys[:, 1] >> np.uint64(13)) & m, keys[:, 1] & m], axis=1).astype(np.int64)
        assert np.array_equal(got, want)
