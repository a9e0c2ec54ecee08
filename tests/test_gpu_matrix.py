"""Dissimilarity-matrix input (VR_DIST) against the oracle, bit-exact."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_matches_oracle, item_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1809_04424_amd as vr

    vr.lib()
    yield


def _host(r):
    import torch

    torch.cuda.synchronize()
    return item_host(r)


def _mat(m):
    import torch

    return torch.from_numpy(np.ascontiguousarray(m, dtype=np.int32)).to("cuda:0")


def test_squared_distance_matrix_equals_points_build(orc):
    import torch

    import paper_1809_04424_amd as vr

    c = workloads.noisy_circle(seed=70, n=400)
    p = c.points.astype(np.int64)
    M = ((p[:, None, :] - p[None, :, :]) ** 2).sum(-1)
    ref = orc.build(c.points, c.thr)
    r = vr.build_matrix(_mat(M), c.thr)
    assert_matches_oracle(_host(r), ref)
    r.free()
    r = vr.build(torch.from_numpy(c.points).to("cuda:0"), c.thr)
    assert_matches_oracle(_host(r), ref)
    r.free()


@pytest.mark.parametrize("seed,n,thr", [
    (71, 300, ("fraction", 10, 100)),
    (72, 517, ("fraction", 25, 100)),   # several tiles, a ragged tail, many ties
    (73, 200, ("sqdist", 20, 0)),
    (74, 130, ("count", 500, 1)),
    (75, 65, ("full", 0, 1)),
])
def test_hamming_matrices(orc, seed, n, thr):
    import paper_1809_04424_amd as vr

    M = workloads.hamming_matrix(seed, n)
    print(f"[gpu] hamming {seed} {n} {thr}", flush=True)
    r = vr.build_matrix(_mat(M), thr)
    assert_matches_oracle(_host(r), orc.build_matrix(M, thr))
    r.free()


def test_hypercube_distance_one_graph(orc):
    import paper_1809_04424_amd as vr

    m = 6
    x = np.arange(1 << m)
    M = np.array([[bin(a ^ b).count("1") for b in x] for a in x], np.int32)
    r = vr.build_matrix(_mat(M), ("sqdist", 2, 0))
    out = _host(r)
    assert tuple(out["counts"]) == (64, m * 32, 0)
    assert_matches_oracle(out, orc.build_matrix(M, ("sqdist", 2, 0)))
    r.free()


def test_only_the_upper_triangle_is_read(orc):
    import paper_1809_04424_amd as vr

    M = workloads.hamming_matrix(76, 150)
    junk = np.tril(np.random.default_rng(0).integers(-1000, 1000, M.shape), 0).astype(np.int32)
    Mj = np.triu(M, 1) + junk  # negative and unrelated entries on and below the diagonal
    thr = ("fraction", 20, 100)
    r = vr.build_matrix(_mat(Mj), thr)
    assert_matches_oracle(_host(r), orc.build_matrix(M, thr))
    r.free()


def test_negative_entry_is_reported():
    import paper_1809_04424_amd as vr

    M = workloads.hamming_matrix(77, 90)
    M[3, 40] = -1
    with pytest.raises(vr.VrError) as e:
        vr.build_matrix(_mat(M), ("fraction", 20, 100))
    assert e.value.code == vr.VR_ERANGE


def test_hamming1088_full_threshold_at_size(orc):
    """The sequence-data shape at full size (1088 sequences, every pair kept,
    C(1088, 3) triangles), in the launch configuration the benchmark times.
    Edges are compared bit-exactly; the 214 million triangle keys through
    properties that pin them: strictly increasing keys, i < j < k, and each
    key's value equal to the largest rank among its three edges, so with the
    closed-form count every triangle appears once, in (value, lex) order."""
    import torch

    import paper_1809_04424_amd as vr

    n = 1088
    M = workloads.hamming_matrix(1088, n)
    f = orc.build_matrix(M, ("full", 0, 1), list_triangles=False)
    assert f.T == n * (n - 1) * (n - 2) // 6
    print("[gpu] hamming1088 full", flush=True)
    r = vr.build_matrix(_mat(M), ("full", 0, 1))
    torch.cuda.synchronize()
    assert tuple(r.counts) == (n, f.K, f.T)
    ij = r.edge_ij().cpu().numpy().astype(np.int64)
    assert np.array_equal(ij[:, 0], f.ei) and np.array_equal(ij[:, 1], f.ej)
    assert np.array_equal(r.edge_q().cpu().numpy(), f.eq)
    keys = r.tri_key()
    R = torch.from_numpy(f.R.astype(np.int64)).to("cuda:0").reshape(-1)
    mask = (1 << 13) - 1
    step = 1 << 24
    for a in range(0, keys.numel(), step):
        k = keys[a:a + step + 1]
        assert bool((k[1:] > k[:-1]).all())
        v, i, j, l = k >> 39, (k >> 26) & mask, (k >> 13) & mask, k & mask
        assert bool(((i < j) & (j < l) & (l < n)).all())
        want = torch.maximum(torch.maximum(R[i * n + j], R[i * n + l]), R[j * n + l])
        assert bool((v == want).all())
    r.free()
