"""Batched builds on the GPU: every cloud of a batch equals the oracle and is
byte-identical to its own single build (the cloud index in the sort key and
the per-cloud numbering must not leak into any output)."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_matches_oracle, gpu_build, gpu_build_batch, host_threads, item_host, pack_rows

pytestmark = pytest.mark.gpu


def _mixed(kind="fraction", seed=100):
    """Uneven clouds: empty, single point, a pair, tiny, several tiles, ties."""
    rng = np.random.default_rng(seed)
    sizes = [0, 1, 2, 3, 5, 17, 64, 65, 130, 200, 333, 700]
    out = []
    for i, n in enumerate(sizes):
        c = workloads.uniform_cloud(seed + i, n, 3, lo=-40, hi=40)
        E = n * (n - 1) // 2
        if kind == "fraction":
            c.thr = ("fraction", int(rng.integers(0, 101)), 100)
        elif kind == "count":
            c.thr = ("count", int(rng.integers(0, E + 1)) if E else 0, 1)
        elif kind == "sqdist":
            c.thr = ("sqdist", int(rng.choice([0, 1, 200, 800, 3000, 1 << 40])), 0)
        else:
            c.thr = ("full", 0, 1)
        out.append(c)
    lattice_thr = {"fraction": ("fraction", 50, 100), "count": ("count", 300, 1), "sqdist": ("sqdist", 7, 0),
                   "full": ("full", 0, 1)}[kind]
    out.append(workloads.lattice_cloud(seed + 50, 90, side=4, d=3, thr=lattice_thr))  # distance ties
    return out


def _assert_same(a, b):
    assert tuple(a["counts"]) == tuple(b["counts"])
    for k in ("edge_ij", "edge_q", "tri"):
        assert a[k].dtype == b[k].dtype and a[k].shape == b[k].shape, k
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("kind", ["fraction", "count", "sqdist", "full"])
def test_batch_matches_oracle_and_single_builds(orc, kind):
    clouds = _mixed(kind)
    b, outs = gpu_build_batch(clouds)
    assert len(b) == len(clouds)
    for c, out in zip(clouds, outs):
        f = orc.build(c.points, c.thr)
        assert_matches_oracle(out, f)
        r, single = gpu_build(c)
        _assert_same(out, single)
        r.free()
    b.free()


def test_batch_lower_maxdim_and_count_only(orc):
    clouds = _mixed("fraction", seed=300)
    _, outs1 = gpu_build_batch(clouds, maxdim=1)
    _, outs0 = gpu_build_batch(clouds, maxdim=0)
    _, outsc = gpu_build_batch(clouds, count_only=True)
    for c, o1, o0, oc in zip(clouds, outs1, outs0, outsc):
        f = orc.build(c.points, c.thr)
        assert tuple(o1["counts"]) == (f.n, f.K, 0)
        assert np.array_equal(o1["edge_q"], f.eq)
        assert tuple(o0["counts"]) == (f.n, 0, 0)
        assert tuple(oc["counts"]) == (f.n, f.K, f.T)
        assert oc["tri"].size == 0 and np.array_equal(oc["edge_q"], f.eq)


def test_batch_torch_allocator_outputs_outlive_handle(orc):
    import torch

    clouds = _mixed("fraction", seed=400)
    b, _ = gpu_build_batch(clouds, allocator="torch")
    keep = [(it.edge_q(), it.edge_ij(), it.tri_key()) for it in b]
    b.free()
    del b
    torch.cuda.synchronize()
    junk = torch.full((1 << 24,), -1, dtype=torch.int64, device="cuda:0")  # reuse of freed memory
    torch.cuda.synchronize()
    for c, (q, ij, t) in zip(clouds, keep):
        f = orc.build(c.points, c.thr)
        out = {"counts": (f.n, q.numel(), t.numel()), "edge_q": q.cpu().numpy(),
               "edge_ij": ij.cpu().numpy().astype(np.int64), "tri": t.cpu().numpy()}
        assert_matches_oracle(out, f)
    del junk


def test_batch_repeat_is_deterministic():
    clouds = _mixed("fraction", seed=500)
    _, a = gpu_build_batch(clouds)
    _, b = gpu_build_batch(clouds)
    for x, y in zip(a, b):
        _assert_same(x, y)


def _oracle_all(clouds, orc, list_for=()):
    """The oracle's filtration of every cloud, clouds spread over host
    threads (the C routines run without the interpreter lock); triangles
    listed only for the clouds in `list_for`, counted for the others."""
    import concurrent.futures as cf

    def one(i):
        c = clouds[i]
        return orc.build_mt(c.points, c.thr, 1, list_triangles=i in list_for)

    with cf.ThreadPoolExecutor(max_workers=host_threads()) as ex:
        return list(ex.map(one, range(len(clouds))))


def test_batched_workload_against_oracle(orc):
    """The 512-cloud R^3 workload (n log-uniform in [50, 2000], 5th-25th
    percentile), one batched build as the benchmark times it: every cloud's
    counts (n, K, T) and kept edges (endpoints, squared lengths) equal the
    oracle's; the triangle lists equal the oracle's element by element for
    the 8 largest clouds and every 16th cloud by size; and every cloud is
    byte-identical to its own single build on the device."""
    import sys

    import torch

    import paper_1809_04424_amd as vr

    clouds = workloads.batched()
    order = sorted(range(len(clouds)), key=lambda i: clouds[i].n)
    listed = set(order[-8:]) | set(order[::16])
    print(f"[gpu] batched512 oracle ({len(listed)} clouds listed)", flush=True)
    sys.stdout.flush()
    fs = _oracle_all(clouds, orc, listed)
    pts = [torch.from_numpy(c.points).to("cuda:0") for c in clouds]
    print("[gpu] batched512 build", flush=True)
    b = vr.build_batch(pts, [c.thr for c in clouds])
    torch.cuda.synchronize()
    for i, (c, f, it) in enumerate(zip(clouds, fs, b)):
        h = item_host(it)
        assert tuple(h["counts"]) == (f.n, f.K, f.T), f"cloud {i}"
        assert np.array_equal(h["edge_ij"][:, 0], f.ei) and np.array_equal(h["edge_ij"][:, 1], f.ej), f"cloud {i}"
        assert np.array_equal(h["edge_q"], f.eq), f"cloud {i}"
        if i in listed:
            assert np.array_equal(h["tri"].view(np.uint64), pack_rows(f.tris)), f"cloud {i}"
    print("[gpu] batched512 single builds", flush=True)
    for c, p, it in zip(clouds, pts, b):
        r = vr.build(p, c.thr)
        assert it.counts == r.counts
        assert torch.equal(it.edge_q(), r.edge_q())
        assert torch.equal(it.edge_ij(), r.edge_ij())
        assert torch.equal(it.tri_key(), r.tri_key())
        r.free()
    b.free()
