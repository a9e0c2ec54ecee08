"""GPU parity: the HIP path against the CPU oracle, bit-exact.

Every comparison is on identical seeded inputs; every output is integer, so
the tolerance is exact equality.
"""
import math
import sys

import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_keys_match_oracle, assert_matches_oracle, decode_keys, gpu_build, host_threads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1809_04424_amd as vr

    vr.lib()  # fails loudly if the library is missing
    yield


SMALL = [
    workloads.uniform_cloud(1, 9, 2, thr=("full", 0, 1)),
    workloads.uniform_cloud(2, 11, 3, thr=("fraction", 40, 100)),
    workloads.lattice_cloud(3, 40, side=3, thr=("fraction", 50, 100)),
    workloads.lattice_cloud(4, 30, side=2, thr=("count", 17, 1)),
    workloads.uniform_cloud(5, 50, 4, thr=("sqdist", 20000, 0)),
    workloads.uniform_cloud(6, 3, 1, thr=("full", 0, 1)),
    workloads.uniform_cloud(7, 2, 2, thr=("full", 0, 1)),
    workloads.uniform_cloud(8, 1, 2, thr=("full", 0, 1)),
    workloads.uniform_cloud(18, 0, 2, thr=("full", 0, 1)),
    workloads.lattice_cloud(9, 80, side=1, thr=("fraction", 60, 100)),  # all points equal
    workloads.uniform_cloud(10, 300, 16, thr=("fraction", 15, 100)),
    workloads.uniform_cloud(11, 257, 3, thr=("count", 1, 1)),
    workloads.uniform_cloud(12, 129, 3, thr=("count", 2, 1)),
    workloads.uniform_cloud(13, 130, 3, thr=("count", 3, 1)),
    workloads.uniform_cloud(14, 131, 3, thr=("count", 0, 1)),
    workloads.uniform_cloud(15, 200, 64, thr=("fraction", 7, 100)),
    workloads.uniform_cloud(16, 150, 5, dtype=np.int16, lo=-10000, hi=10000, thr=("fraction", 30, 100)),  # q < 2^31
    workloads.uniform_cloud(17, 150, 2, dtype=np.int32, lo=0, hi=20000, thr=("fraction", 25, 100)),
    workloads.uniform_cloud(19, 100, 3, thr=("sqdist", 10 ** 12, 0)),  # tau above every q: all kept
    workloads.uniform_cloud(20, 100, 3, thr=("sqdist", 0, 0)),         # nothing kept
    workloads.uniform_cloud(21, 333, 130, thr=("fraction", 12, 100)),  # several coordinate chunks
    workloads.lattice_cloud(22, 500, side=4, d=3, thr=("fraction", 20, 100)),  # heavy ties across tiles
    workloads.uniform_cloud(23, 150, 37, thr=("fraction", 20, 100)),   # matrix-core path, padded depth
    workloads.uniform_cloud(24, 100, 256, thr=("fraction", 30, 100)),  # deepest matrix-core input
    workloads.uniform_cloud(25, 90, 257, thr=("fraction", 30, 100)),   # vector path past it
    workloads.uniform_cloud(26, 150, 64, lo=-128, hi=-100, thr=("count", 4000, 1)),  # -128 extremes
    workloads.uniform_cloud(27, 170, 96, thr=("fraction", 20, 100)),   # matrix cores, 128-deep staging, 16-byte rows
    workloads.uniform_cloud(28, 140, 100, thr=("fraction", 20, 100)),  # 128-deep staging, rows staged bytewise
]


@pytest.mark.parametrize("cloud", SMALL, ids=lambda c: f"{c.name}_{c.thr[0]}{c.thr[1]}")
def test_small_clouds_bit_exact(orc, cloud):
    _say(f"[gpu] {cloud.name} n={cloud.n} d={cloud.d} thr={cloud.thr}")
    f = orc.build(cloud.points, cloud.thr)
    _, out = gpu_build(cloud)
    assert_matches_oracle(out, f)


@pytest.mark.parametrize("maxdim", [0, 1])
def test_lower_maxdim(orc, maxdim):
    c = workloads.uniform_cloud(30, 120, 3, thr=("fraction", 30, 100))
    f = orc.build(c.points, c.thr, maxdim=maxdim)
    _, out = gpu_build(c, maxdim=maxdim)
    assert out["counts"] == (f.n, f.K, 0)
    assert np.array_equal(out["edge_q"], f.eq)


def test_count_only(orc):
    c = workloads.noisy_circle(n=500)
    f = orc.build(c.points, c.thr, list_triangles=False)
    res, out = gpu_build(c, count_only=True)
    assert out["counts"] == f.counts
    assert len(out["tri"]) == 0


def test_plain64_full_threshold(orc):
    c = workloads.plain64()
    f = orc.build(c.points, c.thr)
    _, out = gpu_build(c)
    assert out["counts"] == (64, 2016, 41664)
    assert_matches_oracle(out, f)


def test_circle1000_bit_exact(orc):
    c = workloads.noisy_circle()
    _say("[gpu] circle1000 oracle")
    f = orc.build(c.points, c.thr)
    _say("[gpu] circle1000 build")
    _, out = gpu_build(c)
    assert out["counts"][1] == 99900
    assert_matches_oracle(out, f)


def test_repeat_builds_identical():
    c = workloads.noisy_circle(n=700)
    a = gpu_build(c)[1]
    b = gpu_build(c)[1]
    assert np.array_equal(a["tri"], b["tri"])
    assert np.array_equal(a["edge_ij"], b["edge_ij"])


_MIX_ORACLE = {}


@pytest.mark.parametrize("sched", [None, (512, 1, 4, 512, 2, 8), (512, 1, 4, 256, 0, 8)],
                         ids=["default", "bench_tuned", "wave_per_eighth"])
def test_mixture4000_complete(orc, sched):
    """Full-size 4000 x R^64 mixture at the 10th percentile (the headline
    workload): every kept edge and all 94,017,474 triangle keys equal the
    oracle's, element by element, with the default schedule, the one the
    benchmark's tuning picks (two work-groups per vertex in the write), and
    the write with one wave per vertex and eighth of its partners."""
    import torch

    import paper_1809_04424_amd as vr

    c = workloads.mixture()
    if "f" not in _MIX_ORACLE:
        _say("[gpu] mixture4000 oracle (threaded)")
        _MIX_ORACLE["f"] = orc.build_mt(c.points, c.thr, host_threads(), list_triangles=False)
    f = _MIX_ORACLE["f"]
    if sched is not None:
        vr.set_schedule(torch.from_numpy(np.ascontiguousarray(c.points)).to("cuda:0"), c.thr, sched)
    _say(f"[gpu] mixture4000 build, schedule {sched}")
    res, out = gpu_build(c)
    assert out["counts"] == (4000, 799800, f.T)
    assert np.array_equal(out["edge_ij"][:, 0], f.ei)
    assert np.array_equal(out["edge_ij"][:, 1], f.ej)
    assert np.array_equal(out["edge_q"], f.eq)
    _say("[gpu] mixture4000 compare every key")
    assert_keys_match_oracle(out["tri"], f, orc)
    res.free()


@pytest.mark.parametrize("dtype,lo,hi,d", [(np.int32, -2 ** 30, 2 ** 30, 3), (np.int16, -30000, 30000, 5),
                                            (np.int32, 0, 50000, 4)])
def test_overflow_is_reported(orc, dtype, lo, hi, d):
    """A squared distance of 2^32 or more is rejected with VR_ERANGE."""
    import paper_1809_04424_amd as vr

    c = workloads.uniform_cloud(40, 20, d, dtype=dtype, lo=lo, hi=hi)
    assert orc.sqdist(c.points).max() >= 2 ** 32
    with pytest.raises(vr.VrError) as e:
        gpu_build(c)
    assert e.value.code == vr.VR_ERANGE


def test_full_threshold_binomials():
    for n in (3, 65, 190):
        c = workloads.uniform_cloud(n, n, 2, dtype=np.int32, lo=0, hi=1023)
        _, out = gpu_build(c)
        assert out["counts"] == (n, math.comb(n, 2), math.comb(n, 3))


@pytest.mark.parametrize("pts,ok", [
    ([[0], [65535]], True),            # q = 65535^2 = 2^32 - 2^17 + 1
    ([[0, 0], [65535, 361]], True),    # q = 2^32 - 2^17 + 1 + 130321 < 2^32
    ([[0], [65536]], False),           # q = 2^32
    ([[0, 0], [65535, 363]], False),   # q = 2^32 + 698
])
def test_key_width_boundary(orc, pts, ok):
    import paper_1809_04424_amd as vr

    c = workloads.Cloud(np.array(pts, np.int32), ("full", 0, 1))
    q = int(orc.sqdist(c.points)[0])
    assert (q < 2 ** 32) == ok
    if ok:
        _, out = gpu_build(c)
        assert out["edge_q"].tolist() == [q]
    else:
        with pytest.raises(vr.VrError) as e:
            gpu_build(c)
        assert e.value.code == vr.VR_ERANGE


def test_torch_allocator_path(orc):
    """Outputs through torch's caching allocator equal the library-pool path."""
    c = workloads.noisy_circle(n=600)
    f = orc.build(c.points, c.thr)
    _, out = gpu_build(c, allocator="torch")
    assert_matches_oracle(out, f)


def test_outputs_outlive_handle(orc):
    """Tensors keep the library's output memory alive after the handle goes."""
    import gc

    import torch

    c = workloads.noisy_circle(n=400)
    f = orc.build(c.points, c.thr)
    res, _ = gpu_build(c)
    keys = res.tri_key()
    ij = res.edge_ij()
    del res
    gc.collect()
    for _ in range(3):  # reuse of freed pool memory must not touch live outputs
        gpu_build(workloads.noisy_circle(seed=9, n=400))
    torch.cuda.synchronize()
    assert np.array_equal(decode_keys(keys.cpu().numpy()), f.tris)
    assert np.array_equal(ij.cpu().numpy()[:, 0], f.ei)


def test_stage_timing_reports_every_stage():
    import paper_1809_04424_amd as vr

    c = workloads.noisy_circle(n=300)
    res, _ = gpu_build(c, timing=True)
    st = res.stage_ms()
    assert list(st) == vr.stage_names()
    assert st["tri_write"] > 0 and st["dist"] > 0
    res2, _ = gpu_build(c, timing="write")
    st2 = res2.stage_ms()
    assert st2["tri_write"] > 0 and st2["dist"] == 0


_N8192 = {}


@pytest.mark.parametrize("sched", [None, (512, 1, 4, 512, 0, 8)], ids=["default", "wave_per_eighth"])
def test_largest_point_count(orc, sched):
    """n = 8192 (the key-packing limit) with a sparse threshold: the per-vertex
    LDS staging at its largest; with the wave-per-eighth write, whose 18 KB of
    LDS per wave make the launch drop from 512 to 128 threads per
    work-group."""
    import torch

    import paper_1809_04424_amd as vr

    c = workloads.uniform_cloud(77, 8192, 2, dtype=np.int32, lo=0, hi=6000, thr=("count", 200000, 1))
    if "f" not in _N8192:
        _say("[gpu] n=8192 oracle")
        _N8192["f"] = orc.build(c.points, c.thr)
    if sched is not None:
        vr.set_schedule(torch.from_numpy(np.ascontiguousarray(c.points)).to("cuda:0"), c.thr, sched)
    _say(f"[gpu] n=8192 build, schedule {sched}")
    _, out = gpu_build(c)
    assert_matches_oracle(out, _N8192["f"])


def test_unpacked_triangles(orc):
    import workloads as wl

    c = wl.uniform_cloud(77, 150, 3, lo=-40, hi=40)
    c.thr = ("fraction", 30, 100)
    r, out = gpu_build(c)
    rows = r.triangles().cpu().numpy()
    f = orc.build(c.points, c.thr)
    # oracle rows are (v, i, j, k); the unpacked rows are (i, j, k, v)
    assert rows.shape == (f.T, 4)
    assert np.array_equal(rows[:, :3], f.tris[:, 1:]) and np.array_equal(rows[:, 3], f.tris[:, 0])
    r.free()


def test_output_guess_follows_counts(orc):
    """A build of a shape seen before enqueues its triangle write into outputs
    of the last build's sizes before the counts reach the host: a build with
    more triangles than the last must fall back, one with fewer writes into
    the larger outputs; every result stays exact."""
    few = workloads.uniform_cloud(31, 400, 3, thr=("fraction", 20, 100))
    many = workloads.noisy_circle(seed=32, n=400)
    assert many.thr == few.thr
    ref = {c.name: orc.build(c.points, c.thr) for c in (few, many)}
    assert ref[many.name].T > ref[few.name].T
    for c in (few, many, few, many, many):
        _say(f"[gpu] output guess {c.name}")
        r, out = gpu_build(c)
        assert_matches_oracle(out, ref[c.name])
        r.free()


def test_output_guess_batches(orc):
    """Batches of one shape with the clouds' triangle counts swapped between
    them reuse the outputs' size but not their per-cloud layout."""
    from tests.gpu_util import gpu_build_batch

    few = workloads.uniform_cloud(33, 300, 3, thr=("fraction", 20, 100))
    many = workloads.noisy_circle(seed=34, n=300)
    ref = {c.name: orc.build(c.points, c.thr) for c in (few, many)}
    for order in ([few, many], [many, few], [few, many]):
        _say(f"[gpu] output guess batch {[c.name for c in order]}")
        b, outs = gpu_build_batch(order)
        for c, out in zip(order, outs):
            assert_matches_oracle(out, ref[c.name])
        b.free()
