"""The enumeration schedule picked by the autotuner changes no output."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_matches_oracle, gpu_build, gpu_build_batch

pytestmark = pytest.mark.gpu


def test_autotune_then_build_matches_oracle(orc):
    import torch

    import paper_1809_04424_amd as vr

    c = workloads.noisy_circle(n=600)
    pts = torch.from_numpy(c.points).to("cuda:0")
    ebc, pc, nc, ebw, pw, nw = vr.autotune(pts, c.thr)
    assert ebc in (128, 256, 512) and ebw in (128, 256, 512)
    assert pc in (1, 2, 4, 8, 16) and pw in (0, 1, 2, 4, 8, 16)
    assert nc in (2, 4, 8) and nw in (4, 8)
    r, out = gpu_build(c)
    assert_matches_oracle(out, orc.build(c.points, c.thr))
    r.free()


def test_autotune_batch_then_build_batch(orc):
    import torch

    import paper_1809_04424_amd as vr

    clouds = [workloads.uniform_cloud(70 + i, n, 3, lo=-40, hi=40) for i, n in enumerate([90, 150, 300, 40])]
    for c in clouds:
        c.thr = ("fraction", 25, 100)
    pts = [torch.from_numpy(c.points).to("cuda:0") for c in clouds]
    sched = vr.autotune(pts, [c.thr for c in clouds])
    assert min(sched[:4] + sched[5:]) >= 1 and sched[4] >= 0
    b, outs = gpu_build_batch(clouds)
    for c, out in zip(clouds, outs):
        assert_matches_oracle(out, orc.build(c.points, c.thr))
    b.free()


def test_autotune_without_triangles():
    import torch

    import paper_1809_04424_amd as vr

    c = workloads.uniform_cloud(5, 50, 3)
    c.thr = ("fraction", 10, 100)
    assert vr.autotune(torch.from_numpy(c.points).to("cuda:0"), c.thr, maxdim=1) == (0,) * 6


@pytest.mark.parametrize("sched", [(128, 16, 2, 128, 16, 4), (512, 1, 8, 512, 1, 8), (256, 4, 4, 128, 2, 4),
                                   (512, 1, 4, 256, 0, 8), (256, 2, 4, 128, 0, 4), (128, 1, 2, 512, 0, 8)])
def test_pinned_schedule_builds_match_oracle(orc, sched):
    import torch

    import paper_1809_04424_amd as vr

    c = workloads.noisy_circle(seed=60, n=450)
    pts = torch.from_numpy(c.points).to("cuda:0")
    vr.set_schedule(pts, c.thr, sched)
    r, out = gpu_build(c)
    assert_matches_oracle(out, orc.build(c.points, c.thr))
    r.free()


@pytest.mark.parametrize("sched", [(256, 1, 4, 256, 0, 8), (256, 1, 4, 512, 0, 4), (256, 1, 4, 128, 0, 8)])
def test_wave_per_eighth_write_batch_matches_oracle(orc, sched):
    """The write with one wave per (vertex, eighth of its partners) on a batch
    of clouds of mixed sizes, some smaller than 8 points (eighths with no
    vertex) and some not a multiple of 8, and a dense 64-dimensional one."""
    import torch

    import paper_1809_04424_amd as vr

    small = [workloads.uniform_cloud(300 + i, n, 3, lo=-40, hi=40) for i, n in enumerate([5, 9, 61, 250, 333])]
    for c in small:
        c.thr = ("fraction", 30, 100)
    mix = workloads.mixture(seed=307, n=420)
    mix.thr = ("fraction", 15, 100)
    for group in (small, [mix]):
        pts = [torch.from_numpy(np.ascontiguousarray(c.points)).to("cuda:0") for c in group]
        print(f"[gpu] wave-per-eighth write {sched} clouds {[len(c.points) for c in group]}", flush=True)
        vr.set_schedule(pts, [c.thr for c in group], sched)
        b, outs = gpu_build_batch(group)
        for c, out in zip(group, outs):
            assert_matches_oracle(out, orc.build(c.points, c.thr))
        b.free()
