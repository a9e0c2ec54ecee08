"""Captured first phases (VR_GRAPH): every replay equals the eager build.

A graph is captured on the first build of a request and replayed on later
ones; eager builds of other clouds and device synchronisations run between
the replays, and every replay is compared with the eager result byte for
byte and with the oracle.
"""
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


def _same(a, b):
    assert a["counts"] == b["counts"]
    for k in ("edge_q", "edge_ij", "tri"):
        assert np.array_equal(a[k], b[k]), k


def test_graph_replays_match_eager(orc):
    import torch

    import paper_1809_04424_amd as vr

    a = workloads.noisy_circle(seed=41, n=500)
    b = workloads.uniform_cloud(42, 300, 16, thr=("fraction", 15, 100))
    pa = torch.from_numpy(a.points).to("cuda:0")
    pb = torch.from_numpy(b.points).to("cuda:0")
    ra = vr.build(pa, a.thr)
    eager_a = _host(ra)
    ra.free()
    assert_matches_oracle(eager_a, orc.build(a.points, a.thr))
    rb = vr.build(pb, b.thr)
    eager_b = _host(rb)
    rb.free()
    for i in range(5):
        print(f"[gpu] graph replay {i}", flush=True)
        r = vr.build(pa, a.thr, graph=True)  # capture on the first, replays after
        _same(_host(r), eager_a)
        r.free()
        r = vr.build(pb, b.thr)  # eager work between replays
        _same(_host(r), eager_b)
        r.free()
        torch.cuda.synchronize()
    vr.trim()  # drops the graph; the next build captures again
    r = vr.build(pa, a.thr, graph=True)
    _same(_host(r), eager_a)
    r.free()


def test_graph_sees_points_changed_in_place(orc):
    import torch

    import paper_1809_04424_amd as vr

    a = workloads.noisy_circle(seed=43, n=400)
    b = workloads.noisy_circle(seed=44, n=400)
    pts = torch.from_numpy(a.points).to("cuda:0")
    r = vr.build(pts, a.thr, graph=True)
    assert_matches_oracle(_host(r), orc.build(a.points, a.thr))
    r.free()
    pts.copy_(torch.from_numpy(b.points))  # same pointer, new coordinates
    r = vr.build(pts, b.thr, graph=True)
    assert_matches_oracle(_host(r), orc.build(b.points, b.thr))
    r.free()


def test_graph_results_alive_across_streams(orc):
    import torch

    import paper_1809_04424_amd as vr

    a = workloads.noisy_circle(seed=45, n=350)
    pa = torch.from_numpy(a.points).to("cuda:0")
    ref = orc.build(a.points, a.thr)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    kept = []
    for i in range(6):
        with torch.cuda.stream(streams[i % 2]):
            kept.append(vr.build(pa, a.thr, graph=True))
    torch.cuda.synchronize()
    for r in kept:
        assert_matches_oracle(_host(r), ref)
        r.free()


def test_graph_batch_replays(orc):
    import torch

    import paper_1809_04424_amd as vr

    clouds = [workloads.uniform_cloud(50 + i, n, 3, lo=-60, hi=60) for i, n in enumerate([120, 260, 40])]
    for c in clouds:
        c.thr = ("fraction", 20, 100)
    refs = [orc.build(c.points, c.thr) for c in clouds]
    pts = [torch.from_numpy(c.points).to("cuda:0") for c in clouds]
    for i in range(4):
        print(f"[gpu] graph batch replay {i}", flush=True)
        b = vr.build_batch(pts, [c.thr for c in clouds], graph=True)
        torch.cuda.synchronize()
        for it, ref in zip(b, refs):
            assert_matches_oracle(item_host(it), ref)
        b.free()
        # eager single builds between the replays
        r = vr.build(pts[1], clouds[1].thr)
        assert_matches_oracle(_host(r), refs[1])
        r.free()
