"""The request loop on the GPU: every result is bit-identical to a build of
the same cloud alone, whatever batch and stream it shared, and admission
keeps the reserved bytes within the budget."""
import time

import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_matches_oracle, item_host

pytestmark = pytest.mark.gpu


def _requests(seed=7, count=60):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        d = int(rng.choice([2, 3, 16]))
        n = int(rng.integers(0, 400)) if i % 10 else int(rng.integers(0, 4))
        c = workloads.uniform_cloud(seed * 1000 + i, n, d, lo=-60, hi=60)
        c.thr = ("fraction", int(rng.integers(500, 2001)), 10000)
        out.append(c)
    return out


def _alone(c):
    import torch

    import paper_1809_04424_amd as vr

    r = vr.build(torch.from_numpy(c.points).to("cuda:0"), c.thr)
    torch.cuda.synchronize()
    h = item_host(r)
    r.free()
    return h


def _same(a, b):
    assert tuple(a["counts"]) == tuple(b["counts"])
    for k in ("edge_ij", "edge_q", "tri"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("slots,max_batch", [(1, 1), (3, 8), (4, 32)])
def test_served_results_equal_alone(orc, slots, max_batch):
    import torch

    from paper_1809_04424_amd.serve import Server

    clouds = _requests()
    pts = [torch.from_numpy(c.points).to("cuda:0") for c in clouds]
    torch.cuda.synchronize()
    with Server(slots=slots, max_batch=max_batch) as srv:
        reqs = []
        # bursts arriving while earlier batches run
        for i, (p, c) in enumerate(zip(pts, clouds)):
            reqs.append(srv.submit(p, c.thr))
            if i % 15 == 14:
                time.sleep(0.002)
        for r in reqs:
            r.wait(timeout=120)
    assert max(r.batch_size for r in reqs) <= max_batch
    if max_batch > 1:
        assert any(r.batch_size > 1 for r in reqs)  # the mix really batched
    for c, r in zip(clouds, reqs):
        got = item_host(r.item)
        _same(got, _alone(c))
        r.release()
    assert all(r.counts[0] == c.n for c, r in zip(clouds, reqs))
    f = orc.build(clouds[5].points, clouds[5].thr)
    assert reqs[5].counts == (f.n, f.K, f.T)
    assert srv._held == 0 and srv._reserved == 0


def test_admission_respects_budget():
    import torch

    import paper_1809_04424_amd as vr
    from paper_1809_04424_amd.serve import Server

    clouds = [c for c in _requests(seed=9, count=30) if c.n >= 2]
    pts = [torch.from_numpy(c.points).to("cuda:0") for c in clouds]
    biggest = max(vr.batch_workspace_bytes([(c.n, c.d, vr.VR_I8, c.thr)]) for c in clouds)
    budget = 2 * biggest
    with Server(slots=4, max_batch=16, budget_bytes=budget, keep_results=False) as srv:
        reqs = [srv.submit(p, c.thr) for p, c in zip(pts, clouds)]
        for r in reqs:
            r.wait(timeout=120)
    assert srv.peak_bytes <= budget
    for c, r in zip(clouds, reqs):
        assert r.counts == _alone(c)["counts"]


def test_rejected_request_fails_alone():
    import torch

    import paper_1809_04424_amd as vr
    from paper_1809_04424_amd.serve import Server

    good = workloads.uniform_cloud(11, 50, 3)
    good.thr = ("fraction", 10, 100)
    with Server(slots=2) as srv:
        bad = srv.submit(torch.zeros((9000, 3), dtype=torch.int8, device="cuda:0"), ("fraction", 1, 100))
        ok = srv.submit(torch.from_numpy(good.points).to("cuda:0"), good.thr)
        with pytest.raises(vr.VrError):
            bad.wait(timeout=60)
        ok.wait(timeout=60)
    assert ok.counts == _alone(good)["counts"]
