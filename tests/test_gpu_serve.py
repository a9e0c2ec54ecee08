"""The request loop on the GPU: every result is bit-identical to a build of
the same cloud alone, whatever batch and stream it shared, and admission
keeps the reserved bytes within the budget."""
import time

import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_matches_oracle, host_threads, item_host

pytestmark = pytest.mark.gpu


def _requests(seed=7, count=60):
    """A mix shaped like the serving stream (n log-uniform in [100, 2400], d
    in {2, 3, 16, 64}, 5th-20th percentile), with every fifth request a
    tiny uniform cloud (0 to 3 points, or up to 60) in between."""
    rng = np.random.default_rng(seed)
    stream = [c for _, c in workloads.serving_stream(seed=seed, requests=count - count // 5, nmin=100, nmax=2400)]
    out = []
    for i in range(count):
        if i % 5 == 4:
            n = (i // 10) % 4 if i % 10 == 9 else int(rng.integers(4, 61))
            c = workloads.uniform_cloud(seed * 1000 + i, n, int(rng.choice([2, 3, 16, 64])), lo=-60, hi=60)
            c.thr = ("fraction", int(rng.integers(500, 2001)), 10000)
            out.append(c)
        else:
            out.append(stream.pop(0))
    return out


@pytest.fixture(scope="module")
def mix_oracle(orc):
    """The mix and the oracle's filtration of each of its clouds."""
    import concurrent.futures as cf

    clouds = _requests()
    with cf.ThreadPoolExecutor(max_workers=host_threads()) as ex:
        fs = list(ex.map(lambda c: orc.build_mt(c.points, c.thr, 1), clouds))
    return clouds, fs


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


def test_mix_covers_the_serving_shapes(mix_oracle):
    clouds, _ = mix_oracle
    assert {c.d for c in clouds} == {2, 3, 16, 64}
    assert max(c.n for c in clouds) >= 1500 and min(c.n for c in clouds) == 0


@pytest.mark.parametrize("slots,max_batch", [(1, 1), (3, 8), (4, 32)])
def test_served_results_equal_oracle_and_alone(mix_oracle, slots, max_batch):
    """Every served result equals the oracle's filtration of its cloud
    element by element (edges, lengths, every triangle key) and the bytes
    of the same cloud built alone, whatever batch and stream it shared."""
    import torch

    from paper_1809_04424_amd.serve import Server

    clouds, fs = mix_oracle
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
    for c, f, r in zip(clouds, fs, reqs):
        got = item_host(r.item)
        assert_matches_oracle(got, f)
        _same(got, _alone(c))
        r.release()
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


def test_invalid_submissions_do_not_stop_the_loop():
    """A host tensor or an unknown threshold is refused at submission; the
    valid requests around it still complete, and the loop's counters come
    back to zero."""
    import torch

    from paper_1809_04424_amd.serve import Server

    good = [workloads.uniform_cloud(70 + i, 40 + 10 * i, 3) for i in range(3)]
    with Server(slots=2) as srv:
        reqs = [srv.submit(torch.from_numpy(good[0].points).to("cuda:0"), ("fraction", 10, 100))]
        with pytest.raises(TypeError):
            srv.submit(torch.from_numpy(good[1].points), ("fraction", 10, 100))  # host memory
        reqs.append(srv.submit(torch.from_numpy(good[1].points).to("cuda:0"), ("fraction", 10, 100)))
        with pytest.raises(ValueError):
            srv.submit(torch.from_numpy(good[2].points).to("cuda:0"), ("median", 1, 2))
        reqs.append(srv.submit(torch.from_numpy(good[2].points).to("cuda:0"), ("fraction", 10, 100)))
        for r in reqs:
            r.wait(timeout=60)
            r.release()
    for c, r in zip(good, reqs):
        c.thr = ("fraction", 10, 100)
        assert r.counts == _alone(c)["counts"]
    assert srv._held == 0 and srv._reserved == 0 and srv._inflight == 0


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
