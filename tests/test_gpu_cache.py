"""The library's stream-ordered device cache: blocks are reused across
builds and streams without changing any result, and trim releases them."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_matches_oracle, item_host

pytestmark = pytest.mark.gpu


def test_reuse_across_streams_keeps_results(orc):
    import torch

    import paper_1809_04424_amd as vr

    clouds = []
    for i, n in enumerate([300, 40, 700, 120, 700, 300, 5, 900]):
        c = workloads.uniform_cloud(900 + i, n, 3, lo=-50, hi=50)
        c.thr = ("fraction", 15, 100)
        clouds.append(c)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    vr.trim()
    held = []
    for rep in range(3):
        for i, c in enumerate(clouds):
            s = streams[(i + rep) % 2]
            with torch.cuda.stream(s):
                p = torch.from_numpy(c.points).to("cuda:0")
                r = vr.build(p, c.thr)
                out = item_host(r)  # copies on s, then synchronises
                r.free()  # the block returns to the cache in s's order
            assert_matches_oracle(out, orc.build(c.points, c.thr))
        torch.cuda.synchronize()
        held.append(vr.trim())
    assert min(held) > 0
    assert vr.trim() == 0  # nothing cached after a trim


def test_output_memory_survives_other_builds(orc):
    import torch

    import paper_1809_04424_amd as vr

    a = workloads.uniform_cloud(31, 400, 3, lo=-50, hi=50)
    a.thr = ("fraction", 20, 100)
    ra = vr.build(torch.from_numpy(a.points).to("cuda:0"), a.thr)
    for i in range(6):  # builds that take and return blocks while ra holds its outputs
        c = workloads.uniform_cloud(40 + i, 400, 3, lo=-50, hi=50)
        c.thr = ("fraction", 20, 100)
        vr.build(torch.from_numpy(c.points).to("cuda:0"), c.thr).free()
    torch.cuda.synchronize()
    assert_matches_oracle(item_host(ra), orc.build(a.points, a.thr))
    ra.free()
