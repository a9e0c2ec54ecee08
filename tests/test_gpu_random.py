"""Seeded random cases against the oracle: clouds of random size, dimension,
coordinate type and threshold, built under a random enumeration schedule
(the write with one wave per vertex and eighth included), bit-exact; and
for the smaller ones the whole chain to barcodes (maxdim 2 or 3)."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import assert_matches_oracle, gpu_build

pytestmark = pytest.mark.gpu

SCHEDULES = [(eb_c, p_c, np_c, eb_w, p_w, np_w)
             for eb_c in (128, 256, 512) for p_c in (1, 2, 8) for np_c in (2, 4, 8)
             for eb_w in (128, 256, 512) for p_w in (0, 1, 2, 8, 16) for np_w in (4, 8)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1809_04424_amd as vr

    vr.lib()
    yield


def _case(seed):
    """(cloud, schedule) of case `seed`: the draws depend on the seed alone."""
    rng = np.random.default_rng(10_000 + seed)
    n = int(rng.choice([0, 1, 2, 3, 5, 8, 13, 40, 64, 65, 127, 200, 333, 513, 700]))
    d = int(rng.choice([1, 2, 3, 5, 16, 37, 64, 100]))
    kind = rng.integers(0, 3)
    if kind == 0:
        dtype, lo, hi = np.int8, -128, 127
    elif kind == 1:
        dtype, lo, hi = np.int16, -300, 300
    else:
        dtype, lo, hi = np.int32, -1000, 1000
    if rng.random() < 0.3:  # coarse coordinates: many equal distances
        lo, hi = -3, 3
    pts = rng.integers(lo, hi + 1, (n, d)).astype(dtype)
    pairs = n * (n - 1) // 2
    t = rng.integers(0, 4)
    if t == 0 and n <= 80:
        thr = ("full", 0, 1)
    elif t == 1:
        thr = ("count", int(rng.integers(0, pairs + 1)), 1)
    elif t == 2:
        thr = ("sqdist", int(rng.integers(0, 4 * d * (hi - lo) ** 2 // 10 + 2)), 0)
    else:
        thr = ("fraction", int(rng.integers(1, 40)), 100)
    sched = SCHEDULES[int(rng.integers(0, len(SCHEDULES)))]
    return workloads.Cloud(pts, thr), sched


@pytest.mark.parametrize("seed", range(120))
def test_random_build_bit_exact(orc, seed):
    import torch

    import paper_1809_04424_amd as vr

    c, sched = _case(seed)
    print(f"[gpu] random case {seed}: n={c.points.shape[0]} d={c.points.shape[1]} {c.points.dtype} "
          f"thr={c.thr} sched={sched}", flush=True)
    if c.points.shape[0] >= 2:
        vr.set_schedule(torch.from_numpy(np.ascontiguousarray(c.points)).to("cuda:0"), c.thr, sched)
    _, out = gpu_build(c)
    assert_matches_oracle(out, orc.build(c.points, c.thr))


@pytest.mark.parametrize("seed", range(40))
def test_random_barcodes(orc, seed):
    import torch

    import paper_1809_04424_amd as vr

    c, _ = _case(100 + seed)
    maxdim = 2 + seed % 2
    pts = c.points[: min(len(c.points), 90 if maxdim == 2 else 50)]
    thr = c.thr
    if thr[0] == "count":  # at most the pairs of the points kept
        thr = ("count", min(thr[1], len(pts) * (len(pts) - 1) // 2), 1)
    c = workloads.Cloud(pts, thr)
    print(f"[gpu] random barcodes {seed}: n={len(pts)} d={pts.shape[1]} thr={c.thr} maxdim={maxdim}", flush=True)
    out = vr.persistence(torch.from_numpy(np.ascontiguousarray(pts)).to("cuda:0"), c.thr, maxdim=maxdim)
    f = orc.build(pts, c.thr)
    p = orc.reduce(f, "cohomology")
    if maxdim == 3:
        tets = orc.tetra_list(f)
        want = orc.barcode(f, orc.with_dim2(f, p, tets), tets)
    else:
        want = orc.barcode(f, p)
    got = sorted(tuple(int(x) for x in b) for b in out["bars"].cpu().numpy())
    assert got == sorted(b for b in want if b[0] < maxdim)
    assert out["essential_top"] == sum(1 for b in want if b[0] == maxdim)
