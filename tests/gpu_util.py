"""Helpers for tests that call the HIP library through its Python binding."""
from __future__ import annotations

import numpy as np


def decode_keys(keys) -> np.ndarray:
    """Packed triangle keys (v<<39 | i<<26 | j<<13 | k) -> (T, 4) rows (v, i, j, k)."""
    k = np.asarray(keys).astype(np.int64).view(np.uint64)
    m13 = np.uint64(0x1FFF)
    return np.stack([k >> np.uint64(39), (k >> np.uint64(26)) & m13, (k >> np.uint64(13)) & m13, k & m13],
                    axis=1).astype(np.int64)


def gpu_build(cloud, maxdim=2, count_only=False, timing=False, device="cuda:0", allocator="library"):
    """Run one build on the GPU; returns (result, host dict of numpy arrays)."""
    import torch

    import paper_1809_04424_amd as vr

    pts = torch.from_numpy(np.ascontiguousarray(cloud.points)).to(device)
    res = vr.build(pts, cloud.thr, maxdim=maxdim, count_only=count_only, timing=timing, allocator=allocator)
    torch.cuda.synchronize()
    out = {
        "counts": res.counts,
        "edge_ij": res.edge_ij().cpu().numpy().astype(np.int64),
        "edge_q": res.edge_q().cpu().numpy(),
        "tri": res.tri_key().cpu().numpy(),
    }
    return res, out


def assert_matches_oracle(out, f, check_tri=True):
    """Bit-exact comparison of a GPU build with an oracle Filtration."""
    assert tuple(out["counts"]) == (f.n, f.K, f.T)
    assert np.array_equal(out["edge_ij"][:, 0], f.ei)
    assert np.array_equal(out["edge_ij"][:, 1], f.ej)
    assert np.array_equal(out["edge_q"], f.eq)
    if check_tri:
        got = decode_keys(out["tri"])
        assert got.shape == f.tris.shape
        assert np.array_equal(got, f.tris)


def item_host(item):
    """Host copies of one result's arrays (a Result or a batch item)."""
    return {
        "counts": item.counts,
        "edge_ij": item.edge_ij().cpu().numpy().astype(np.int64),
        "edge_q": item.edge_q().cpu().numpy(),
        "tri": item.tri_key().cpu().numpy(),
    }


def gpu_build_batch(clouds, maxdim=2, count_only=False, device="cuda:0", allocator="library"):
    """One batched build of `clouds` (one threshold kind); returns (batch, [host dicts])."""
    import torch

    import paper_1809_04424_amd as vr

    pts = [torch.from_numpy(np.ascontiguousarray(c.points)).to(device) for c in clouds]
    b = vr.build_batch(pts, [c.thr for c in clouds], maxdim=maxdim, count_only=count_only, allocator=allocator)
    torch.cuda.synchronize()
    return b, [item_host(it) for it in b]


def host_threads() -> int:
    """Host threads for the oracle: the CPU share of one GPU (16), or fewer."""
    import os

    return max(1, min(16, os.cpu_count() or 1))


def pack_rows(rows) -> np.ndarray:
    """Oracle rows (v, i, j, k) in the device's key layout (uint64); one to
    one while v < 2^24 and i, j, k < 2^13, so equal keys mean equal rows."""
    t = np.asarray(rows, dtype=np.int64).astype(np.uint64).reshape(-1, 4)
    return (t[:, 0] << np.uint64(39)) | (t[:, 1] << np.uint64(26)) | (t[:, 2] << np.uint64(13)) | t[:, 3]


def assert_keys_match_oracle(keys, f, orc, threads=None, chunk=1 << 16):
    """Every triangle key of a device result (host uint64 array) against the
    oracle's triangles, listed value range by value range so that the host
    never holds the whole oracle list at once."""
    threads = threads or host_threads()
    keys = np.asarray(keys).view(np.uint64)
    pos = 0
    for r0 in range(0, f.K, chunk):
        r1 = min(f.K, r0 + chunk)
        want = pack_rows(orc.triangles_by_value(f, r0, r1, threads))
        got = keys[pos: pos + len(want)]
        assert len(got) == len(want), f"values [{r0}, {r1}): {len(got)} keys, oracle {len(want)}"
        if not np.array_equal(got, want):
            bad = int(np.nonzero(got != want)[0][0])
            raise AssertionError(f"values [{r0}, {r1}): key {pos + bad} differs "
                                 f"(device {int(got[bad]):#x}, oracle {int(want[bad]):#x})")
        pos += len(want)
    assert pos == len(keys), f"device lists {len(keys)} triangles, oracle {pos}"
