"""The request loop's scheduling policy (host only, no GPU)."""
import collections

import pytest
import torch

from paper_1809_04424_amd import serve


class _R:
    def __init__(self, n, d, kind="fraction", dtype=torch.int8):
        self.points = torch.zeros((n, d), dtype=dtype)
        self.thr = (kind, 10, 100)

    key = serve.Request.key


def _ws(group):
    return sum(r.points.shape[0] for r in group)


def test_oldest_first_and_same_key_only():
    q = collections.deque([_R(10, 3), _R(20, 16), _R(30, 3), _R(40, 3, "count")])
    g, ws = serve.take_batch(q, 1000, 8, _ws)
    assert [r.points.shape[0] for r in g] == [10, 30] and ws == 40


def test_budget_stops_the_batch_in_arrival_order():
    q = collections.deque([_R(10, 3), _R(50, 3), _R(5, 3)])
    g, ws = serve.take_batch(q, 40, 8, _ws)
    assert [r.points.shape[0] for r in g] == [10] and ws == 10  # no overtaking past a request that does not fit


def test_head_larger_than_budget_waits_unless_idle():
    q = collections.deque([_R(100, 3), _R(5, 3)])
    assert serve.take_batch(q, 50, 8, _ws, idle=False) == (None, 0)
    g, ws = serve.take_batch(q, 50, 8, _ws, idle=True)
    assert len(g) == 1 and ws == 100


def test_batch_caps():
    q = collections.deque([_R(3, 3) for _ in range(20)])
    g, _ = serve.take_batch(q, 10 ** 9, 8, _ws)
    assert len(g) == 8
    q16 = collections.deque([_R(3, 3, dtype=torch.int16) for _ in range(4)])
    g, _ = serve.take_batch(q16, 10 ** 9, 8, _ws)
    assert len(g) == 1  # 32-bit squared distances leave no bits for a cloud index
    assert serve.take_batch(collections.deque(), 10, 8, _ws) == (None, 0)


def test_output_bytes():
    assert serve.output_bytes((10, 0, 0)) == 0
    assert serve.output_bytes((10, 1, 3)) == 2 * 256 + 24
    assert serve.output_bytes((10, 32, 0)) == 2 * 256
    assert serve.output_bytes((10, 33, 0)) == 2 * 512


@pytest.mark.parametrize("n", [0, 5])
def test_workspace_of_requests(n):
    r = _R(n, 3)
    w = __import__("paper_1809_04424_amd").batch_workspace_bytes([(n, 3, 1, r.thr)])
    assert (w == 0) == (n < 2)


@pytest.mark.parametrize("points,thr,exc", [
    (torch.zeros((5, 3), dtype=torch.int8), ("fraction", 10, 100), TypeError),      # host tensor
    ("not a tensor", ("fraction", 10, 100), TypeError),
    (torch.zeros((5, 3), dtype=torch.float32), ("fraction", 10, 100), TypeError),  # checked after the device
    (torch.zeros(5, dtype=torch.int8), ("fraction", 10, 100), TypeError),
    (torch.zeros((5, 3), dtype=torch.int8), ("median", 1, 2), TypeError),
])
def test_submit_rejects_what_no_build_takes(points, thr, exc):
    """Host tensors, other types and unknown threshold kinds are refused at
    submission (before they could reach a worker thread)."""
    with pytest.raises(exc):
        serve.check_request(points, thr)


def test_check_request_thresholds_without_gpu(monkeypatch):
    """With the device test bypassed, the shape, dtype and threshold checks
    still apply in that order."""
    class _Dev:
        type = "cuda"

    class _T(torch.Tensor):
        pass

    t = torch.zeros((5, 3), dtype=torch.int8).as_subclass(_T)
    monkeypatch.setattr(_T, "device", property(lambda self: _Dev()))
    serve.check_request(t, ("fraction", 10, 100))
    for bad in [("median", 1, 2), ("fraction", 1), "full", None]:
        with pytest.raises(ValueError):
            serve.check_request(t, bad)
    t1 = torch.zeros(5, dtype=torch.int8).as_subclass(_T)
    with pytest.raises(ValueError):
        serve.check_request(t1, ("fraction", 10, 100))
    tf = torch.zeros((5, 3), dtype=torch.float32).as_subclass(_T)
    with pytest.raises(TypeError):
        serve.check_request(tf, ("fraction", 10, 100))
