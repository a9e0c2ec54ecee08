"""Request loop for filtration builds: continuous batching over
vr_build_batch with admission by device-memory footprint.

Requests (a device point cloud plus a threshold) arrive at any time through
``Server.submit``.  ``slots`` worker threads each own a HIP stream.  A free
worker takes the oldest waiting request and, after it in arrival order, the
waiting requests that can share its batch (same coordinate type, dimension,
threshold kind and maxdim), as long as the batch's exact workspace
(vr_batch_workspace_bytes) fits in what the budget has left, and builds them
with one vr_build_batch call.  Requests that arrive while other batches run
are admitted as soon as a worker and memory are free, and the builds of
different workers overlap on the device.  A request's output (16 bytes per
edge, 8 per triangle) is charged against the budget once its counts are known
and released with ``Request.release``.  Every result is bit-identical to a
build of the same cloud alone.

Host scheduling only: every step of a build runs in the library's kernels.
"""
from __future__ import annotations

import collections
import threading
import time

import paper_1809_04424_amd as vr


class Request:
    """One build request; ``wait()`` blocks until its result is on the device."""

    __slots__ = ("rid", "points", "thr", "arrival", "t_start", "t_done", "batch_size", "item", "counts", "error",
                 "out_bytes", "_done", "_server")

    def __init__(self, rid, points, thr, arrival, server):
        self.rid = rid
        self.points = points
        self.thr = thr
        self.arrival = arrival
        self.t_start = self.t_done = None
        self.batch_size = 0
        self.item = None
        self.counts = None
        self.error = None
        self.out_bytes = 0
        self._done = threading.Event()
        self._server = server

    @property
    def key(self):
        p = self.points
        return (p.dtype, int(p.shape[1]), self.thr[0])

    @property
    def shape(self):
        return (int(self.points.shape[0]), int(self.points.shape[1]), vr._dtype_code(self.points), self.thr)

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival

    def wait(self, timeout=None):
        if not self._done.wait(timeout):
            raise TimeoutError(f"request {self.rid} not done")
        if self.error is not None:
            raise self.error
        return self.item

    def release(self):
        """Drop the result and return its output bytes to the budget."""
        if self.item is not None or self.out_bytes:
            self.item = None
            self._server._release_output(self.out_bytes)
            self.out_bytes = 0


def check_request(points, thr):
    """Reject at submission what no build could take: points that are not a
    2-D int8/int16/int32 tensor on a HIP device, or a threshold that is not a
    (kind, num, den) tuple of a known kind.  Raises TypeError or ValueError."""
    import torch

    if not isinstance(points, torch.Tensor) or points.device.type != "cuda":
        raise TypeError("points must be a torch tensor on a HIP device")
    if points.dim() != 2:
        raise ValueError("points must be 2-D (n, d)")
    vr._dtype_code(points)  # TypeError for other dtypes
    if not isinstance(thr, (tuple, list)) or len(thr) != 3 or thr[0] not in vr.VR_THR:
        raise ValueError(f"threshold must be (kind, num, den) with kind in {sorted(vr.VR_THR)}")


def output_bytes(counts) -> int:
    """Device bytes of one result's outputs (as allocated, 256-byte aligned)."""
    _, K, T = counts
    up = lambda x: (x + 255) // 256 * 256  # noqa: E731
    return 2 * up(8 * K) + 8 * T


def take_batch(pending, free_bytes, max_batch, ws_of, limit_of=vr.batch_limit, idle=True):
    """Scheduling policy (pure): the oldest waiting request plus the later
    ones sharing its key, in arrival order, while the batch's workspace
    ``ws_of(batch)`` fits in ``free_bytes``.  Returns (batch, workspace) or
    (None, 0) when even the oldest request does not fit; when nothing else is
    in flight (``idle``) the oldest request is taken alone regardless, so the
    loop cannot stall on a request larger than the budget."""
    if not pending:
        return None, 0
    head = pending[0]
    group = [head]
    ws = ws_of(group)
    if ws > free_bytes:
        return ([head], ws) if idle else (None, 0)
    cap = min(max_batch, limit_of(vr._dtype_code(head.points), int(head.points.shape[1])))
    for r in list(pending)[1:]:
        if len(group) >= cap:
            break
        if r.key != head.key:
            continue
        try:
            w2 = ws_of(group + [r])
        except vr.VrError:  # the batch would exceed a key width: stop here
            break
        if w2 > free_bytes:
            break
        group.append(r)
        ws = w2
    return group, ws


class Server:
    """Continuous-batching request loop on one device.

    slots:        worker threads (each with its own stream): builds in flight.
    max_batch:    most requests per vr_build_batch call.
    budget_bytes: device bytes for workspaces plus held outputs (default: half
                  of the device's free memory at start).
    keep_results: False releases every result as soon as it is complete
                  (measurement runs); True keeps it until Request.release.
    """

    def __init__(self, device="cuda:0", slots=4, max_batch=32, budget_bytes=None, maxdim=2, keep_results=True,
                 clock=time.perf_counter):
        import torch

        self.device = torch.device(device)
        self.maxdim = maxdim
        self.max_batch = max_batch
        self.keep = keep_results
        self.clock = clock
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = free // 2
        self.budget = int(budget_bytes)
        self._pending = collections.deque()
        self._cv = threading.Condition()
        self._reserved = 0  # workspaces of batches in flight
        self._held = 0      # outputs of finished requests not yet released
        self._inflight = 0
        self._stop = False
        self._next = 0
        self.peak_bytes = 0
        self.batches = 0
        self._workers = [threading.Thread(target=self._work, name=f"vr-slot{i}", daemon=True) for i in range(slots)]
        for t in self._workers:
            t.start()

    # ---------------------------------------------------------------- API --
    def submit(self, points, thr, arrival=None) -> Request:
        """Queue one build.  Raises TypeError/ValueError at once for a request
        no build could take (see check_request); a request the library
        rejects later fails alone (its wait() raises)."""
        check_request(points, thr)
        with self._cv:
            r = Request(self._next, points, thr, self.clock() if arrival is None else arrival, self)
            self._next += 1
            self._pending.append(r)
            self._cv.notify()
        return r

    def close(self):
        """Finish every submitted request, then stop the workers."""
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for t in self._workers:
            t.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---------------------------------------------------------- internals --
    def _ws_of(self, group):
        return vr.batch_workspace_bytes([r.shape for r in group], self.maxdim)

    def _release_output(self, nbytes):
        with self._cv:
            self._held -= nbytes
            self._cv.notify_all()

    def _take(self):
        while self._pending:  # a request the library rejects fails alone, at once
            head = self._pending[0]
            try:
                self._ws_of([head])
                break
            except Exception as e:  # noqa: BLE001 -- any rejection fails this request only
                self._pending.popleft()
                head.error = e
                head.t_done = self.clock()
                head._done.set()
        free = self.budget - self._reserved - self._held
        group, ws = take_batch(self._pending, free, self.max_batch, self._ws_of, idle=self._inflight == 0)
        if group is None:
            return None, 0
        for r in group:
            self._pending.remove(r)
        self._reserved += ws
        self._inflight += 1
        self.peak_bytes = max(self.peak_bytes, self._reserved + self._held)
        return group, ws

    def _work(self):
        import torch

        stream = torch.cuda.Stream(self.device)
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            while True:
                with self._cv:
                    while True:
                        group, ws = self._take()
                        if group is not None or (self._stop and not self._pending):
                            break
                        self._cv.wait()
                    if group is None:
                        self._cv.notify_all()
                        return
                self._run(group, ws, stream)

    def _run(self, group, ws, stream):
        t0 = self.clock()
        err, items, b = None, None, None
        try:
            try:
                b = vr.build_batch([r.points for r in group], [r.thr for r in group], maxdim=self.maxdim)
                stream.synchronize()
                items = list(b)
            except Exception as e:  # noqa: BLE001 -- the group fails, the loop goes on
                err = e
            t1 = self.clock()
            charged = 0
            with self._cv:
                self.batches += 1
                for i, r in enumerate(group):
                    r.t_start, r.t_done, r.batch_size = t0, t1, len(group)
                    if err is not None:
                        r.error = err
                        continue
                    r.counts = items[i].counts
                    if self.keep:
                        r.item = items[i]
                        r.out_bytes = output_bytes(r.counts)
                        charged += r.out_bytes
                self._held += charged
            if not self.keep and b is not None:
                items = None
                b.free()
        finally:
            # the workspace and the slot come back whatever happened, and
            # every request of the group is released to its waiter
            with self._cv:
                self._reserved -= ws
                self._inflight -= 1
                self.peak_bytes = max(self.peak_bytes, self._reserved + self._held)
                self._cv.notify_all()
            for r in group:
                if r.t_done is None:
                    r.t_start, r.t_done, r.batch_size = t0, self.clock(), len(group)
                    if r.error is None and r.counts is None:
                        r.error = RuntimeError("build did not complete")
                r._done.set()
