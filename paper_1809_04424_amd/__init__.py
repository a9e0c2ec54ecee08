"""Python binding of the gfx950 Vietoris-Rips filtration library (libvrhip.so).

Argument marshalling only: every step of the build runs in the library's HIP
kernels.  PyTorch supplies device memory (through the library's allocator
hook, so outputs are ordinary torch tensors) and the stream.  There is no CPU
fallback: importing works without the library, but every call raises until
``make_lib.py`` has produced ``libvrhip.so``.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvrhip.so")

VR_OK, VR_EINVAL, VR_ENOMEM, VR_E2BIG, VR_EHIP, VR_ERANGE = 0, -1, -2, -3, -4, -5
VR_I8, VR_I16, VR_I32, VR_DIST = 1, 2, 3, 4
VR_THR = {"full": 0, "count": 1, "fraction": 2, "sqdist": 3}
VR_COUNT_ONLY, VR_TIMING, VR_TIMING_WRITE, VR_GRAPH = 1, 2, 4, 8
VR_MAX_POINTS = 8192
VR_MAX_EDGES = 1 << 24

# C symbols declared in include/vr.h
SYMBOLS = ("vr_build", "vr_query_counts", "vr_unpack_triangles", "vr_query_stage_ms", "vr_stage_name", "vr_free",
           "vr_workspace_bytes", "vr_batch_workspace_bytes", "vr_build_batch", "vr_batch_result", "vr_batch_stage_ms", "vr_batch_free", "vr_autotune", "vr_set_schedule", "vr_trim", "vr_column_order", "vr_column_order_noalloc", "vr_pairs_dim0", "vr_pairs_dim1_apparent", "vr_pairs_dim1", "vr_barcode", "vr_tetra_counts", "vr_tetra_offsets", "vr_tetra_write", "vr_pairs_dim2", "vr_barcode_dim2", "vr_blockprodsum_count", "vr_blockprodsum_write",
           "vr_status_string", "vr_version")

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class VrAllocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class VrRequest(ctypes.Structure):
    _fields_ = [
        ("points", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("d", ctypes.c_int64),
        ("dtype", ctypes.c_int32),
        ("thr_kind", ctypes.c_int32),
        ("thr_num", ctypes.c_int64),
        ("thr_den", ctypes.c_int64),
        ("maxdim", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("alloc", ctypes.POINTER(VrAllocator)),
    ]


class VrResult(ctypes.Structure):
    _fields_ = [
        ("n_vertices", ctypes.c_int64),
        ("n_edges", ctypes.c_int64),
        ("n_triangles", ctypes.c_int64),
        ("edge_ij", ctypes.c_void_p),
        ("edge_q", ctypes.c_void_p),
        ("tri_key", ctypes.c_void_p),
        ("n_tetrahedra", ctypes.c_int64),
        ("tet_off", ctypes.c_void_p),
        ("tet_key", ctypes.c_void_p),
    ]


class VrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None
_lock = threading.Lock()


def lib():
    """The loaded libvrhip.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1809_04424_amd/make_lib.py (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        L.vr_build.argtypes = [ctypes.POINTER(VrRequest), ctypes.c_void_p, ctypes.POINTER(ctypes.POINTER(VrResult))]
        L.vr_build.restype = ctypes.c_int
        L.vr_query_counts.argtypes = [ctypes.POINTER(VrResult), ctypes.POINTER(ctypes.c_int64)]
        L.vr_query_counts.restype = ctypes.c_int
        L.vr_query_stage_ms.argtypes = [ctypes.POINTER(VrResult), ctypes.POINTER(ctypes.c_float), ctypes.c_int]
        L.vr_query_stage_ms.restype = ctypes.c_int
        L.vr_stage_name.argtypes = [ctypes.c_int]
        L.vr_stage_name.restype = ctypes.c_char_p
        L.vr_free.argtypes = [ctypes.POINTER(VrResult), ctypes.c_void_p]
        L.vr_free.restype = None
        L.vr_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
        L.vr_workspace_bytes.restype = ctypes.c_int64
        L.vr_batch_workspace_bytes.argtypes = [ctypes.POINTER(VrRequest), ctypes.c_int64]
        L.vr_batch_workspace_bytes.restype = ctypes.c_int64
        L.vr_build_batch.argtypes = [ctypes.POINTER(VrRequest), ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_void_p)]
        L.vr_build_batch.restype = ctypes.c_int
        L.vr_batch_result.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(VrResult)]
        L.vr_batch_result.restype = ctypes.c_int
        L.vr_batch_stage_ms.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int]
        L.vr_batch_stage_ms.restype = ctypes.c_int
        L.vr_batch_free.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.vr_batch_free.restype = None
        L.vr_unpack_triangles.argtypes = [ctypes.POINTER(VrResult), ctypes.c_void_p, ctypes.c_void_p]
        L.vr_unpack_triangles.restype = ctypes.c_int
        L.vr_autotune.argtypes = [ctypes.POINTER(VrRequest), ctypes.c_int64, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_int32)]
        L.vr_autotune.restype = ctypes.c_int
        L.vr_set_schedule.argtypes = [ctypes.POINTER(VrRequest), ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]
        L.vr_set_schedule.restype = ctypes.c_int
        L.vr_column_order.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_void_p]
        L.vr_column_order.restype = ctypes.c_int
        L.vr_column_order_noalloc.argtypes = L.vr_column_order.argtypes
        L.vr_column_order_noalloc.restype = ctypes.c_int
        L.vr_pairs_dim0.argtypes = [ctypes.POINTER(VrResult), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.vr_pairs_dim0.restype = ctypes.c_int
        L.vr_pairs_dim1_apparent.argtypes = [ctypes.POINTER(VrResult), ctypes.c_void_p, ctypes.c_void_p]
        L.vr_pairs_dim1_apparent.restype = ctypes.c_int
        L.vr_pairs_dim1.argtypes = [ctypes.POINTER(VrResult), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.vr_pairs_dim1.restype = ctypes.c_int
        L.vr_pairs_dim2.argtypes = [ctypes.POINTER(VrResult), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.vr_pairs_dim2.restype = ctypes.c_int
        L.vr_barcode_dim2.argtypes = [ctypes.POINTER(VrResult), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
        L.vr_barcode_dim2.restype = ctypes.c_int
        L.vr_barcode.argtypes = [ctypes.POINTER(VrResult), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
        L.vr_barcode.restype = ctypes.c_int
        L.vr_tetra_counts.argtypes = [ctypes.POINTER(VrResult), ctypes.c_void_p, ctypes.c_void_p]
        L.vr_tetra_counts.restype = ctypes.c_int
        L.vr_tetra_offsets.argtypes = [ctypes.POINTER(VrResult), ctypes.c_void_p, ctypes.c_void_p]
        L.vr_tetra_offsets.restype = ctypes.c_int
        L.vr_tetra_write.argtypes = [ctypes.POINTER(VrResult), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p]
        L.vr_tetra_write.restype = ctypes.c_int
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        L.vr_blockprodsum_count.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.vr_blockprodsum_count.restype = ctypes.c_int
        L.vr_blockprodsum_write.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.vr_blockprodsum_write.restype = ctypes.c_int
        L.vr_trim.argtypes = []
        L.vr_trim.restype = ctypes.c_int64
        L.vr_status_string.argtypes = [ctypes.c_int]
        L.vr_status_string.restype = ctypes.c_char_p
        L.vr_version.argtypes = []
        L.vr_version.restype = ctypes.c_int
        _lib = L
    return _lib


def trim() -> int:
    """Release the library's cached device blocks not in use (current device)."""
    return int(lib().vr_trim())


def status_string(code: int) -> str:
    return lib().vr_status_string(code).decode()


def stage_names():
    L = lib()
    out, s = [], 0
    while True:
        p = L.vr_stage_name(s)
        if not p:
            return out
        out.append(p.decode())
        s += 1


def workspace_bytes(n: int, d: int, dtype: int = VR_I8, thr_kind: str = "fraction") -> int:
    return int(lib().vr_workspace_bytes(n, d, dtype, VR_THR[thr_kind]))


def batch_workspace_bytes(shapes, maxdim: int = 2) -> int:
    """Exact workspace of build_batch over clouds given as (n, d, dtype, thr)
    tuples (no device memory needed); raises VrError for rejected shapes."""
    reqs = (VrRequest * len(shapes))()
    for r, (n, d, dtype, thr) in zip(reqs, shapes):
        kind, num, den = thr
        r.points, r.n, r.d, r.dtype = (16 if n else None), n, d, dtype
        r.thr_kind, r.thr_num, r.thr_den, r.maxdim, r.flags = VR_THR[kind], int(num), int(den), maxdim, 0
    v = int(lib().vr_batch_workspace_bytes(reqs, len(shapes)))
    if v < 0:
        raise VrError(v, status_string(v))
    return v


class _TorchAllocator:
    """Allocator hook: the library's device memory comes from torch's caching
    allocator on the build's stream, so outputs are torch tensors."""

    def __init__(self, device):
        self.device = device
        self.live = {}
        self._a = _ALLOC_FN(self._alloc)
        self._f = _FREE_FN(self._free)
        self.struct = VrAllocator(self._a, self._f, None)

    def _alloc(self, nbytes, stream, ctx):
        import torch

        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except Exception:  # out of memory: the library reports VR_ENOMEM
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free(self, ptr, nbytes, stream, ctx):
        self.live.pop(ptr, None)


_allocators = {}


def _allocator_for(device):
    a = _allocators.get(device)
    if a is None:
        a = _allocators[device] = _TorchAllocator(device)
    return a


def _dtype_code(t):
    import torch

    m = {torch.int8: VR_I8, torch.int16: VR_I16, torch.int32: VR_I32}
    if t.dtype not in m:
        raise TypeError("points must be int8, int16 or int32")
    return m[t.dtype]


class _DeviceArray:
    """Zero-copy view of library-owned device memory for torch.as_tensor;
    holds the owning Result so the memory outlives every tensor made from it."""

    def __init__(self, owner, ptr, shape, typestr):
        self._owner = owner
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 2, "strides": None}


class _Arrays:
    """Counts and device arrays of one cloud's filtration (a vr_result view)."""

    def _init_arrays(self, r, device, block=None, block_ptr=0, alloc=None):
        self._device = device
        self.n, self.K, self.T = int(r.n_vertices), int(r.n_edges), int(r.n_triangles)
        self._p_q, self._p_ij, self._p_tri = r.edge_q, r.edge_ij, r.tri_key
        self._block, self._block_ptr = block, block_ptr
        # maxdim 3: the tetrahedra, in blocks of their own
        self.T3 = int(r.n_tetrahedra)
        self._p_toff, self._p_tkey = r.tet_off, r.tet_key
        self._tet_blocks = {}
        if alloc is not None:
            for p in (r.tet_off, r.tet_key):
                if p and p in alloc.live:
                    self._tet_blocks[p] = alloc.live[p]

    @property
    def counts(self):
        return (self.n, self.K, self.T)

    def _tensor(self, ptr, count, dtype, typestr, itemsize, shape):
        import torch

        if not ptr or count == 0:  # nothing written (count-only build) or empty
            return torch.empty((0,) + tuple(shape[1:]), dtype=dtype, device=self._device)
        if self._block is not None:  # torch-allocated block
            off = ptr - self._block_ptr
            return self._block[off: off + count * itemsize].view(dtype).view(shape)
        return torch.as_tensor(_DeviceArray(self, ptr, shape, typestr), device=self._device)

    def edge_q(self):
        """int64 (K,) squared lengths of the kept edges in rank order."""
        import torch

        return self._tensor(self._p_q, self.K, torch.int64, "<i8", 8, (self.K,))

    def edge_ij(self):
        """int32 (K, 2) endpoints i < j of the kept edges in rank order."""
        import torch

        return self._tensor(self._p_ij, 2 * self.K, torch.int32, "<i4", 4, (self.K, 2))

    def tri_key(self):
        """int64 (T,) packed triangle keys v<<39 | i<<26 | j<<13 | k, ascending."""
        import torch

        return self._tensor(self._p_tri, self.T, torch.int64, "<i8", 8, (self.T,))

    def _c_result(self):
        """This view as a vr_result (for calls that take one)."""
        return VrResult(self.n, self.K, self.T, self._p_ij, self._p_q, self._p_tri, self.T3, self._p_toff,
                        self._p_tkey)

    def _tet_tensor(self, ptr, count, shape):
        import torch

        if not ptr or count == 0:
            return torch.empty((0,) + tuple(shape[1:]), dtype=torch.int64, device=self._device)
        blk = self._tet_blocks.get(ptr)
        if blk is not None:  # torch-allocated block
            return blk[: count * 8].view(torch.int64).view(shape)
        return torch.as_tensor(_DeviceArray(self, ptr, shape, "<i8"), device=self._device)

    def tet_off(self):
        """int64 (K + 1,) of a maxdim-3 build: tet_off[r] = the first
        tetrahedron of value r, tet_off[K] = T3 (empty otherwise)."""
        return self._tet_tensor(self._p_toff, self.K + 1 if self._p_toff else 0, (self.K + 1,))

    def tet_key(self):
        """int64 (T3, 2) of a maxdim-3 build: rows (value, a<<39 | b<<26 |
        c<<13 | d), a<b<c<d, in filtration order (empty otherwise)."""
        return self._tet_tensor(self._p_tkey, 2 * self.T3, (self.T3, 2))

    def triangles(self):
        """int32 (T, 4) rows (i, j, k, v) in filtration order, unpacked on the device."""
        import torch

        rows = torch.empty((self.T, 4), dtype=torch.int32, device=self._device)
        if self.T == 0:
            return rows
        r = VrResult(self.n, self.K, self.T, self._p_ij, self._p_q, self._p_tri)
        stream = torch.cuda.current_stream(self._device)
        rc = lib().vr_unpack_triangles(ctypes.byref(r), ctypes.c_void_p(rows.data_ptr()),
                                       ctypes.c_void_p(stream.cuda_stream))
        if rc != VR_OK:
            raise VrError(rc, status_string(rc))
        return rows


def _stage_dict(fn, handle):
    buf = (ctypes.c_float * 32)()
    k = fn(handle, buf, 32)
    if k < 0:
        raise VrError(k, status_string(k))
    return dict(zip(stage_names(), list(buf)[:k]))


class Result(_Arrays):
    """Handle of one build.  Device arrays are torch tensors over the
    library's output block; they stay valid while any of them is referenced."""

    def __init__(self, ptr, alloc, stream, device):
        self._ptr = ptr
        self._alloc = alloc
        self._stream = stream
        r = ptr.contents
        blk = alloc.live.get(r.edge_q) if (alloc is not None and r.edge_q) else None
        self._init_arrays(r, device, blk, r.edge_q or 0, alloc)

    def stage_ms(self):
        """{stage: ms} of a build made with timing=True."""
        return _stage_dict(lib().vr_query_stage_ms, self._ptr)

    def free(self):
        if self._ptr is not None:
            lib().vr_free(self._ptr, self._stream)
            self._ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class BatchItem(_Arrays):
    """One cloud of a batch: a view into the batch's output block."""

    def __init__(self, batch, r, device, block, block_ptr):
        self._batch = batch  # library-owned memory lives as long as the batch
        self._init_arrays(r, device, block, block_ptr)


class Batch:
    """Handle of one batched build; batch[i] is the result of request i."""

    def __init__(self, ptr, alloc, stream, device, count):
        self._ptr = ptr
        self._alloc = alloc
        self._stream = stream
        L = lib()
        views = []
        for i in range(count):
            r = VrResult()
            rc = L.vr_batch_result(ptr, i, ctypes.byref(r))
            if rc != VR_OK:
                raise VrError(rc, status_string(rc))
            views.append(r)
        blk, base = None, 0
        if alloc is not None:  # the view whose edges start the block
            for r in views:
                if r.edge_q and r.edge_q in alloc.live:
                    blk, base = alloc.live[r.edge_q], r.edge_q
                    break
        self.items = [BatchItem(self, r, device, blk, base) for r in views]

    def __len__(self):
        return len(self.items)

    def __getitem__(self, i):
        return self.items[i]

    def __iter__(self):
        return iter(self.items)

    def stage_ms(self):
        """{stage: ms} of a batch built with timing=True."""
        return _stage_dict(lib().vr_batch_stage_ms, self._ptr)

    def free(self):
        if self._ptr is not None:
            lib().vr_batch_free(self._ptr, self._stream)
            self._ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _flags(count_only, timing, graph=False):
    return ((VR_COUNT_ONLY if count_only else 0) | (VR_TIMING_WRITE if timing == "write" else
                                                    VR_TIMING if timing else 0) |
            (VR_GRAPH if graph else 0))


def _request(pts, thr, maxdim, flags, alloc, matrix=False):
    kind, num, den = thr
    return VrRequest(
        points=pts.data_ptr() if pts.numel() else None,
        n=pts.shape[0],
        d=pts.shape[1] if pts.shape[0] or not matrix else 1,
        dtype=VR_DIST if matrix else _dtype_code(pts),
        thr_kind=VR_THR[kind],
        thr_num=int(num),
        thr_den=int(den),
        maxdim=int(maxdim),
        flags=flags,
        alloc=ctypes.pointer(alloc.struct) if alloc is not None else None,
    )


def _check_points(points):
    import torch

    if not isinstance(points, torch.Tensor) or points.device.type != "cuda":
        raise TypeError("points must be a torch tensor on a HIP device")
    if points.dim() != 2:
        raise ValueError("points must be 2-D (n, d)")
    return points.contiguous()


def autotune(points, thr, maxdim: int = 2, matrix: bool = False):
    """Tune the triangle kernels' schedule for the size class of these clouds
    (one tensor or a list, as build_batch; matrix=True: one dissimilarity
    matrix, as build_matrix); returns (count block size, count work-groups
    per vertex, count pieces, write block size, write work-groups per vertex,
    write pieces), which later builds of the class use.  Outputs do not
    depend on it."""
    import torch

    L = lib()
    pts = [_check_points(p) for p in (points if isinstance(points, (list, tuple)) else [points])]
    thrs = list(thr) if isinstance(thr, list) else [thr] * len(pts)
    dev = pts[0].device
    stream = torch.cuda.current_stream(dev)
    reqs = (VrRequest * len(pts))(*[_request(p, t, maxdim, 0, None, matrix) for p, t in zip(pts, thrs)])
    sched = (ctypes.c_int32 * 6)()
    with torch.cuda.device(dev):
        rc = L.vr_autotune(reqs, len(pts), ctypes.c_void_p(stream.cuda_stream), sched)
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return tuple(int(x) for x in sched)


def set_schedule(points, thr, sched, maxdim: int = 2, matrix: bool = False):
    """Pin the triangle kernels' schedule (the 6-tuple autotune returns) for
    the size class of these clouds, without tuning."""
    L = lib()
    pts = [_check_points(p) for p in (points if isinstance(points, (list, tuple)) else [points])]
    thrs = list(thr) if isinstance(thr, list) else [thr] * len(pts)
    reqs = (VrRequest * len(pts))(*[_request(p, t, maxdim, 0, None, matrix) for p, t in zip(pts, thrs)])
    arr = (ctypes.c_int32 * 6)(*[int(x) for x in sched])
    rc = L.vr_set_schedule(reqs, len(pts), arr)
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))


def batch_limit(dtype: int, d: int) -> int:
    """Most clouds one batch of this coordinate type and dimension may hold:
    the sort key keeps the cloud index above a squared distance in 32 bits."""
    if dtype != VR_I8:
        return 1
    qbits = (65025 * int(d)).bit_length()
    return 1 << max(0, 32 - qbits)


def build(points, thr=("full", 0, 1), maxdim: int = 2, count_only: bool = False, timing=False,
          allocator: str = "library", graph: bool = False) -> Result:
    """Build the Vietoris-Rips filtration (dim <= maxdim) of a device point cloud.
    maxdim 3 also lists the tetrahedra (Result.tet_off, Result.tet_key).

    points:    torch tensor on a HIP device, (n, d) int8/int16/int32, rows are points.
    thr:       ("full", 0, 1) | ("count", K, 1) | ("fraction", num, den) | ("sqdist", tau, 0).
    allocator: "library" (the library's stream-ordered cache) or "torch" (torch's
               caching allocator through the library's allocator hook).
    timing:    True: HIP events between all stages; "write": around the
               triangle write only (see Result.stage_ms).
    graph:     capture the first phase into a hipGraph on the first build of
               this request (points pointer, size, threshold) on this thread
               and replay it on later ones (not with timing=True).
    The work runs on torch's current stream of the points' device.
    """
    import torch

    L = lib()
    pts = _check_points(points)
    alloc = _allocator_for(pts.device) if allocator == "torch" else None
    stream = torch.cuda.current_stream(pts.device)
    req = _request(pts, thr, maxdim, _flags(count_only, timing, graph), alloc)
    out = ctypes.POINTER(VrResult)()
    with torch.cuda.device(pts.device):
        rc = L.vr_build(ctypes.byref(req), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(out))
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return Result(out, alloc, ctypes.c_void_p(stream.cuda_stream), pts.device)


def build_matrix(dist, thr=("full", 0, 1), maxdim: int = 2, count_only: bool = False, timing=False,
                 allocator: str = "library") -> Result:
    """As build, from a dissimilarity matrix instead of points.

    dist: torch int32 tensor (n, n) on a HIP device, entries >= 0; entry
          [i][j] with i < j is the squared distance of the pair (entries on
          and below the diagonal are not read).  thr as for build ("sqdist"
          compares the entries).
    """
    import torch

    L = lib()
    m = _check_points(dist)
    if m.dtype != torch.int32 or m.shape[0] != m.shape[1]:
        raise ValueError("a dissimilarity matrix must be a square int32 tensor")
    alloc = _allocator_for(m.device) if allocator == "torch" else None
    stream = torch.cuda.current_stream(m.device)
    req = _request(m, thr, maxdim, _flags(count_only, timing), alloc, matrix=True)
    out = ctypes.POINTER(VrResult)()
    with torch.cuda.device(m.device):
        rc = L.vr_build(ctypes.byref(req), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(out))
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return Result(out, alloc, ctypes.c_void_p(stream.cuda_stream), m.device)


def build_batch(points, thr, maxdim: int = 2, count_only: bool = False, timing=False,
                allocator: str = "library", graph: bool = False) -> Batch:
    """Build the filtrations of many clouds with one launch sequence.

    points: list of device tensors (n_c, d), one dtype and d for all.
    thr:    one threshold tuple for all clouds, or a list of them (one kind).
    Each batch[c] is bit-identical to build(points[c], thr[c]).  At most
    batch_limit(dtype, d) clouds per batch.  graph: as for build.
    """
    import torch

    L = lib()
    pts = [_check_points(p) for p in points]
    if not pts:
        raise ValueError("empty batch")
    thrs = list(thr) if isinstance(thr, list) else [thr] * len(pts)
    if len(thrs) != len(pts):
        raise ValueError("one threshold per cloud")
    dev = pts[0].device
    if any(p.device != dev for p in pts):
        raise ValueError("all clouds must be on one device")
    alloc = _allocator_for(dev) if allocator == "torch" else None
    stream = torch.cuda.current_stream(dev)
    flags = _flags(count_only, timing, graph)
    reqs = (VrRequest * len(pts))(*[_request(p, t, maxdim, flags, alloc) for p, t in zip(pts, thrs)])
    out = ctypes.c_void_p()
    with torch.cuda.device(dev):
        rc = L.vr_build_batch(reqs, len(pts), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(out))
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return Batch(out, alloc, ctypes.c_void_p(stream.cuda_stream), dev, len(pts))


def column_order(colptr, v, out=None, noalloc=False):
    """Per-column stable order of a compressed-sparse-column array (Section
    4.3): z[e] = the slot of entry e when its column is sorted by value,
    equal values keeping their order.

    colptr: int64 (ncols + 1,) device tensor (0, ..., nnz); v: int32 (nnz,)
    device tensor; out: optional int64 (nnz,) device tensor.  Returns z.
    noalloc=True calls vr_column_order_noalloc (scratch in the library's
    per-GPU array, nothing allocated; pass `out` to allocate nothing here
    either).
    """
    import torch

    L = lib()
    for name, t, dt in (("colptr", colptr, torch.int64), ("v", v, torch.int32)):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != dt or t.dim() != 1:
            raise TypeError(f"{name} must be a 1-D {dt} tensor on a HIP device")
    colptr, v = colptr.contiguous(), v.contiguous()
    nnz = v.numel()
    z = out if out is not None else torch.empty(nnz, dtype=torch.int64, device=v.device)
    if z.dtype != torch.int64 or z.numel() != nnz or not z.is_contiguous():
        raise ValueError("out must be a contiguous int64 tensor of nnz entries")
    stream = torch.cuda.current_stream(v.device)
    fn = L.vr_column_order_noalloc if noalloc else L.vr_column_order
    with torch.cuda.device(v.device):
        rc = fn(ctypes.c_void_p(colptr.data_ptr()), colptr.numel() - 1, ctypes.c_void_p(v.data_ptr() if nnz else 0),
                nnz, ctypes.c_void_p(z.data_ptr() if nnz else 0), ctypes.c_void_p(stream.cuda_stream))
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return z


def pairs_dim0(result):
    """Persistence pairs in dimension 0 of a build (Section 2.2.1): returns
    (e_low, death) as int32 device tensors; e_low[r] = the vertex paired with
    edge r or -1, death[v] = the edge rank pairing vertex v or -1."""
    import torch

    L = lib()
    n, K, T = result.counts
    dev = result._device
    e_low = torch.empty(K, dtype=torch.int32, device=dev)
    death = torch.empty(n, dtype=torch.int32, device=dev)
    r = VrResult(n, K, T, result._p_ij, result._p_q, result._p_tri)
    stream = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        rc = L.vr_pairs_dim0(ctypes.byref(r), ctypes.c_void_p(e_low.data_ptr() if K else 0),
                             ctypes.c_void_p(death.data_ptr() if n else 0), ctypes.c_void_p(stream.cuda_stream))
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return e_low, death


def blockprodsum(m, C, E, D):
    """S = D + C E over F2 (Section 4.6) for device CSC matrices given as
    (colptr int64, rows int32) tensors: C is m x k, E is k x n, D is m x n.
    Returns S as (colptr, rows), rows ascending in each column."""
    import torch

    L = lib()
    mats = []
    for name, (cp, rw) in (("C", C), ("E", E), ("D", D)):
        if cp.dtype != torch.int64 or rw.dtype != torch.int32 or cp.device.type != "cuda" or rw.device != cp.device:
            raise TypeError(f"{name} must be (int64 colptr, int32 rows) tensors on a HIP device")
        mats.append((cp.contiguous(), rw.contiguous()))
    for name, (cp, rw) in zip("CED", mats):
        if cp.numel() < 1 or int(cp[-1].item()) != rw.numel():
            raise ValueError(f"{name}: colptr must end at the number of rows listed")
    (cpc, rc), (cpe, re_), (cpd, rd) = mats
    k, n = cpc.numel() - 1, cpe.numel() - 1
    if cpd.numel() - 1 != n:
        raise ValueError("D must have as many columns as E")
    dev = cpc.device
    stream = torch.cuda.current_stream(dev)
    s_colptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t.numel() else 0)
    args = (int(m), k, n, ptr(cpc), ptr(rc), ptr(cpe), ptr(re_), ptr(cpd), ptr(rd))
    with torch.cuda.device(dev):
        rc_ = L.vr_blockprodsum_count(*args, ptr(s_colptr), ctypes.c_void_p(stream.cuda_stream))
        if rc_ != VR_OK:
            raise VrError(rc_, status_string(rc_))
        nnz = int(s_colptr[-1].item())
        s_rows = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        rc_ = L.vr_blockprodsum_write(*args, ptr(s_colptr), ptr(s_rows), ctypes.c_void_p(stream.cuda_stream))
        if rc_ != VR_OK:
            raise VrError(rc_, status_string(rc_))
    return s_colptr, s_rows[:nnz]


def pairs_dim1_apparent(result):
    """Apparent pairs of dimension 1 (Section 2.2.1): an int32 device tensor
    of K entries, the index in tri_key of the triangle paired with edge r
    (the first triangle of value r), or -1."""
    import torch

    L = lib()
    n, K, T = result.counts
    out = torch.empty(K, dtype=torch.int32, device=result._device)
    r = VrResult(n, K, T, result._p_ij, result._p_q, result._p_tri)
    stream = torch.cuda.current_stream(result._device)
    with torch.cuda.device(result._device):
        rc = L.vr_pairs_dim1_apparent(ctypes.byref(r), ctypes.c_void_p(out.data_ptr() if K else 0),
                                      ctypes.c_void_p(stream.cuda_stream))
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return out


def pairs_dim1(result, e_low):
    """All persistence pairs of dimension 1 (Section 2.2.1, reduced as in
    Section 2.2.2): an int32 device tensor of K entries, the index in tri_key
    of the triangle paired with edge r, or -1.  e_low is pairs_dim0's."""
    import torch

    L = lib()
    n, K, T = result.counts
    dev = result._device
    if not isinstance(e_low, torch.Tensor) or e_low.dtype != torch.int32 or e_low.numel() != K or e_low.device != dev:
        raise TypeError("e_low must be pairs_dim0's int32 tensor of K entries on the result's device")
    e_low = e_low.contiguous()
    out = torch.empty(K, dtype=torch.int32, device=dev)
    r = VrResult(n, K, T, result._p_ij, result._p_q, result._p_tri)
    stream = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        rc = L.vr_pairs_dim1(ctypes.byref(r), ctypes.c_void_p(e_low.data_ptr() if K else 0),
                             ctypes.c_void_p(out.data_ptr() if K else 0), ctypes.c_void_p(stream.cuda_stream))
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return out


def barcode(result, e_low, tri_of_edge):
    """Bars of dimensions 0 and 1: an (m, 3) int64 device tensor of
    (dimension, birth, death) rows (death 2^63 - 1 for a bar that never
    ends; bars of length zero left out), and the number of triangles paired
    with nothing (bars of dimension 2 that never end, not listed)."""
    import torch

    L = lib()
    n, K, T = result.counts
    dev = result._device
    bars = torch.empty((n + K, 3), dtype=torch.int64, device=dev)
    counts = (ctypes.c_int64 * 3)()
    r = VrResult(n, K, T, result._p_ij, result._p_q, result._p_tri)
    stream = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        rc = L.vr_barcode(ctypes.byref(r), ctypes.c_void_p(e_low.data_ptr() if K else 0),
                          ctypes.c_void_p(tri_of_edge.data_ptr() if K else 0),
                          ctypes.c_void_p(bars.data_ptr() if n + K else 0), counts, ctypes.c_void_p(stream.cuda_stream))
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return bars[: counts[0] + counts[1]], int(counts[2])


def pairs_dim2(result, tri_of_edge):
    """Persistence pairs of dimension 2 of a maxdim-3 build (Section 2.2.1,
    Alg. 1 on the anti-transpose with clearing, Section 2.2.2): an int64
    device tensor of T entries, the index in tet_key of the tetrahedron
    paired with triangle t, or -1.  tri_of_edge: pairs_dim1's output."""
    import torch

    L = lib()
    dev = result._device
    out = torch.empty(max(result.T, 1), dtype=torch.int64, device=dev)
    r = result._c_result()
    stream = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        rc = L.vr_pairs_dim2(ctypes.byref(r), ctypes.c_void_p(tri_of_edge.data_ptr() if result.K else 0),
                             ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return out[: result.T]


def barcode_dim2(result, tri_of_edge, tri_tet):
    """Bars of dimension 2 of a maxdim-3 build from the pairs of dimensions
    1 and 2 (Section 2.2.1), computed on the device: (bars, ess3) with bars
    an int64 (m, 3) device tensor of (2, birth, death) rows in triangle
    order (death INT64_MAX for a class that never dies; no zero-length
    bars) and ess3 the number of tetrahedra no triangle pairs with."""
    import torch

    L = lib()
    dev = result._device
    bars = torch.empty((max(result.T, 1), 3), dtype=torch.int64, device=dev)
    counts = (ctypes.c_int64 * 2)()
    r = result._c_result()
    stream = torch.cuda.current_stream(dev)
    with torch.cuda.device(dev):
        rc = L.vr_barcode_dim2(ctypes.byref(r), ctypes.c_void_p(tri_of_edge.data_ptr() if result.K else 0),
                               ctypes.c_void_p(tri_tet.data_ptr() if result.T else 0), ctypes.c_void_p(bars.data_ptr()),
                               counts, ctypes.c_void_p(stream.cuda_stream))
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return bars[: counts[0]], int(counts[1])


def persistence(points, thr=("full", 0, 1), maxdim: int = 2):
    """The whole device path, from points to barcodes (Section 3: the
    package's main call takes a cloud, an upper limit on the scale and how
    many dimensions to compute, and returns their persistence): the build,
    then the pairs of
    dimensions 0 and 1 and their barcode; with maxdim 3 also the
    tetrahedra, the pairs of dimension 2 and their barcode.  Returns a dict:
    "bars" an (m, 3) int64 device tensor of (dimension, birth, death) rows
    (values are largest edge ranks, -1 for vertices; death 2^63 - 1 for a
    class that never dies; no zero-length bars), "essential_top" the
    classes of the top dimension that never die (counted, not listed:
    dimension 2 for maxdim 2, 3 for maxdim 3), and "counts" (n, K, T[,
    T3]).  Every step runs in the library's kernels; this only chains the
    calls."""
    import torch

    if maxdim not in (2, 3):
        raise ValueError("maxdim must be 2 or 3")
    r = build(points, thr, maxdim=maxdim)
    try:
        e_low, _ = pairs_dim0(r)
        toe = pairs_dim1(r, e_low)
        bars, ess2 = barcode(r, e_low, toe)
        counts = r.counts
        if maxdim == 3:
            tt = pairs_dim2(r, toe)
            bars2, ess3 = barcode_dim2(r, toe, tt)
            bars = torch.cat([bars, bars2])
            return {"bars": bars, "essential_top": ess3, "counts": counts + (r.T3,)}
        return {"bars": bars, "essential_top": ess2, "counts": counts}
    finally:
        torch.cuda.current_stream(r._device).synchronize()
        r.free()


def tetra_counts(result):
    """Tetrahedra per largest edge (dimension 3): an int64 device tensor of
    K entries."""
    import torch

    L = lib()
    n, K, T = result.counts
    out = torch.empty(K, dtype=torch.int64, device=result._device)
    r = VrResult(n, K, T, result._p_ij, result._p_q, result._p_tri)
    stream = torch.cuda.current_stream(result._device)
    with torch.cuda.device(result._device):
        rc = L.vr_tetra_counts(ctypes.byref(r), ctypes.c_void_p(out.data_ptr() if K else 0),
                               ctypes.c_void_p(stream.cuda_stream))
    if rc != VR_OK:
        raise VrError(rc, status_string(rc))
    return out


def tetrahedra(result):
    """The tetrahedra of a build in filtration order: (offsets, keys) device
    tensors; offsets int64 (K + 1,) (offsets[r] = the first of value r),
    keys int64 (T3, 2) rows (value, a<<39 | b<<26 | c<<13 | d), a<b<c<d."""
    import torch

    L = lib()
    n, K, T = result.counts
    dev = result._device
    off = torch.empty(K + 1, dtype=torch.int64, device=dev)
    r = VrResult(n, K, T, result._p_ij, result._p_q, result._p_tri)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    with torch.cuda.device(dev):
        rc = L.vr_tetra_offsets(ctypes.byref(r), ctypes.c_void_p(off.data_ptr()), stream)
        if rc != VR_OK:
            raise VrError(rc, status_string(rc))
        total = int(off[-1].item())
        keys = torch.empty((max(total, 1), 2), dtype=torch.int64, device=dev)
        rc = L.vr_tetra_write(ctypes.byref(r), ctypes.c_void_p(off.data_ptr()), total,
                              ctypes.c_void_p(keys.data_ptr()), stream)
        if rc != VR_OK:
            raise VrError(rc, status_string(rc))
    return off, keys[:total]
