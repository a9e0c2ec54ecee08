"""The C-ABI library loads, exports every symbol include/vr.h declares, and
rejects invalid requests before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_1809_04424_amd as vr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vr_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_binding_symbols():
    assert _declared() == sorted(vr.SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = vr.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_only_c_abi_is_exported():
    import subprocess

    out = subprocess.run(["nm", "-D", "--defined-only", vr.LIB_PATH], capture_output=True, text=True).stdout
    syms = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert syms == sorted(_declared())


def test_status_strings_and_version():
    assert vr.status_string(vr.VR_OK) == "ok"
    assert "32 bits" in vr.status_string(vr.VR_ERANGE)
    assert vr.lib().vr_version() >= 100
    assert vr.stage_names()[0] == "dist" and "tri_write" in vr.stage_names()


def _req(**kw):
    base = dict(points=16, n=10, d=3, dtype=vr.VR_I8, thr_kind=0, thr_num=0, thr_den=1, maxdim=2, flags=0, alloc=None)
    base.update(kw)
    return vr.VrRequest(**base)


@pytest.mark.parametrize("kw,code", [
    (dict(d=0), vr.VR_EINVAL),
    (dict(n=-1), vr.VR_EINVAL),
    (dict(dtype=7), vr.VR_EINVAL),
    (dict(points=None), vr.VR_EINVAL),
    (dict(maxdim=4), vr.VR_EINVAL),
    (dict(maxdim=3, flags=vr.VR_GRAPH), vr.VR_EINVAL),  # tetrahedra are not captured
    (dict(thr_kind=9), vr.VR_EINVAL),
    (dict(thr_kind=1, thr_num=46), vr.VR_EINVAL),      # more than C(10,2) edges
    (dict(thr_kind=2, thr_num=3, thr_den=0), vr.VR_EINVAL),
    (dict(thr_kind=2, thr_num=5, thr_den=4), vr.VR_EINVAL),
    (dict(thr_kind=3, thr_num=-1), vr.VR_EINVAL),
    (dict(n=8193), vr.VR_E2BIG),
    (dict(n=8000), vr.VR_E2BIG),                        # C(8000,2) > 2^24 kept edges
])
def test_invalid_requests_rejected_before_device_work(kw, code):
    out = ctypes.POINTER(vr.VrResult)()
    rc = vr.lib().vr_build(ctypes.byref(_req(**kw)), None, ctypes.byref(out))
    assert rc == code
    assert not out


def test_batch_rejects_maxdim3():
    """Tetrahedra are vr_build's alone: a batch asking for them is refused."""
    reqs = (vr.VrRequest * 2)(_req(), _req(maxdim=3))
    out = ctypes.c_void_p()
    assert vr.lib().vr_build_batch(reqs, 2, None, ctypes.byref(out)) == vr.VR_EINVAL
    assert not out.value


def test_workspace_bytes():
    a = vr.workspace_bytes(1000, 3)
    b = vr.workspace_bytes(4000, 64)
    assert 0 < a < b
    assert vr.workspace_bytes(9000, 3) == -1
    assert vr.lib().vr_query_counts(None, None) == vr.VR_EINVAL
    vr.lib().vr_free(None, None)  # NULL-safe


def _batch_rc(reqs):
    arr = (vr.VrRequest * max(1, len(reqs)))(*reqs)
    out = ctypes.c_void_p()
    rc = vr.lib().vr_build_batch(arr, len(reqs), None, ctypes.byref(out))
    return rc, out


@pytest.mark.parametrize("reqs,code", [
    ([], vr.VR_EINVAL),                                                     # empty batch
    ([_req(), _req(dtype=vr.VR_I16)], vr.VR_EINVAL),                        # mixed coordinate types
    ([_req(), _req(d=4)], vr.VR_EINVAL),                                    # mixed dimensions
    ([_req(), _req(thr_kind=2, thr_num=1, thr_den=5)], vr.VR_EINVAL),        # mixed threshold kinds
    ([_req(), _req(maxdim=1)], vr.VR_EINVAL),                               # mixed maxdim
    ([_req(), _req(flags=vr.VR_COUNT_ONLY)], vr.VR_EINVAL),                 # mixed flags
    ([_req(), _req(n=-1)], vr.VR_EINVAL),                                   # one bad request
    ([_req(), _req(n=8193)], vr.VR_E2BIG),
    ([_req(dtype=vr.VR_I16), _req(dtype=vr.VR_I16)], vr.VR_E2BIG),          # 32-bit distances: one cloud per batch
    ([_req(d=40000)] * 2, vr.VR_E2BIG),                                     # 255^2 d needs 32 bits, 2 clouds 1 more
])
def test_invalid_batches_rejected_before_device_work(reqs, code):
    rc, out = _batch_rc(reqs)
    assert rc == code
    assert not out.value


def test_batch_key_budget():
    # int8, d = 3: squared distances need 18 bits, so 2^14 clouds fit the 32-bit key
    assert vr.batch_limit(vr.VR_I8, 3) == 1 << 14
    assert vr.batch_limit(vr.VR_I8, 64) == 1 << 10
    assert vr.batch_limit(vr.VR_I16, 3) == 1
    rc, _ = _batch_rc([_req(d=3)] * ((1 << 14) + 1))
    assert rc == vr.VR_E2BIG


def test_batch_handles_null_safe():
    L = vr.lib()
    r = vr.VrResult()
    assert L.vr_batch_result(None, 0, ctypes.byref(r)) == vr.VR_EINVAL
    assert L.vr_batch_stage_ms(None, None, 0) == vr.VR_EINVAL
    L.vr_batch_free(None, None)
    out = ctypes.c_void_p()
    assert L.vr_build_batch(None, 1, None, ctypes.byref(out)) == vr.VR_EINVAL


def test_batch_workspace_bytes():
    one = vr.batch_workspace_bytes([(10, 3, vr.VR_I8, ("fraction", 1, 1))])
    assert one == vr.workspace_bytes(10, 3)  # K = E: the shape's maximum
    a = vr.batch_workspace_bytes([(500, 3, vr.VR_I8, ("fraction", 20, 100))])
    b = vr.batch_workspace_bytes([(700, 3, vr.VR_I8, ("fraction", 10, 100))])
    ab = vr.batch_workspace_bytes([(500, 3, vr.VR_I8, ("fraction", 20, 100)), (700, 3, vr.VR_I8, ("fraction", 10, 100))])
    assert max(a, b) < ab <= a + b
    assert vr.batch_workspace_bytes([(1, 3, vr.VR_I8, ("full", 0, 1)), (0, 3, vr.VR_I8, ("full", 0, 1))]) == 0
    assert vr.batch_workspace_bytes([(40, 3, vr.VR_I8, ("count", 0, 1))]) == 0  # nothing kept
    with pytest.raises(vr.VrError):
        vr.batch_workspace_bytes([(10, 3, vr.VR_I8, ("full", 0, 1)), (10, 4, vr.VR_I8, ("full", 0, 1))])


def test_autotune_rejects_bad_arguments():
    L = vr.lib()
    parts = (ctypes.c_int32 * 6)()
    assert L.vr_autotune(None, 1, None, parts) == vr.VR_EINVAL
    arr = (vr.VrRequest * 1)(_req())
    assert L.vr_autotune(arr, 1, None, None) == vr.VR_EINVAL
    arr = (vr.VrRequest * 1)(_req(d=0))
    assert L.vr_autotune(arr, 1, None, parts) == vr.VR_EINVAL


def test_unpack_rejects_bad_arguments():
    L = vr.lib()
    assert L.vr_unpack_triangles(None, None, None) == vr.VR_EINVAL
    r = vr.VrResult(10, 5, 3, None, None, None)  # count-only result: no keys
    assert L.vr_unpack_triangles(ctypes.byref(r), 16, None) == vr.VR_EINVAL
    empty = vr.VrResult(10, 5, 0, None, None, None)
    assert L.vr_unpack_triangles(ctypes.byref(empty), None, None) == vr.VR_OK


def test_set_schedule_validates():
    L = vr.lib()
    arr = (vr.VrRequest * 1)(_req())
    good = (ctypes.c_int32 * 6)(256, 1, 4, 256, 2, 8)
    assert L.vr_set_schedule(arr, 1, good) == vr.VR_OK
    # 0 work-groups per vertex: the write's one-wave-per-eighth form (not the count's)
    assert L.vr_set_schedule(arr, 1, (ctypes.c_int32 * 6)(256, 1, 4, 512, 0, 8)) == vr.VR_OK
    for bad in [(64, 1, 4, 256, 2, 8), (256, 3, 4, 256, 2, 8), (256, 1, 5, 256, 2, 8), (256, 1, 4, 256, 2, 2),
                (256, 1, 4, 1024, 2, 8), (256, 1, 4, 256, 32, 8), (256, 0, 4, 256, 2, 8), (256, 1, 4, 256, -1, 8)]:
        assert L.vr_set_schedule(arr, 1, (ctypes.c_int32 * 6)(*bad)) == vr.VR_EINVAL
    assert L.vr_set_schedule(None, 1, good) == vr.VR_EINVAL
    assert L.vr_set_schedule(arr, 0, good) == vr.VR_EINVAL
    assert L.vr_set_schedule(arr, 1, None) == vr.VR_EINVAL
    arr = (vr.VrRequest * 1)(_req(d=0))
    assert L.vr_set_schedule(arr, 1, good) == vr.VR_EINVAL


def test_dissimilarity_matrix_request_shape():
    L = vr.lib()
    assert L.vr_workspace_bytes(100, 100, vr.VR_DIST, vr.VR_THR["fraction"]) > 0
    assert L.vr_workspace_bytes(100, 3, vr.VR_DIST, vr.VR_THR["fraction"]) == -1  # d must equal n
    arr = (vr.VrRequest * 1)(_req(d=3))
    arr[0].dtype = vr.VR_DIST
    out = ctypes.POINTER(vr.VrResult)()
    assert L.vr_build(arr, None, ctypes.byref(out)) == vr.VR_EINVAL


def test_column_order_argument_checks():
    """Argument errors come back before any device work."""
    L = vr.lib()
    assert L.vr_column_order(None, -1, None, 0, None, None) == vr.VR_EINVAL
    assert L.vr_column_order(None, 0, None, -1, None, None) == vr.VR_EINVAL
    assert L.vr_column_order(None, 3, None, 0, None, None) == vr.VR_EINVAL  # colptr missing
    assert L.vr_column_order(None, 0, None, 0, None, None) == vr.VR_OK      # nothing to do


def test_column_order_noalloc_argument_checks():
    """The same argument errors, plus VR_E2BIG once one call's scratch would
    not fit the library's per-GPU array; all before any device work (the
    pointers below are never read)."""
    L = vr.lib()
    f = L.vr_column_order_noalloc
    assert f(None, -1, None, 0, None, None) == vr.VR_EINVAL
    assert f(None, 0, None, -1, None, None) == vr.VR_EINVAL
    assert f(None, 3, None, 0, None, None) == vr.VR_EINVAL
    assert f(None, 0, None, 0, None, None) == vr.VR_OK
    fake = ctypes.c_void_p(0x1000)
    limit = 32 << 20  # VR_COLORDER_NOALLOC_BYTES
    nnz_over = limit // 4  # 4 bytes per entry alone fill the array
    assert f(fake, 1, fake, nnz_over, fake, None) == vr.VR_E2BIG
    # the largest nnz whose scratch fits, and one more
    fits = lambda m: ((8 * ((m + 4095) // 4096) + 255) // 256) * 256 + 4 * m <= limit  # noqa: E731
    m = max(x for x in range(nnz_over - 20000, nnz_over) if fits(x))
    assert not fits(m + 1)
    assert f(fake, 1, fake, m + 1, fake, None) == vr.VR_E2BIG


def test_matrix_batches_hold_one_matrix():
    """A dissimilarity matrix takes all 32 bits of the sort key, so a batch
    holds one matrix of two or more points (VR_E2BIG otherwise)."""
    L = vr.lib()
    arr = (vr.VrRequest * 2)(_req(n=50, d=50, dtype=vr.VR_DIST), _req(n=50, d=50, dtype=vr.VR_DIST))
    assert L.vr_batch_workspace_bytes(arr, 2) == vr.VR_E2BIG
    assert L.vr_batch_workspace_bytes(arr, 1) > 0
    arr2 = (vr.VrRequest * 2)(_req(n=50, d=50, dtype=vr.VR_DIST), _req(n=1, d=50, dtype=vr.VR_DIST))
    assert L.vr_batch_workspace_bytes(arr2, 2) == -1  # a one-point request must say d = 1


def test_pairs_dim0_argument_checks():
    L = vr.lib()
    assert L.vr_pairs_dim0(None, None, None, None) == vr.VR_EINVAL
    r = vr.VrResult(0, 0, 0, None, None, None)
    assert L.vr_pairs_dim0(ctypes.byref(r), None, None, None) == vr.VR_OK  # empty: nothing to do
    r = vr.VrResult(10, 5, 0, None, None, None)
    assert L.vr_pairs_dim0(ctypes.byref(r), None, None, None) == vr.VR_EINVAL  # edges but no arrays
    r = vr.VrResult(9000, 0, 0, None, None, None)
    assert L.vr_pairs_dim0(ctypes.byref(r), None, None, None) == vr.VR_EINVAL


def test_blockprodsum_argument_checks():
    L = vr.lib()
    p = ctypes.c_void_p(8)  # never dereferenced: every call below is refused first
    assert L.vr_blockprodsum_count(-1, 1, 1, p, p, p, p, p, p, p, None) == vr.VR_EINVAL
    assert L.vr_blockprodsum_count(1, 1, 1, None, p, p, p, p, p, p, None) == vr.VR_EINVAL
    assert L.vr_blockprodsum_count(300000, 1, 1, p, p, p, p, p, p, p, None) == vr.VR_E2BIG
    assert L.vr_blockprodsum_write(1, 1, 1, p, p, p, p, p, p, None, p, None) == vr.VR_EINVAL


def test_pairs_dim1_apparent_argument_checks():
    L = vr.lib()
    assert L.vr_pairs_dim1_apparent(None, None, None) == vr.VR_EINVAL
    r = vr.VrResult(10, 0, 0, None, None, None)
    assert L.vr_pairs_dim1_apparent(ctypes.byref(r), None, None) == vr.VR_OK  # no edges
    r = vr.VrResult(10, 5, 3, None, None, None)
    assert L.vr_pairs_dim1_apparent(ctypes.byref(r), ctypes.c_void_p(8), None) == vr.VR_EINVAL  # no keys


def test_tetra_counts_argument_checks():
    L = vr.lib()
    assert L.vr_tetra_counts(None, None, None) == vr.VR_EINVAL
    r = vr.VrResult(10, 0, 0, None, None, None)
    assert L.vr_tetra_counts(ctypes.byref(r), None, None) == vr.VR_OK
    r = vr.VrResult(10, 4, 0, None, None, None)
    assert L.vr_tetra_counts(ctypes.byref(r), None, None) == vr.VR_EINVAL


def test_persistence_rejects_other_dimensions():
    """The chained call takes maxdim 2 or 3 and refuses others before any
    device work."""
    import torch

    pts = torch.zeros((4, 2), dtype=torch.int32)
    for bad in (1, 4):
        with pytest.raises(ValueError):
            vr.persistence(pts, ("full", 0, 1), maxdim=bad)
