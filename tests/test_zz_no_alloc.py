"""vr_column_order_noalloc (scratch in the library's per-GPU array) against
vr_column_order (scratch from the library's cache), bit-exact, on two calls
in a row, the second smaller, and both against the oracle."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1809_04424_amd as vr

    vr.lib()
    yield


def _both(colptr, v):
    import torch

    import paper_1809_04424_amd as vr

    cp = torch.from_numpy(np.ascontiguousarray(colptr, np.int64)).to("cuda:0")
    vv = torch.from_numpy(np.ascontiguousarray(v, np.int32)).to("cuda:0")
    z_static = torch.full((len(v),), -7, dtype=torch.int64, device="cuda:0")
    vr.column_order(cp, vv, out=z_static, noalloc=True)
    z_cache = vr.column_order(cp, vv)
    torch.cuda.synchronize()
    return z_static.cpu().numpy(), z_cache.cpu().numpy()


def test_noalloc_equals_cached_scratch_twice(orc):
    # first call: 2000 columns of 1999 entries each (4 million entries,
    # long segments sorted in LDS); second: short columns, far fewer entries
    big_cp, big_v = workloads.full_columns(seed=11, ncols=2000, length=1999, maxvalue=2**20)
    small_cp, small_v = workloads.csc_columns(seed=12, ncols=3000, mean_len=8, maxvalue=20)
    assert len(small_v) < len(big_v)
    for label, (cp, v) in (("big", (big_cp, big_v)), ("small", (small_cp, small_v))):
        print(f"[gpu] column_order_noalloc {label} ncols={len(cp) - 1} nnz={len(v)}", flush=True)
        zs, zc = _both(cp, v)
        assert np.array_equal(zs, zc), label
        assert np.array_equal(zs, orc.column_order(cp, v)), label


def test_noalloc_rejects_oversize_without_launch():
    import torch

    import paper_1809_04424_amd as vr

    nnz = (32 << 20) // 4  # 4 bytes per entry alone exceed the array
    cp = torch.tensor([0, nnz], dtype=torch.int64, device="cuda:0")
    v = torch.zeros(nnz, dtype=torch.int32, device="cuda:0")
    z = torch.full((nnz,), -3, dtype=torch.int64, device="cuda:0")
    with pytest.raises(vr.VrError):
        vr.column_order(cp, v, out=z, noalloc=True)
    torch.cuda.synchronize()
    assert int(z[0]) == -3 and int(z[-1]) == -3
