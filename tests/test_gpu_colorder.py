"""Per-column stable order (vr_column_order) against the oracle, bit-exact."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

WIN = 4096  # entries per window of the kernels: cases straddle its multiples


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1809_04424_amd as vr

    vr.lib()
    yield


def _run(colptr, v):
    import torch

    import paper_1809_04424_amd as vr

    cp = torch.from_numpy(np.ascontiguousarray(colptr, np.int64)).to("cuda:0")
    vv = torch.from_numpy(np.ascontiguousarray(v, np.int32)).to("cuda:0")
    z = vr.column_order(cp, vv)
    torch.cuda.synchronize()
    return z.cpu().numpy()


def _check(orc, colptr, v, label):
    print(f"[gpu] column_order {label} ncols={len(colptr) - 1} nnz={len(v)}", flush=True)
    assert np.array_equal(_run(colptr, v), orc.column_order(colptr, v))


CASES = {
    # short columns only: every window ranks by counting
    "short": dict(seed=1, ncols=3000, mean_len=8, maxvalue=20),
    "short_wide": dict(seed=2, ncols=2000, mean_len=60, maxvalue=2**30),
    # long segments: windows sort in LDS; columns span 2..12 windows
    "long_mixed": dict(seed=3, ncols=400, mean_len=100, maxvalue=50, long_cols=6, long_len=9000),
    "long_span12": dict(seed=4, ncols=50, mean_len=20, maxvalue=1000, long_cols=2, long_len=12 * WIN + 77),
    "mid": dict(seed=5, ncols=200, mean_len=400, maxvalue=100000),
    "ties": dict(seed=6, ncols=100, mean_len=600, maxvalue=1, long_cols=1, long_len=5 * WIN),
    "signed": dict(seed=7, ncols=300, mean_len=50, maxvalue=2**32 - 1, lo=-2**31, long_cols=2, long_len=7000),
    "mostly_empty": dict(seed=8, ncols=20000, mean_len=2, maxvalue=9, empty=0.9),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_random_csc(orc, name):
    colptr, v = workloads.csc_columns(**CASES[name])
    _check(orc, colptr, v, name)


def test_columns_on_window_boundaries(orc):
    """Columns that start or end exactly at window starts, empty columns at
    the boundaries, and one column of exactly one window."""
    lens = [WIN, 0, 0, WIN - 1, 1, 0, 2 * WIN, 3, WIN - 3, 0, WIN, 5, 0]
    colptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    v = np.random.default_rng(9).integers(0, 300, int(colptr[-1])).astype(np.int32)
    _check(orc, colptr, v, "boundaries")


@pytest.mark.parametrize("nnz", [1, 2, 63, 64, 65, 255, 256, 257, WIN - 1, WIN, WIN + 1])
def test_one_column_sizes(orc, nnz):
    v = np.random.default_rng(nnz).integers(-5, 6, nnz).astype(np.int32)
    _check(orc, np.array([0, nnz]), v, f"one column {nnz}")


def test_empty_and_degenerate(orc):
    import torch

    import paper_1809_04424_amd as vr

    z = vr.column_order(torch.zeros(4, dtype=torch.int64, device="cuda:0"),
                        torch.zeros(0, dtype=torch.int32, device="cuda:0"))
    assert z.numel() == 0
    _check(orc, np.array([0, 0, 0, 5, 5]), np.array([3, 3, 3, 3, 3]), "constant")
    _check(orc, np.array([0, 6]), np.array([2**31 - 1, -2**31, 0, -1, 1, -2**31]), "extremes")
    colptr = np.arange(0, 10001, dtype=np.int64)  # 10000 columns of one entry
    _check(orc, colptr, np.random.default_rng(3).integers(0, 9, 10000).astype(np.int32), "singletons")


def test_rank_matrix_columns(orc):
    """The paper's use: the columns of the kept-edge rank matrix of a cloud
    (neighbours in vertex order, values = edge ranks); the order of a column
    is the vertex's star sorted by rank."""
    c = workloads.noisy_circle(seed=11, n=1500)
    f = orc.build(c.points, c.thr, list_triangles=False)
    R = f.R.reshape(c.n, c.n)
    cols = [np.nonzero(R[:, j] >= 0)[0] for j in range(c.n)]
    colptr = np.concatenate([[0], np.cumsum([len(x) for x in cols])]).astype(np.int64)
    v = np.concatenate([R[x, j] for j, x in enumerate(cols)]).astype(np.int32)
    z = _run(colptr, v)
    assert np.array_equal(z, orc.column_order(colptr, v))
    # ranks are distinct: entry placed at z holds the column's ranks ascending
    out = np.empty_like(v)
    out[z] = v
    for j in range(0, c.n, 97):
        assert np.array_equal(out[colptr[j]:colptr[j + 1]], np.sort(R[cols[j], j]))


def test_full_size_bench_workload(orc):
    """2000 columns of 1999 entries, values in 0..1999000: the shape of a
    complete 2000-point graph's rank matrix, as the benchmark times it."""
    colptr, v = workloads.full_columns(2000, 2000, 1999, 1999000)
    _check(orc, colptr, v, "full 2000x1999")


def test_out_argument_and_repeat(orc):
    import torch

    import paper_1809_04424_amd as vr

    colptr, v = workloads.csc_columns(12, ncols=700, mean_len=30, maxvalue=40, long_cols=1, long_len=6000)
    cp = torch.from_numpy(colptr).to("cuda:0")
    vv = torch.from_numpy(v).to("cuda:0")
    out = torch.full((len(v),), -7, dtype=torch.int64, device="cuda:0")
    a = vr.column_order(cp, vv, out=out).cpu().numpy()
    b = vr.column_order(cp, vv).cpu().numpy()
    assert np.array_equal(a, b) and np.array_equal(a, orc.column_order(colptr, v))
