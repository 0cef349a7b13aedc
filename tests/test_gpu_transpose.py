"""GPU transpose (hcsp_csr_transpose), used to form A^T for the hierarchical plan's overlap matrix A A^T
(Alg. 3): rows of A^T must list their columns ascending and carry exactly A's values.  The reference is
the definition, written with numpy: entry (i, j) of A becomes entry (j, i), then each row is sorted.
Rows of A^T of every length class are covered (short, a few hundred to a few thousand, and longer than
8,192 entries), plus rectangular and empty matrices."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2507_21253_amd as hc  # noqa: E402


def ref_transpose(A):
    rows = np.repeat(np.arange(A.nrows, dtype=np.int64), np.diff(A.rp))
    order = np.lexsort((rows, A.col.astype(np.int64)))   # by column, then by row
    rp = np.zeros(A.ncols + 1, np.int64)
    np.add.at(rp, A.col.astype(np.int64) + 1, 1)
    return np.cumsum(rp), rows[order].astype(np.int32), A.val[order]


def hub_matrix(n, m, seed):
    """n x m with column 0 in every row, column 1 in every other row (long rows of A^T), column 2 in every
    fourth row and column 3 in every 40th (mid-length rows), and 5 random columns per row besides."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        c = {0}
        if i % 2 == 0:
            c.add(1)
        if i % 4 == 0:
            c.add(2)
        if i % 40 == 0:
            c.add(3)
        c.update(rng.integers(4, m, 5).tolist())
        rows.append(sorted(c))
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([c for r in rows for c in r], np.int32)
    return synth.HostCSR(rp, col, rng.uniform(-1, 1, len(col)), n, m)


def inputs():
    yield "uniform_300x200", synth.uniform(300, 200, 6, 3)
    yield "uniform_5000_nonsym", synth.uniform(5000, 5000, 12, 4)
    yield "stencil27_12_relabelled", synth.workload_stencil27(12, 2, 3)[0]
    yield "rmat12", synth.rmat(12, 16, 0.57, 0.19, 0.19, 5)
    yield "hubs_40000x3000", hub_matrix(40000, 3000, 6)
    yield "empty_rows", synth.HostCSR(np.zeros(8, np.int64), np.zeros(0, np.int32), np.zeros(0), 7, 5)


@pytest.mark.parametrize("name,A", list(inputs()))
def test_transpose_matches_definition(name, A):
    Ad = hc.DeviceCSR.from_host(A)
    rp, col, val = ref_transpose(A)
    for values in (True, False):
        T = hc.csr_transpose(Ad, values)
        torch.cuda.synchronize()
        assert (T.nrows, T.ncols, T.nnz) == (A.ncols, A.nrows, A.nnz)
        np.testing.assert_array_equal(T.row_ptr.cpu().numpy(), rp, err_msg=name)
        np.testing.assert_array_equal(T.col.cpu().numpy(), col, err_msg=name)
        if values:
            np.testing.assert_array_equal(T.val.cpu().numpy().view(np.int64), val.view(np.int64), err_msg=name)


def test_transpose_twice_is_identity_and_rejects_bad_shapes():
    A = hub_matrix(20000, 500, 7)
    Ad = hc.DeviceCSR.from_host(A)
    TT = hc.csr_transpose(hc.csr_transpose(Ad))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(TT.row_ptr.cpu().numpy(), A.rp)
    np.testing.assert_array_equal(TT.col.cpu().numpy(), A.col)
    np.testing.assert_array_equal(TT.val.cpu().numpy(), A.val)
    import ctypes
    bad = hc.c_csr(A.nrows, A.ncols, A.nnz, hc._tp(Ad.row_ptr), hc._tp(Ad.col), hc._tp(Ad.val))
    a = Ad.c()
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    assert hc.lib().hcsp_csr_transpose(ctypes.byref(a), ctypes.byref(bad), hc._tp(ws), ws.numel(),
                                       hc._stream()) == -1     # At must be ncols x nrows
