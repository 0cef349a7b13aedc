"""R-MAT scale 20 (1,048,576 rows, edge factor 16, a=0.57 b=c=0.19, seed 4,
self-loops dropped, symmetrised, values 1.0) at full size: C = A*A has about
2.4e10 entries (about 288 GB), more than one GPU holds beside its inputs, so
the symbolic phase runs over all rows and the numeric phase in row panels.
Checked: every row count against the oracle's structure count and the
product bound; the 1,000 rows with the most products, and sampled rows, bit
for bit, each computed as its own one-row panel; one large panel's sampled
rows.  At scale 18 the whole product is checked row by row against the
oracle's streaming per-row statistics (count, column hash, value sum)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2507_21253_amd as hc  # noqa: E402


@pytest.fixture(scope="module")
def rmat20():
    R = synth.workload_rmat(20, 4)
    D = hc.DeviceCSR.from_host(R)
    P = hc.Product(D, D)
    # symbolic phase only: C itself (about 288 GB) is never allocated whole
    P.info = hc.spgemm_symbolic(D, D, P.C_row_ptr, P.ws, P.o)
    yield R, D, P, int(P.info.nnz)
    del P, D
    torch.cuda.empty_cache()


def test_rmat20_symbolic_counts(rmat20):
    R, D, P, nnz = rmat20
    rp = P.C_row_ptr.cpu().numpy()
    cnt = np.diff(rp)
    ub = np.zeros(R.nrows, np.int64)
    np.add.at(ub, np.repeat(np.arange(R.nrows), np.diff(R.rp)), np.diff(R.rp)[R.col])
    assert rp[0] == 0 and rp[-1] == nnz and np.all(cnt >= 0) and np.all(cnt <= ub)
    assert np.all((cnt == 0) == (ub == 0))
    # every row against the oracle's count of distinct columns (host threads, C never formed)
    ref = oracle.spgemm_count(R, R, min(16, len(os.sched_getaffinity(0))))
    bad = np.flatnonzero(cnt != ref)
    assert bad.size == 0, "rows %s: gpu %s oracle %s" % (bad[:5], cnt[bad[:5]], ref[bad[:5]])
    assert int(ref.sum()) == nnz


def test_rmat20_heaviest_rows_bitwise(rmat20):
    # the 1,000 rows with the most products (the column-window path's hub rows), each as a one-row panel
    R, D, P, nnz = rmat20
    rp = P.C_row_ptr.cpu().numpy()
    ub = np.zeros(R.nrows, np.int64)
    np.add.at(ub, np.repeat(np.arange(R.nrows), np.diff(R.rp)), np.diff(R.rp)[R.col])
    rows = np.argsort(-ub, kind="stable")[:1000]
    with ThreadPoolExecutor(max_workers=min(16, len(os.sched_getaffinity(0)))) as ex:
        refs = list(ex.map(lambda r: oracle.spgemm(R, R, (int(r), int(r) + 1)), rows))
    width = int(max(rp[r + 1] - rp[r] for r in rows))
    col = torch.empty(max(width, 1), dtype=torch.int32, device="cuda")
    val = torch.empty(max(width, 1), dtype=torch.float64, device="cuda")
    for r, ref in zip(rows, refs):
        b, e = int(rp[r]), int(rp[r + 1])
        assert e - b == ref.nnz, "row %d" % r
        o = hc.opts(unit_lo=int(r), unit_hi=int(r) + 1, out_base=b, flags=hc.F_SYNC_CHECK)
        hc.spgemm_numeric(D, D, P.info, P.C_row_ptr, col, val, P.ws, o, capacity=e - b)
        np.testing.assert_array_equal(col[:e - b].cpu().numpy(), ref.col, err_msg="row %d" % r)
        np.testing.assert_array_equal(val[:e - b].cpu().numpy(), ref.val, err_msg="row %d" % r)


def test_rmat20_sampled_rows_bitwise(rmat20):
    R, D, P, nnz = rmat20
    rp = P.C_row_ptr.cpu().numpy()
    rng = np.random.default_rng(21)
    ub = np.diff(R.rp)
    rows = list(rng.integers(0, R.nrows, 24)) + [int(np.argmax(np.diff(rp)))]
    for r in rows:
        b, e = int(rp[r]), int(rp[r + 1])
        col = torch.empty(max(e - b, 1), dtype=torch.int32, device="cuda")
        val = torch.empty(max(e - b, 1), dtype=torch.float64, device="cuda")
        o = hc.opts(unit_lo=int(r), unit_hi=int(r) + 1, out_base=b, flags=hc.F_SYNC_CHECK)
        hc.spgemm_numeric(D, D, P.info, P.C_row_ptr, col, val, P.ws, o, capacity=e - b)
        ref = oracle.spgemm(R, R, (int(r), int(r) + 1))
        np.testing.assert_array_equal(col[:e - b].cpu().numpy(), ref.col, err_msg="row %d" % r)
        np.testing.assert_array_equal(val[:e - b].cpu().numpy(), ref.val, err_msg="row %d" % r)


def test_rmat20_large_panel(rmat20):
    # rows [0, hi) with about 1.5e9 entries (18 GB) in one numeric call, sampled rows checked
    R, D, P, nnz = rmat20
    rp = P.C_row_ptr.cpu().numpy()
    hi = int(np.searchsorted(rp, 1_500_000_000, side="right")) - 1
    hi = max(hi, 1)
    cap = int(rp[hi])
    col = torch.empty(cap, dtype=torch.int32, device="cuda")
    val = torch.empty(cap, dtype=torch.float64, device="cuda")
    o = hc.opts(unit_lo=0, unit_hi=hi, out_base=0, flags=hc.F_SYNC_CHECK)
    hc.spgemm_numeric(D, D, P.info, P.C_row_ptr, col, val, P.ws, o, capacity=cap)
    torch.cuda.synchronize()
    rng = np.random.default_rng(22)
    for r in rng.integers(0, hi, 12):
        b, e = int(rp[r]), int(rp[r + 1])
        ref = oracle.spgemm(R, R, (int(r), int(r) + 1))
        np.testing.assert_array_equal(col[b:e].cpu().numpy(), ref.col, err_msg="row %d" % r)
        np.testing.assert_array_equal(val[b:e].cpu().numpy(), ref.val, err_msg="row %d" % r)
    del col, val


def test_rmat18_every_row_checksum():
    # R-MAT scale 18 (262,144 rows, 9.5e9 products, 3.0e9 entries, 35 GB): the
    # whole C computed in row panels, and every row's count, hash of its sorted
    # columns and value sum (exact: the values are integers) against the
    # oracle's streaming per-row statistics (C never stored on the host side)
    import os
    R = synth.workload_rmat(18, 4)
    D = hc.DeviceCSR.from_host(R)
    P = hc.Product(D, D)
    P.info = hc.spgemm_symbolic(D, D, P.C_row_ptr, P.ws, P.o)
    rp = P.C_row_ptr.cpu().numpy()
    nthreads = min(16, len(os.sched_getaffinity(0)))
    ref_n, ref_h, ref_s = oracle.rowstats(R, R, (0, R.nrows), nthreads)
    np.testing.assert_array_equal(np.diff(rp), ref_n)
    cap = 700_000_000  # entries per panel (8.4 GB)
    col = torch.empty(cap, dtype=torch.int32, device="cuda")
    val = torch.empty(cap, dtype=torch.float64, device="cuda")
    lo = 0
    while lo < R.nrows:
        hi = max(int(np.searchsorted(rp, rp[lo] + cap, side="right")) - 1, lo + 1)
        b0 = int(rp[lo])
        o = hc.opts(unit_lo=lo, unit_hi=hi, out_base=b0, flags=hc.F_SYNC_CHECK)
        hc.spgemm_numeric(D, D, P.info, P.C_row_ptr, col, val, P.ws, o, capacity=cap)
        n = int(rp[hi]) - b0
        c = col[:n].cpu().numpy()
        v = val[:n].cpu().numpy()
        for r in range(lo, hi):
            b, e = int(rp[r]) - b0, int(rp[r + 1]) - b0
            assert oracle.hash_cols(c[b:e]) == int(ref_h[r]), "row %d columns" % r
        starts = (rp[lo:hi] - b0).astype(np.int64)
        nonempty = rp[lo + 1:hi + 1] > rp[lo:hi]
        sums = np.zeros(hi - lo)
        if n:
            sums[nonempty] = np.add.reduceat(v, starts[nonempty])
        np.testing.assert_array_equal(sums, ref_s[lo:hi], err_msg="value sums of rows %d..%d" % (lo, hi))
        lo = hi
    del col, val, P, D
    torch.cuda.empty_cache()
