"""GPU parity of the long-row path: rows whose output is too large for one
shared-memory table (CSR rows, or the member rows of clusters) hold their
output columns in bitmaps, counted per column chunk in the symbolic phase;
the numeric phase takes a whole row, or for rows of many items one column
chunk, per workgroup, in windows whose slots are the keys' ranks; C must
still equal the oracle bit for bit, since every output entry gets its
products in ascending k.

Cases: rows counted by chunks in the symbolic phase (products beyond the
largest symbolic table; a bitmap per row, the counts split at the numeric
chunks), with one chunk or up to 256 (win_chunk_log2 sets the products per
chunk); rows whose column range is wider than one bitmap segment (CSR
rows and the member rows of clusters); rows counted whole in shared memory but too large
for the numeric tables (one chunk over the row's column range); output
columns packed densely into part of a chunk; row panels; R-MAT rows (the
whole R-MAT 16 product among them); clustered
operands (fixed and hierarchical plans); a numeric call whose chunking
differs from its symbolic call's is refused."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2507_21253_amd as hc  # noqa: E402


def product(A, B, o=None):
    torch.cuda.synchronize()
    C = hc.spgemm(hc.DeviceCSR.from_host(A), hc.DeviceCSR.from_host(B), o)
    torch.cuda.synchronize()
    return C.to_host()


def assert_same(Cg, Cr, where=""):
    np.testing.assert_array_equal(Cg.rp, Cr.rp, err_msg="row_ptr " + where)
    np.testing.assert_array_equal(Cg.col, Cr.col, err_msg="col " + where)
    np.testing.assert_array_equal(Cg.val, Cr.val, err_msg="val " + where)


def csr_from_rows(rows, ncols, rng):
    rp = np.zeros(len(rows) + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate([np.sort(r) for r in rows]).astype(np.int32) if rows else np.zeros(0, np.int32)
    val = rng.uniform(-1, 1, len(col))
    return synth.HostCSR(rp, col, val, len(rows), ncols)


def packed_case(seed, dense_cols, ncols=80_000, m=30, n=40):
    """B's rows hold most columns of [0, dense_cols) and a few spread ones, so
    the output columns crowd into the start of the first chunk."""
    rng = np.random.default_rng(seed)
    brows = [np.concatenate([rng.choice(dense_cols, dense_cols - 100, replace=False),
                             rng.choice(np.arange(dense_cols, ncols), 50, replace=False)]) for _ in range(m)]
    arows = [rng.choice(m, int(rng.integers(0, 16)), replace=False) for _ in range(n)]
    return csr_from_rows(arows, m, rng), csr_from_rows(brows, ncols, rng)


@pytest.mark.parametrize("dense_cols", [2_300, 4_000])
def test_packed_columns_force_narrower_windows(dense_cols):
    A, B = packed_case(dense_cols, dense_cols)
    assert_same(product(A, B), oracle.spgemm(A, B), "default tables")
    # every row on the window path, through both phases, with one chunk per
    # row and with many
    for log2 in (30, 8):
        o = hc.opts(sym_tmax_log2=7, num_tmax=96, win_chunk_log2=log2)
        assert_same(product(A, B, o), oracle.spgemm(A, B), "forced, chunks of 2^%d products" % log2)


def test_rows_wider_than_one_bitmap_segment():
    # output columns spread over 1.3M columns: the symbolic bitmap takes each
    # row in three segments of 2^19 columns; chunk edges fall inside words
    rng = np.random.default_rng(21)
    ncols = 1_300_000
    brows = [rng.choice(ncols, int(rng.integers(1_000, 4_000)), replace=False) for _ in range(40)]
    arows = [rng.choice(40, int(rng.integers(0, 24)), replace=False) for _ in range(30)]
    A, B = csr_from_rows(arows, 40, rng), csr_from_rows(brows, ncols, rng)
    ref = oracle.spgemm(A, B)
    for o in (None, hc.opts(sym_tmax_log2=8, num_tmax=128), hc.opts(sym_tmax_log2=8, num_tmax=128, win_chunk_log2=9)):
        assert_same(product(A, B, o), ref, str(o))


def test_cluster_rows_wider_than_one_bitmap_segment():
    # member rows of clusters whose output spans 1.3M columns (three bitmap
    # segments), with few items (whole-row tasks, every segment filled by a
    # walk over all of the row's products) and with more than 1,024 items
    # (column-chunk tasks), an empty member among them
    rng = np.random.default_rng(23)
    ncols, nb = 1_300_000, 1_200
    brows = [rng.choice(ncols, int(rng.integers(20, 200)), replace=False) for _ in range(nb)]
    arows = [rng.choice(nb, m, replace=False) for m in (5, 40, 1030, 12, 1100, 300, 0, 64, 1025, 2)]
    A, B = csr_from_rows(arows, nb, rng), csr_from_rows(brows, ncols, rng)
    ref = oracle.spgemm(A, B)
    Ad, Bd = hc.DeviceCSR.from_host(A), hc.DeviceCSR.from_host(B)
    opts = (None, hc.opts(sym_tmax_log2=8, num_tmax=128), hc.opts(sym_tmax_log2=8, num_tmax=128, win_chunk_log2=9))
    for o in opts:
        assert_same(product(A, B, o), ref, "csr %s" % o)
    for K in (2, 4):
        Dc = hc.cluster_build(Ad, hc.plan_fixed(A.nrows, K))
        for o in opts:
            torch.cuda.synchronize()
            C = hc.spgemm(Dc, Bd, o)
            torch.cuda.synchronize()
            assert_same(C.to_host(), ref, "clusters of %d %s" % (K, o))


@pytest.mark.parametrize("log2", [30, 7])
def test_rows_at_the_item_limit_of_whole_row_tasks(log2):
    # rows of 1,023, 1,024 and 1,025 items (whole-row tasks up to 1,024 items,
    # column-chunk tasks beyond when the symbolic phase cut the row), plain and
    # as hierarchical clusters of up to 4 rows
    rng = np.random.default_rng(31)
    nb, ncols = 1100, 300_000
    brows = [rng.choice(ncols, int(rng.integers(5, 60)), replace=False) for _ in range(nb)]
    B = csr_from_rows(brows, ncols, rng)
    arows = [rng.choice(nb, m, replace=False) for m in (1023, 1024, 1025, 3, 1025, 1024, 700)]
    A = csr_from_rows(arows, nb, rng)
    ref = oracle.spgemm(A, B)
    o = hc.opts(sym_tmax_log2=8, num_tmax=128, win_chunk_log2=log2)
    assert_same(product(A, B, o), ref, "csr")
    Ad, Bd = hc.DeviceCSR.from_host(A), hc.DeviceCSR.from_host(B)
    Dc = hc.cluster_build(Ad, hc.plan_hierarchical(A, (1, 10), 4))
    torch.cuda.synchronize()
    C = hc.spgemm(Dc, Bd, o)
    torch.cuda.synchronize()
    assert_same(C.to_host(), ref, "clusters")


def test_rows_of_b_longer_than_the_two_byte_lengths():
    # rows of B with 65,535 entries and more: the work estimate's 2-byte row lengths saturate there and it
    # reads those rows' offsets instead; products over them, with default and with small chunks
    rng = np.random.default_rng(41)
    ncols = 300_000
    brows = [rng.choice(ncols, m, replace=False) for m in (65_534, 65_535, 65_536, 90_000)]
    brows += [rng.choice(ncols, int(rng.integers(1, 50)), replace=False) for _ in range(20)]
    B = csr_from_rows(brows, ncols, rng)
    arows = [[0], [1], [2], [3], [0, 1, 2, 3], [3, 7, 9], [5, 6], [], [1, 23]]
    A = csr_from_rows([np.array(r, np.int64) for r in arows], len(brows), rng)
    ref = oracle.spgemm(A, B)
    for o in (None, hc.opts(win_chunk_log2=12)):
        assert_same(product(A, B, o), ref, str(o))


def test_rows_counted_whole_then_windowed():
    # symbolic tables large enough for every row, numeric tables too small:
    # the numeric phase takes each row as one chunk over its column range
    A = synth.uniform(400, 300, 24, 31)
    B = synth.uniform(300, 5000, 40, 32)
    o = hc.opts(num_tmax=96)
    assert_same(product(A, B, o), oracle.spgemm(A, B))


@pytest.mark.parametrize("scale", [11, 13])
def test_rmat_window_path_bitwise(scale):
    R = synth.rmat(scale, 16, 0.57, 0.19, 0.19, 5)
    ref = oracle.spgemm(R, R)
    assert_same(product(R, R), ref, "default")
    assert_same(product(R, R, hc.opts(sym_tmax_log2=8, num_tmax=128)), ref, "small tables")
    assert_same(product(R, R, hc.opts(sym_tmax_log2=8, num_tmax=128, win_chunk_log2=6)), ref, "many chunks")


def test_rmat16_whole_product_bitwise():
    # 65,536 rows, 1.24e9 products, 3.5e8 entries: most products on the
    # long-row path (bitmaps, whole-row tasks and column-chunk tasks)
    import os
    R = synth.workload_rmat(16, 4)
    ref = oracle.spgemm_mt(R, R, min(16, len(os.sched_getaffinity(0))))
    assert_same(product(R, R), ref, "rmat16")


def test_window_rows_in_panels():
    R = synth.rmat(11, 16, 0.57, 0.19, 0.19, 6)
    D = hc.DeviceCSR.from_host(R)
    o0 = hc.opts(sym_tmax_log2=7, num_tmax=96, win_chunk_log2=7)
    P = hc.Product(D, D, o0)
    nnz = P.symbolic()
    rp = P.C_row_ptr.cpu().numpy()
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz)
    cuts = [0, 1, 700, 701, 1500, R.nrows]
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        base, end = int(rp[lo]), int(rp[hi])
        bc = torch.empty(max(end - base, 1), dtype=torch.int32, device="cuda")
        bv = torch.empty(max(end - base, 1), dtype=torch.float64, device="cuda")
        o = hc.opts(sym_tmax_log2=7, num_tmax=96, win_chunk_log2=7, unit_lo=lo, unit_hi=hi, out_base=base,
                    flags=hc.F_SYNC_CHECK)
        hc.spgemm_numeric(D, D, P.info, P.C_row_ptr, bc, bv, P.ws, o, capacity=end - base)
        col[base:end] = bc[:end - base].cpu().numpy()
        val[base:end] = bv[:end - base].cpu().numpy()
    ref = oracle.spgemm(R, R)
    np.testing.assert_array_equal(rp, ref.rp)
    np.testing.assert_array_equal(col, ref.col)
    np.testing.assert_array_equal(val, ref.val)


def test_window_capacity_too_small_is_reported():
    A, B = packed_case(7, 2_300)
    Ad, Bd = hc.DeviceCSR.from_host(A), hc.DeviceCSR.from_host(B)
    P = hc.Product(Ad, Bd)
    nnz = P.symbolic()
    assert nnz > 10
    small = nnz // 2
    col = torch.zeros(small, dtype=torch.int32, device="cuda")
    val = torch.zeros(small, dtype=torch.float64, device="cuda")
    with pytest.raises(hc.HcspError):
        hc.spgemm_numeric(Ad, Bd, P.info, P.C_row_ptr, col, val, P.ws, hc.opts(flags=hc.F_SYNC_CHECK),
                          capacity=small)


def test_numeric_with_other_chunking_is_refused():
    A, B = packed_case(8, 2_300)
    Ad, Bd = hc.DeviceCSR.from_host(A), hc.DeviceCSR.from_host(B)
    P = hc.Product(Ad, Bd, hc.opts(win_chunk_log2=8))
    nnz = P.symbolic()
    col = torch.zeros(nnz, dtype=torch.int32, device="cuda")
    val = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    with pytest.raises(hc.HcspError):
        hc.spgemm_numeric(Ad, Bd, P.info, P.C_row_ptr, col, val, P.ws, hc.opts(win_chunk_log2=9), capacity=nnz)
    hc.spgemm_numeric(Ad, Bd, P.info, P.C_row_ptr, col, val, P.ws, hc.opts(win_chunk_log2=8, flags=hc.F_SYNC_CHECK),
                      capacity=nnz)
    ref = oracle.spgemm(A, B)
    np.testing.assert_array_equal(col.cpu().numpy(), ref.col)
    np.testing.assert_array_equal(val.cpu().numpy(), ref.val)


@pytest.mark.parametrize("plan_kind", ["fixed4", "hier8"])
def test_clusters_on_window_path(plan_kind):
    # a CSR_Cluster A whose clusters outgrow shared memory: each member row
    # takes the window path on its own (union columns with its mask bit)
    A, B = packed_case(11, 2_300, m=30, n=60)
    Ad, Bd = hc.DeviceCSR.from_host(A), hc.DeviceCSR.from_host(B)
    plan = hc.plan_fixed(A.nrows, 4) if plan_kind == "fixed4" else hc.plan_hierarchical(A, (1, 10), 8)
    Dc = hc.cluster_build(Ad, plan)
    ref = oracle.spgemm(A, B)
    for o in (None, hc.opts(sym_tmax_log2=7, num_tmax=96), hc.opts(sym_tmax_log2=7, num_tmax=96, win_chunk_log2=8),
              hc.opts(num_tmax=96)):
        torch.cuda.synchronize()
        C = hc.spgemm(Dc, Bd, o)
        torch.cuda.synchronize()
        assert_same(C.to_host(), ref, "%s %s" % (plan_kind, o))


def test_rmat_clusters_on_window_path():
    R = synth.rmat(12, 16, 0.57, 0.19, 0.19, 7)
    Rd = hc.DeviceCSR.from_host(R)
    plan = hc.plan_hierarchical(R, (3, 10), 4, perm_in=hc.order_rcm(R))
    Dc = hc.cluster_build(Rd, plan)
    ref = oracle.spgemm(R, R)
    for o in (None, hc.opts(sym_tmax_log2=8, num_tmax=128, win_chunk_log2=6)):
        torch.cuda.synchronize()
        C = hc.spgemm(Dc, Rd, o)
        torch.cuda.synchronize()
        assert_same(C.to_host(), ref, str(o))


def test_too_many_window_pairs_is_reported():
    # 20,000 rows of 4,096 products each, all on the window path and cut into
    # 256 chunks each: 5.1M (row, chunk) pairs, more than the workspace holds
    # counts for (4 per row + 4M); the call fails cleanly, and fewer chunks fit
    A = synth.uniform(20_000, 2_000, 16, 41)
    B = synth.uniform(2_000, 100_000, 256, 42)
    Ad, Bd = hc.DeviceCSR.from_host(A), hc.DeviceCSR.from_host(B)
    with pytest.raises(hc.HcspError) as e:
        hc.spgemm(Ad, Bd, hc.opts(sym_tmax_log2=7, num_tmax=96, win_chunk_log2=4))
    assert "win_chunk_log2" in str(e.value)
    torch.cuda.synchronize()
    C = hc.spgemm(Ad, Bd, hc.opts(sym_tmax_log2=7, num_tmax=96, win_chunk_log2=12))
    torch.cuda.synchronize()
    assert_same(C.to_host(), oracle.spgemm(A, B))
