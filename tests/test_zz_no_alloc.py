"""The entry point that allocates nothing (hcsp_spgemm_noalloc): its workspace
is the library's static device array.  Its C must equal, bit for bit, the C
of the symbolic + numeric entry points on the same inputs and options (and
the oracle's), over two calls in a row, the second with a smaller input (the
array keeps the first call's contents); sizes beyond the array and an output
that is too small are refused with HCSP_E_CAPACITY."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2507_21253_amd as hc  # noqa: E402


def noalloc_product(A, B, o=None, capacity=None):
    dev = B.row_ptr.device
    rp = torch.full((A.nrows + 1,), -7, dtype=torch.int64, device=dev)
    cap = capacity
    if cap is None:
        cap = hc.Product(A, B, o).symbolic()
    col = torch.full((max(cap, 1),), -7, dtype=torch.int32, device=dev)[:cap]
    val = torch.full((max(cap, 1),), np.nan, dtype=torch.float64, device=dev)[:cap]
    nnz = hc.spgemm_noalloc(A, B, rp, col, val, o)
    torch.cuda.synchronize()
    return nnz, rp.cpu().numpy(), col[:nnz].cpu().numpy(), val[:nnz].cpu().numpy()


def check(A, B, Ah, Bh, o=None):
    nnz, rp, col, val = noalloc_product(A, B, o)
    ref = hc.spgemm(A, B, o).to_host()
    torch.cuda.synchronize()
    print("noalloc: %d rows, nnz(C) = %d" % (A.nrows, nnz), flush=True)
    assert nnz == len(ref.col)
    np.testing.assert_array_equal(rp, ref.rp)
    np.testing.assert_array_equal(col, ref.col)
    np.testing.assert_array_equal(val, ref.val)
    orc = oracle.spgemm(Ah, Bh)
    np.testing.assert_array_equal(rp, orc.rp)
    np.testing.assert_array_equal(col, orc.col)
    np.testing.assert_array_equal(val, orc.val)


def test_noalloc_two_calls_second_smaller():
    # first: a clustered relabelled stencil (several bins, clusters of up to 4 rows)
    M, _, _ = synth.workload_stencil27(24, 2, 3)
    Md = hc.DeviceCSR.from_host(M)
    plan = hc.plan_hierarchical(M, (3, 10), 4)
    Mc = hc.cluster_build(Md, plan)
    check(Mc, Md, M, M, hc.opts(load_pct=70, sym_load_pct=100))
    # second, smaller: plain CSR, ragged uniform rows
    U = synth.uniform(3000, 2500, 9, 17)
    V = synth.uniform(2500, 3100, 5, 18)
    check(hc.DeviceCSR.from_host(U), hc.DeviceCSR.from_host(V), U, V)


def test_noalloc_refuses_sizes_beyond_the_scratch():
    n = 2_000_000  # the workspace of a 2e6-row product exceeds the static array
    rp = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    col = torch.zeros(1, dtype=torch.int32, device="cuda")
    val = torch.zeros(1, dtype=torch.float64, device="cuda")
    A = hc.DeviceCSR(rp, col[:0], val[:0], n, n)
    assert hc.spgemm_workspace(A, A) > hc.NOALLOC_SCRATCH_BYTES
    out_rp = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(hc.HcspError) as e:
        hc.spgemm_noalloc(A, A, out_rp, col, val)
    assert e.value.status == -5 and "static scratch" in str(e.value)


def test_noalloc_refuses_a_small_output_then_recovers():
    U = synth.uniform(800, 800, 6, 5)
    Ud = hc.DeviceCSR.from_host(U)
    nnz_true = hc.Product(Ud, Ud).symbolic()
    rp = torch.empty(U.nrows + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(nnz_true - 1, dtype=torch.int32, device="cuda")
    val = torch.empty(nnz_true - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(hc.HcspError) as e:
        hc.spgemm_noalloc(Ud, Ud, rp, col, val)
    assert e.value.status == -5 and "exceeds the capacity" in str(e.value)
    # the same call with room for C succeeds and equals the oracle
    check(Ud, Ud, U, U)
