"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Structure and values must match bit for bit: both sides add each output
entry's products in ascending k with fused multiply-adds from +0.0, so any
difference is a bug (the 1e-12 relative tolerance the product contract allows
is never needed here).  Sizes span several bins, ragged rows and empty rows.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2507_21253_amd as hc  # noqa: E402


def to_dev(H):
    return hc.DeviceCSR.from_host(H)


def gpu_product(A_dev, B_dev, o=None):
    torch.cuda.synchronize()
    C = hc.spgemm(A_dev, B_dev, o)
    torch.cuda.synchronize()
    return C.to_host()


def assert_same(Cg, Cr, where=""):
    np.testing.assert_array_equal(Cg.rp, Cr.rp, err_msg="row_ptr " + where)
    np.testing.assert_array_equal(Cg.col, Cr.col, err_msg="col " + where)
    np.testing.assert_array_equal(Cg.val, Cr.val, err_msg="val " + where)


def ragged(seed, n, m, p):
    """Rows of very different lengths, some empty; explicit zeros stored."""
    rng = np.random.default_rng(seed)
    dens = rng.choice([0.0, 0.01, 0.05, 0.3, 0.9], size=n)
    pat = rng.random((n, m)) < dens[:, None]
    vals = rng.uniform(-1, 1, (n, m))
    vals[rng.random((n, m)) < 0.05] = 0.0
    A = synth.from_dense(np.where(pat, vals, 0.0), pat)
    pb = rng.random((m, p)) < rng.choice([0.0, 0.02, 0.1, 0.5], size=m)[:, None]
    B = synth.from_dense(np.where(pb, rng.uniform(-1, 1, (m, p)), 0.0), pb)
    return A, B


def test_uniform_2000_bitwise():
    A = synth.workload_uniform_2000()
    Ad = to_dev(A)
    assert_same(gpu_product(Ad, Ad), oracle.spgemm(A, A))


@pytest.mark.parametrize("seed", range(6))
def test_ragged_random_bitwise(seed):
    rng = np.random.default_rng(100 + seed)
    n, m, p = (int(x) for x in rng.integers(1, 400, 3))
    A, B = ragged(seed, n, m, p)
    assert_same(gpu_product(to_dev(A), to_dev(B)), oracle.spgemm(A, B), "seed %d" % seed)


@pytest.mark.parametrize("kind,m", [(5, 40), (7, 14), (27, 10)])
def test_stencils_bitwise(kind, m):
    S = synth.stencil(kind, m, 7)
    Sd = to_dev(S)
    assert_same(gpu_product(Sd, Sd), oracle.spgemm(S, S))


def test_relabelled_stencil_bitwise():
    M, _, _ = synth.workload_stencil27(12, 2, 3)
    Md = to_dev(M)
    assert_same(gpu_product(Md, Md), oracle.spgemm(M, M))


@pytest.mark.parametrize("d", [1, 3, 9, 40, 130])
def test_row_length_mix(d):
    # B rows from 1 to 130 entries: items shorter and longer than a 64-lane pass
    A = synth.uniform(700, 500, 9, 5)
    B = synth.uniform(500, 900, d, 6)
    assert_same(gpu_product(to_dev(A), to_dev(B), hc.opts(lanes=64)), oracle.spgemm(A, B))


def test_long_items_cross_rounds():
    # rows whose products exceed one 4096-entry round, items cut across rounds
    A = synth.uniform(40, 3000, 60, 7)
    B = synth.uniform(3000, 5000, 150, 8)
    assert_same(gpu_product(to_dev(A), to_dev(B)), oracle.spgemm(A, B))


def test_bad_lanes_rejected():
    A = to_dev(synth.uniform(10, 10, 2, 1))
    with pytest.raises(hc.HcspError):
        hc.spgemm(A, A, hc.opts(lanes=32))


def plans_for(A):
    yield "fixed4", hc.plan_fixed(A.nrows, 4)
    yield "fixed16_perm", hc.plan_fixed(A.nrows, 16, synth.perm(A.nrows, 9))
    yield "variable", hc.plan_variable(A, (3, 10), 8)
    yield "variable_t0", hc.plan_variable(A, (0, 1), 3)
    yield "hier_root", hc.plan_hierarchical(A, (3, 10), 8, hc.SIM_ROOT)
    yield "hier_union", hc.plan_hierarchical(A, (3, 10), 8, hc.SIM_UNION)
    yield "hier_perm16", hc.plan_hierarchical(A, (1, 5), 16, hc.SIM_ROOT, perm_in=synth.perm(A.nrows, 4))
    # the benchmark's method path: rows in reverse Cuthill-McKee order, pairs by hierarchical clustering
    yield "hier_rcm2", hc.plan_hierarchical(A, (3, 10), 2, hc.SIM_ROOT, perm_in=oracle.order_rcm(A))


def host_cluster_of(Dc):
    return dict(cl_col_ptr=Dc.cl_col_ptr.cpu().numpy(), cl_col=Dc.cl_col.cpu().numpy(),
                cl_mask=Dc.cl_mask.cpu().numpy().view(np.uint16), cl_val_ptr=Dc.cl_val_ptr.cpu().numpy(),
                cl_val=Dc.cl_val.cpu().numpy())


def test_cluster_build_matches_oracle():
    M, _, _ = synth.workload_stencil27(9, 2, 3)
    Md = to_dev(M)
    for name, plan in plans_for(M):
        ref = oracle.cluster_build(M, oracle.Plan(plan.perm, plan.cl_row_ptr))
        Dc = hc.cluster_build(Md, plan)
        torch.cuda.synchronize()
        got = host_cluster_of(Dc)
        for k in got:
            np.testing.assert_array_equal(got[k], getattr(ref, k), err_msg="%s %s" % (name, k))
        assert Dc.max_cluster == int(np.diff(plan.cl_row_ptr).max())


@pytest.mark.parametrize("which", ["stencil_relabel", "uniform", "ragged"])
def test_clustered_product_bitwise(which):
    if which == "stencil_relabel":
        A, _, _ = synth.workload_stencil27(10, 2, 3)
        B = A
    elif which == "uniform":
        A = synth.uniform(600, 400, 8, 3)
        B = synth.uniform(400, 700, 12, 4)
    else:
        A, B = ragged(7, 300, 250, 280)
    ref = oracle.spgemm(A, B)
    Ad, Bd = to_dev(A), to_dev(B)
    for name, plan in plans_for(A):
        Dc = hc.cluster_build(Ad, plan)
        assert_same(gpu_product(Dc, Bd), ref, name)


def test_forced_dense_path_bitwise():
    # tiny shared-memory tables push every unit onto the global-memory path
    A = synth.uniform(300, 200, 20, 8)
    B = synth.uniform(200, 350, 25, 9)
    o = hc.opts(sym_tmax_log2=7, num_tmax=96)
    ref = oracle.spgemm(A, B)
    assert_same(gpu_product(to_dev(A), to_dev(B), o), ref, "csr")
    plan = hc.plan_hierarchical(A, (1, 10), 8)
    assert_same(gpu_product(hc.cluster_build(to_dev(A), plan), to_dev(B), o), ref, "cluster")


def test_rmat_small_bitwise():
    R = synth.rmat(12, 16, 0.57, 0.19, 0.19, 4)
    Rd = to_dev(R)
    ref = oracle.spgemm(R, R)
    assert_same(gpu_product(Rd, Rd), ref, "csr")
    plan = hc.plan_hierarchical(R, (3, 10), 8)
    assert_same(gpu_product(hc.cluster_build(Rd, plan), Rd), ref, "hier")


def test_empty_and_degenerate():
    Z = synth.HostCSR(np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0), 5, 4)
    B = synth.uniform(4, 7, 2, 1)
    C = gpu_product(to_dev(Z), to_dev(B))
    assert C.rp.tolist() == [0] * 6 and len(C.col) == 0
    A = synth.uniform(5, 4, 2, 2)
    Bz = synth.HostCSR(np.zeros(5, np.int64), np.zeros(0, np.int32), np.zeros(0), 4, 9)
    C = gpu_product(to_dev(A), to_dev(Bz))
    assert C.rp.tolist() == [0] * 6
    one = synth.from_dense(np.array([[2.0]]))
    C = gpu_product(to_dev(one), to_dev(one))
    assert C.col.tolist() == [0] and C.val.tolist() == [4.0]
    # inner dimension zero: A has no columns, B no rows
    A0 = synth.HostCSR(np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0), 5, 0)
    B0 = synth.HostCSR(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0), 0, 9)
    C = gpu_product(to_dev(A0), to_dev(B0))
    assert C.rp.tolist() == [0] * 6 and len(C.col) == 0


def test_panels_with_out_base():
    A = synth.uniform(1000, 800, 7, 21)
    B = synth.uniform(800, 900, 11, 22)
    Ad, Bd = to_dev(A), to_dev(B)
    P = hc.Product(Ad, Bd)
    nnz = P.symbolic()
    rp = P.C_row_ptr.cpu().numpy()
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz)
    for lo, hi in [(0, 333), (333, 334), (334, 1000)]:
        base, end = int(rp[lo]), int(rp[hi])
        bc = torch.empty(end - base, dtype=torch.int32, device="cuda")
        bv = torch.empty(end - base, dtype=torch.float64, device="cuda")
        o = hc.opts(unit_lo=lo, unit_hi=hi, out_base=base, flags=hc.F_SYNC_CHECK)
        hc.spgemm_numeric(Ad, Bd, P.info, P.C_row_ptr, bc, bv, P.ws, o, capacity=end - base)
        col[base:end] = bc.cpu().numpy()
        val[base:end] = bv.cpu().numpy()
    ref = oracle.spgemm(A, B)
    np.testing.assert_array_equal(rp, ref.rp)
    np.testing.assert_array_equal(col, ref.col)
    np.testing.assert_array_equal(val, ref.val)


def test_capacity_too_small_is_reported_and_bounded():
    A = synth.uniform(200, 200, 6, 31)
    Ad = to_dev(A)
    P = hc.Product(Ad, Ad)
    nnz = P.symbolic()
    cap = nnz // 2
    guard = 4096
    bc = torch.full((cap + guard,), -7, dtype=torch.int32, device="cuda")
    bv = torch.full((cap + guard,), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(hc.HcspError) as e:
        hc.spgemm_numeric(Ad, Ad, P.info, P.C_row_ptr, bc, bv, P.ws, hc.opts(flags=hc.F_SYNC_CHECK), capacity=cap)
    assert e.value.status == -5
    assert bool((bc[cap:] == -7).all()) and bool((bv[cap:] == -7.0).all())


def test_csr_check_reports_malformed_inputs():
    A = synth.uniform(50, 40, 5, 3)
    assert hc.csr_check(to_dev(A)) == 0
    bad = synth.HostCSR(A.rp.copy(), A.col.copy(), A.val, 50, 40)
    bad.col[7], bad.col[8] = bad.col[8], bad.col[7]
    assert hc.csr_check(to_dev(bad)) == -4
    bad = synth.HostCSR(A.rp.copy(), A.col.copy(), A.val, 50, 40)
    bad.col[3] = 40
    assert hc.csr_check(to_dev(bad)) == -3
    bad = synth.HostCSR(A.rp.copy(), A.col.copy(), A.val, 50, 40)
    bad.rp[10] = bad.rp[11] + 1
    assert hc.csr_check(to_dev(bad)) == -2


def test_run_twice_bitwise_identical():
    M, _, _ = synth.workload_stencil27(12, 5, 6)
    Md = to_dev(M)
    plan = hc.plan_hierarchical(M, (3, 10), 8)
    Dc = hc.cluster_build(Md, plan)
    P = hc.Product(Dc, Md)
    C1 = P.run().to_host()
    C2 = P.run().to_host()
    assert_same(C1, C2)


def _clumped_case(n=300, seed=11):
    """Output rows whose columns crowd at the top of their range: the order-preserving numeric hash sends
    them all to the last home slots, so probe runs pass the end of the table and wrap around (the general
    ranking), next to rows that do not wrap (the occupancy-bitmap ranking)."""
    rng = np.random.default_rng(seed)
    brows = [np.array([0]), np.arange(10000, 10100), np.arange(20000, 20150),
             np.concatenate([[5000], np.arange(29990, 30000)]), np.sort(rng.choice(30000, 120, replace=False))]
    bvals = [rng.uniform(-1, 1, len(c)) for c in brows]
    B = synth.HostCSR(np.concatenate([[0], np.cumsum([len(c) for c in brows])]).astype(np.int64),
                      np.concatenate(brows).astype(np.int32), np.concatenate(bvals), len(brows), 30000)
    acols = [np.array(sorted({0, 1 + i % 4} | ({4} if i % 5 == 0 else set()))) for i in range(n)]
    A = synth.HostCSR(np.concatenate([[0], np.cumsum([len(c) for c in acols])]).astype(np.int64),
                      np.concatenate(acols).astype(np.int32), rng.uniform(-1, 1, sum(len(c) for c in acols)),
                      n, len(brows))
    return A, B


@pytest.mark.parametrize("load", [50, 60, 90])
def test_wrapped_probe_runs_bitwise(load):
    A, B = _clumped_case()
    ref = oracle.spgemm(A, B)
    Ad, Bd = to_dev(A), to_dev(B)
    assert_same(gpu_product(Ad, Bd, hc.opts(load_pct=load)), ref, "csr load %d" % load)
    for K in (2, 3):
        Dc = hc.cluster_build(Ad, hc.plan_fixed(A.nrows, K))
        assert_same(gpu_product(Dc, Bd, hc.opts(load_pct=load)), ref, "clusters of %d, load %d" % (K, load))


def _ref_cluster_out(A, B, plan):
    """The oracle's C = A*B put into CSR_Cluster form on the plan's clusters."""
    return oracle.cluster_build(oracle.spgemm(A, B), oracle.Plan(plan.perm, plan.cl_row_ptr))


@pytest.mark.parametrize("which", ["stencil_relabel", "ragged"])
def test_cluster_output_bitwise(which):
    # C written in CSR_Cluster form (Alg. 1's output) equals the oracle's C clustered on A's clusters
    if which == "stencil_relabel":
        A, _, _ = synth.workload_stencil27(9, 2, 3)
        B = A
    else:
        A, B = ragged(21, 300, 250, 280)
    Ad, Bd = to_dev(A), to_dev(B)
    for name, plan in plans_for(A):
        Dc = hc.cluster_build(Ad, plan)
        C = hc.spgemm_cluster_out(Dc, Bd)
        torch.cuda.synchronize()
        ref = _ref_cluster_out(A, B, plan)
        got = host_cluster_of(C)
        for k in got:
            np.testing.assert_array_equal(got[k], getattr(ref, k), err_msg="%s %s %s" % (which, name, k))


def test_cluster_output_chains():
    # a clustered C is the left operand of the next product as it stands: (A*A)*A with A*A kept clustered
    A, _, _ = synth.workload_stencil27(8, 2, 3)
    Ad = to_dev(A)
    plan = hc.plan_hierarchical(A, (3, 10), 4, hc.SIM_ROOT, perm_in=oracle.order_rcm(A))
    C2 = hc.spgemm_cluster_out(hc.cluster_build(Ad, plan), Ad)
    C3 = hc.spgemm(C2, Ad)
    torch.cuda.synchronize()
    assert_same(C3.to_host(), oracle.spgemm(oracle.spgemm(A, A), A))


def test_concurrent_host_threads_on_own_streams():
    # two host threads, each with its own stream, run products at once: the library's side streams for
    # small bins are shared, so their fork/join must stay per call (results bitwise, no hang)
    import threading
    cases = [synth.workload_stencil27(10, 2, 3)[0], synth.rmat(11, 16, 0.57, 0.19, 0.19, 6)]
    refs = [oracle.spgemm(A, A) for A in cases]
    devs = [to_dev(A) for A in cases]
    errors = []

    def work(k):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(4):
                    C = hc.Product(devs[k], devs[k]).run(s)
                    s.synchronize()
                    got = C.to_host()
                    assert np.array_equal(got.rp, refs[k].rp) and np.array_equal(got.col, refs[k].col)
                    assert np.array_equal(got.val, refs[k].val)
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append(repr(e))

    th = [threading.Thread(target=work, args=(k,)) for k in (0, 1)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in th), "a thread did not finish"
    assert not errors, errors


@pytest.mark.parametrize("maxc,sim", [(4, hc.SIM_ROOT), (2, hc.SIM_ROOT), (8, hc.SIM_UNION)])
def test_benchmark_configuration_bitwise(maxc, sim):
    # the benchmark's configuration on a 32^3 relabelled 27-point stencil: rows of A in reverse
    # Cuthill-McKee order, hierarchical clusters (the tuned size 4, and 2 / 8), symbolic tables filled up to
    # 100 %, numeric tables 70 % (clustered) and 50 % (plain, given order and RCM rows)
    M, _, _ = synth.workload_stencil27(32, 2, 3)
    ref = oracle.spgemm(M, M)
    Md = to_dev(M)
    rcm = oracle.order_rcm(M)
    plan = hc.plan_hierarchical(M, (3, 10), maxc, sim, perm_in=rcm)
    Dc = hc.cluster_build(Md, plan)
    for o in (hc.opts(sym_load_pct=100, load_pct=70), hc.opts(sym_load_pct=70, load_pct=70),
              hc.opts(sym_load_pct=100, load_pct=85)):
        assert_same(gpu_product(Dc, Md, o), ref, "clustered %d s%d n%d" % (maxc, o.sym_load_pct, o.load_pct))
    o = hc.opts(sym_load_pct=100, load_pct=50)
    assert_same(gpu_product(Md, Md, o), ref, "plain")
    R = hc.permute_h(M, rcm)
    C = gpu_product(to_dev(R), Md, o)
    np.testing.assert_array_equal(np.diff(C.rp), np.diff(ref.rp)[rcm])    # rows of C in RCM order
    inv = np.empty_like(rcm)
    inv[rcm] = np.arange(len(rcm))
    for r in (0, 1, M.nrows // 2, M.nrows - 1):
        p = inv[r]
        np.testing.assert_array_equal(C.col[C.rp[p]:C.rp[p + 1]], ref.col[ref.rp[r]:ref.rp[r + 1]])
        np.testing.assert_array_equal(C.val[C.rp[p]:C.rp[p + 1]], ref.val[ref.rp[r]:ref.rp[r + 1]])


def test_status_reports_dropped_writes_without_sync_flag():
    # the numeric phase's error word, read back by hcsp_spgemm_status after an asynchronous call
    A = synth.uniform(200, 200, 6, 31)
    Ad = to_dev(A)
    P = hc.Product(Ad, Ad)
    nnz = P.symbolic()
    cap = nnz // 3
    bc = torch.empty(cap, dtype=torch.int32, device="cuda")
    bv = torch.empty(cap, dtype=torch.float64, device="cuda")
    hc.spgemm_numeric(Ad, Ad, P.info, P.C_row_ptr, bc, bv, P.ws, capacity=cap)
    with pytest.raises(hc.HcspError) as e:
        hc.spgemm_status(P.ws)
    assert e.value.status == -5
    P.run()                                     # a full run clears it
    hc.spgemm_status(P.ws)


def test_large_tables_bitwise():
    # units whose numeric tables hold 1024 slots or more place keys by a multiplicative hash and rank them by
    # a bucket sort: R-MAT rows (output columns crowded at the low-numbered hubs), uniform rows of ~830
    # outputs, two-row clusters of those, C written as CSR_Cluster, and the predicted-size product
    R = synth.rmat(13, 16, 0.57, 0.19, 0.19, 31)
    Rd = to_dev(R)
    ref = oracle.spgemm(R, R)
    cnt = np.diff(ref.rp)
    assert ((cnt >= 700) & (cnt <= 4300)).sum() > 4000  # rows in the hashed shared-memory bins
    assert_same(gpu_product(Rd, Rd), ref, "rmat13")
    plan = hc.plan_hierarchical(R, (3, 10), 2, hc.SIM_ROOT)
    assert_same(gpu_product(hc.cluster_build(Rd, plan), Rd), ref, "rmat13 clusters")
    U = synth.uniform(5000, 5000, 30, 32)
    Ud = to_dev(U)
    refu = oracle.spgemm(U, U)
    assert_same(gpu_product(Ud, Ud), refu, "uniform")
    plan2 = hc.plan_fixed(U.nrows, 2)
    Uc = hc.cluster_build(Ud, plan2)
    assert_same(gpu_product(Uc, Ud), refu, "uniform pairs")
    C = hc.spgemm_cluster_out(Uc, Ud)
    torch.cuda.synchronize()
    got = host_cluster_of(C)
    want = _ref_cluster_out(U, U, plan2)
    for k in got:
        np.testing.assert_array_equal(got[k], getattr(want, k), err_msg="uniform pairs CSR_Cluster %s" % k)
    P = hc.PredictedProduct(Ud, Ud, 1.02 * refu.nnz / int(np.diff(U.rp)[U.col].sum()))
    Cp = P.run()
    torch.cuda.synchronize()
    assert_same(Cp.to_host(), refu, "uniform predicted")
