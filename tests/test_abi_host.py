"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point the public header declares, and its host cluster plans give
exactly the oracle's plans."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2507_21253_amd as hc
import synth

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "hcsp.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hcsp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = hc.lib()
    names = declared_symbols()
    assert len(names) == len(hc._SIGS)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(hc._SIGS), "binding and header disagree"
    assert hc.version().startswith("hcsp")
    assert hc.strerror(-5) == "buffer too small"


def same_plan(p, q):
    np.testing.assert_array_equal(p.perm, q.perm)
    np.testing.assert_array_equal(p.cl_row_ptr, q.cl_row_ptr)


@pytest.mark.parametrize("K", [1, 3, 8, 16])
def test_plan_fixed_matches_oracle(K):
    pi = synth.perm(37, 5)
    same_plan(hc.plan_fixed(37, K), oracle.plan_fixed(37, K))
    same_plan(hc.plan_fixed(37, K, pi), oracle.plan_fixed(37, K, pi))


def inputs():
    yield "uniform", synth.uniform(300, 120, 6, 3)
    yield "stencil27", synth.stencil(27, 6, 2)
    M, _, _ = synth.workload_stencil27(7, 2, 3)
    yield "stencil27_relabel", M
    yield "rmat10", synth.rmat(10, 16, 0.57, 0.19, 0.19, 4)
    yield "stencil5", synth.stencil(5, 20, 1)


@pytest.mark.parametrize("t,maxc", [((3, 10), 8), ((1, 5), 4), ((0, 1), 16), ((1, 2), 2)])
def test_plan_variable_matches_oracle(t, maxc):
    for name, A in inputs():
        same_plan(hc.plan_variable(A, t, maxc), oracle.plan_variable(A, t, maxc))
        pi = synth.perm(A.nrows, 11)
        same_plan(hc.plan_variable(A, t, maxc, pi), oracle.plan_variable(A, t, maxc, pi))


@pytest.mark.parametrize("sim", [hc.SIM_ROOT, hc.SIM_UNION])
@pytest.mark.parametrize("t,maxc", [((3, 10), 8), ((1, 5), 4), ((1, 3), 16), ((1, 2), 2), ((3, 10), 1)])
def test_plan_hierarchical_matches_oracle(sim, t, maxc):
    for name, A in inputs():
        ref = oracle.plan_hierarchical(A, t, maxc, sim)
        for nthreads in (1, 3):
            same_plan(hc.plan_hierarchical(A, t, maxc, sim, nthreads), ref)
        pi = synth.perm(A.nrows, 12)
        same_plan(hc.plan_hierarchical(A, t, maxc, sim, 2, pi), oracle.plan_hierarchical(A, t, maxc, sim, pi))


@pytest.mark.parametrize("sim", [hc.SIM_ROOT, hc.SIM_UNION])
@pytest.mark.parametrize("t,maxc", [((3, 10), 8), ((1, 5), 4), ((1, 2), 2)])
def test_plan_from_given_candidates_matches_oracle(sim, t, maxc):
    # the merge loop alone, fed with the oracle's SpGEMM_TopK lists, gives the oracle's plan
    for name, A in inputs():
        for pi in (None, synth.perm(A.nrows, 13)):
            cnt, nbr, ov, _ = oracle.topk_candidates(A, t, maxc - 1, pi)
            same_plan(hc.plan_hierarchical_candidates(A, t, maxc, sim, cnt, nbr, ov, pi),
                      oracle.plan_hierarchical(A, t, maxc, sim, pi))


def test_plan_hierarchical_hand_examples_both_readings():
    # the library's plans on the hand-worked examples, under both readings of the merged-cluster similarity
    import json
    from test_oracle import csr_from_rows
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hierarchical_hand_examples.json")))
    for ex in g["examples"]:
        A = csr_from_rows(ex["rows"], ex["ncols"])
        for case in ex["cases"]:
            for sim, key in ((hc.SIM_ROOT, "expected_clusters_root"), (hc.SIM_UNION, "expected_clusters_union")):
                p = hc.plan_hierarchical(A, tuple(case["jacc_th"]), case["max_cluster"], sim, 1)
                got = [p.perm[p.cl_row_ptr[c]:p.cl_row_ptr[c + 1]].tolist() for c in range(p.nclusters)]
                assert got == case.get(key, case.get("expected_clusters")), case["trace"]


def test_plan_from_candidates_rejects_bad_lists():
    A = synth.stencil(27, 4, 2)
    cnt, nbr, ov, _ = oracle.topk_candidates(A, (3, 10), 3)
    bad = nbr.copy()
    bad[0, 0] = A.nrows                                   # partner out of range
    cnt1 = cnt.copy()
    cnt1[0] = max(cnt1[0], 1)
    with pytest.raises(hc.HcspError):
        hc.plan_hierarchical_candidates(A, (3, 10), 4, hc.SIM_ROOT, cnt1, bad, ov)
    with pytest.raises(hc.HcspError):
        hc.plan_hierarchical_candidates(A, (3, 10), 4, hc.SIM_ROOT, np.full_like(cnt, 4), nbr, ov)


def test_plan_hierarchical_larger_multithreaded():
    M, _, _ = synth.workload_stencil27(20, 2, 3)
    same_plan(hc.plan_hierarchical(M, (3, 10), 8, hc.SIM_ROOT, 8), oracle.plan_hierarchical(M, (3, 10), 8))


def test_plan_argument_errors():
    A = synth.uniform(10, 10, 3, 1)
    with pytest.raises(hc.HcspError) as e:
        hc.plan_fixed(10, 0)
    assert e.value.status == -1
    with pytest.raises(hc.HcspError):
        hc.plan_variable(A, (1, 0), 8)
    with pytest.raises(hc.HcspError):
        hc.plan_hierarchical(A, (3, 10), 17)
    bad = np.zeros(10, np.int32)                      # not a permutation
    with pytest.raises(hc.HcspError) as e:
        hc.plan_hierarchical(A, (3, 10), 8, perm_in=bad)
    assert "permutation" in str(e.value)


def test_workspace_query_is_host_only():
    # shape checks and the size query need no device
    B = hc.DeviceCSR.__new__(hc.DeviceCSR)
    op = hc.c_operand()
    op.kind = hc.OP_CSR
    op.csr = hc.c_csr(100, 50, 10, 1, 1, 1)
    b = hc.c_csr(50, 70, 10, 1, 1, 1)
    n = ctypes.c_size_t()
    rc = hc.lib().hcsp_spgemm_workspace(ctypes.byref(op), ctypes.byref(b), None, ctypes.byref(n))
    assert rc == 0 and n.value > 0
    # rows too long for shared memory take the column-window path, whose chunk
    # size option is checked with the other options
    for bad in (3, 31, -1):
        rc = hc.lib().hcsp_spgemm_workspace(ctypes.byref(op), ctypes.byref(b),
                                            ctypes.byref(hc.opts(win_chunk_log2=bad)), ctypes.byref(n))
        assert rc == -1 and "win_chunk_log2" in hc.last_error()
    rc = hc.lib().hcsp_spgemm_workspace(ctypes.byref(op), ctypes.byref(b), ctypes.byref(hc.opts(win_chunk_log2=4)),
                                        ctypes.byref(n))
    assert rc == 0
    b.nrows = 49                                      # A.ncols != B.nrows
    rc = hc.lib().hcsp_spgemm_workspace(ctypes.byref(op), ctypes.byref(b), None, ctypes.byref(n))
    assert rc == -1 and "B.nrows" in hc.last_error()


def fake_item(kind, nrows, ncols, p):
    it = hc.c_batch_item()
    it.A.kind = kind
    if kind == hc.OP_CSR:
        it.A.csr = hc.c_csr(nrows, ncols, 10, 1, 1, 1)
    else:
        it.A.cl = hc.c_csr_cluster(nrows, ncols, (nrows + 1) // 2, 10, 20, 2, 0, 1, 1, 1, 1, 1, 1, 1)
    it.B = hc.c_csr(ncols, p, 10, 1, 1, 1)
    return it


def test_batch_plan_init_is_host_only():
    # sizes only: unit and row totals, flat row-offset length, widest B, workspace bytes
    items = (hc.c_batch_item * 3)(fake_item(0, 100, 50, 70), fake_item(0, 0, 5, 5), fake_item(0, 30, 40, 900))
    plan = hc.batch_plan_init(items)
    assert (plan.count, plan.units, plan.rows, plan.row_ptr_len, plan.max_ncols) == (3, 130, 130, 133, 900)
    assert plan.ws_bytes > 0 and plan.prepared == 0
    cl = (hc.c_batch_item * 2)(fake_item(1, 9, 50, 70), fake_item(1, 4, 5, 5))
    plan = hc.batch_plan_init(cl)
    assert plan.kind == hc.OP_CLUSTER and plan.units == 5 + 2 and plan.max_class == 1


def test_batch_plan_init_errors():
    mixed = (hc.c_batch_item * 2)(fake_item(0, 10, 5, 5), fake_item(1, 10, 5, 5))
    with pytest.raises(hc.HcspError) as e:
        hc.batch_plan_init(mixed)
    assert e.value.status == -1 and "same kind" in str(e.value)
    bad = (hc.c_batch_item * 2)(fake_item(0, 10, 5, 5), fake_item(0, 10, 6, 5))
    bad[1].B.nrows = 7                                # A.ncols != B.nrows in item 1
    with pytest.raises(hc.HcspError) as e:
        hc.batch_plan_init(bad)
    assert "item 1" in str(e.value)
    # an unprepared plan is refused before any device work
    plan = hc.batch_plan_init((hc.c_batch_item * 1)(fake_item(0, 10, 5, 5)))
    rc = hc.lib().hcsp_spgemm_batched(ctypes.byref(plan), None, None, None, None, 0, None)
    assert rc == -1 and "prepared" in hc.last_error()


def test_orderings_match_oracle():
    for name, A in inputs():
        if A.nrows == A.ncols:
            np.testing.assert_array_equal(hc.order_rcm(A), oracle.order_rcm(A), err_msg=name)
        np.testing.assert_array_equal(hc.order_degree(A), oracle.order_degree(A), err_msg=name)
    # square patterns that are not symmetric (A + A^T is built explicitly), and one that is
    # symmetric but for a single entry
    for seed in (5, 6):
        A = synth.uniform(400, 400, 5, seed)
        np.testing.assert_array_equal(hc.order_rcm(A), oracle.order_rcm(A), err_msg="uniform %d" % seed)
    S = synth.stencil(27, 5, 2)
    rp, col = S.rp.copy(), S.col.copy()
    keep = np.ones(len(col), bool)
    keep[rp[3] + 1] = False  # drop one off-diagonal entry of row 3 only
    lens = np.diff(rp) - np.add.reduceat(~keep, rp[:-1]).astype(np.int64)
    A = synth.HostCSR(np.concatenate([[0], np.cumsum(lens)]).astype(np.int64), col[keep], S.val[keep], S.nrows,
                      S.ncols)
    np.testing.assert_array_equal(hc.order_rcm(A), oracle.order_rcm(A), err_msg="stencil minus one entry")


def test_permute_h_is_the_symmetric_permutation():
    A = synth.uniform(60, 60, 7, 4)
    p = synth.perm(60, 8)
    B = hc.permute_h(A, p, p, nthreads=3)
    D, P = synth.to_dense(A)
    Db, Pb = synth.to_dense(B)
    np.testing.assert_array_equal(Pb, P[np.ix_(p, p)])
    np.testing.assert_array_equal(Db, D[np.ix_(p, p)])
    assert all(np.all(np.diff(B.col[B.rp[i]:B.rp[i + 1]]) > 0) for i in range(60))
    with pytest.raises(hc.HcspError):
        hc.permute_h(A, np.zeros(60, np.int32), None)        # not a permutation
