"""Pins for the CPU oracle: each test ties it to something other than itself —
brute force, closed forms, special cases, the paper's worked examples and
invariants — so that a dropped term, a wrong index or a transposed operand
in the oracle fails at least one of them."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_pattern_matrix(rng, n, m, density, zero_frac=0.1):
    pat = rng.random((n, m)) < density
    vals = rng.uniform(-1, 1, (n, m))
    vals[rng.random((n, m)) < zero_frac] = 0.0          # stored explicit zeros
    vals[~pat] = 0.0
    return vals, pat


def assert_csr_equal(C1, C2, bitwise=True):
    assert C1.nrows == C2.nrows and C1.ncols == C2.ncols
    np.testing.assert_array_equal(C1.rp, C2.rp)
    np.testing.assert_array_equal(C1.col, C2.col)
    if bitwise:
        # +0.0 and -0.0 compare equal; everything else must match to the bit
        np.testing.assert_array_equal(C1.val, C2.val)
    else:
        np.testing.assert_allclose(C1.val, C2.val, rtol=1e-12, atol=0)


# ------------------------------------------------------------- product pins

@pytest.mark.parametrize("seed", range(12))
def test_gustavson_equals_bruteforce_dense(seed):
    rng = np.random.default_rng(seed)
    n, m, p = rng.integers(1, 64, 3)
    density = rng.choice([0.02, 0.1, 0.3, 0.8])
    A, Ap = rand_pattern_matrix(rng, n, m, density)
    B, Bp = rand_pattern_matrix(rng, m, p, density)
    Ad = synth.from_dense(A, Ap)
    Bd = synth.from_dense(B, Bp)
    C = oracle.spgemm(Ad, Bd)
    Cd, Cp = oracle.dense_product(A, Ap, B, Bp)
    # structure: exactly the boolean product (numpy boolean matmul, independent)
    boolprod = (Ap.astype(np.int64) @ Bp.astype(np.int64)) > 0
    np.testing.assert_array_equal(Cp, boolprod)
    ref = synth.from_dense(Cd, Cp)
    assert_csr_equal(C, ref, bitwise=True)
    # values: independent library product within rounding
    np.testing.assert_allclose(synth.to_dense(C)[0], A @ B, rtol=0, atol=1e-12 * max(1.0, np.abs(A).sum()))


def test_numeric_zero_is_kept():
    # c_00 = 1*1 + (-1)*1 = 0 exactly, but the entry is structurally present
    A = synth.from_dense(np.array([[1.0, -1.0]]), np.array([[True, True]]))
    B = synth.from_dense(np.array([[1.0], [1.0]]), np.array([[True], [True]]))
    C = oracle.spgemm(A, B)
    assert C.nnz == 1 and C.col[0] == 0 and C.val[0] == 0.0


def test_empty_and_degenerate():
    Z = synth.HostCSR(np.zeros(5, np.int64), np.zeros(0, np.int32), np.zeros(0), 4, 3)
    B = synth.uniform(3, 6, 2, 9)
    C = oracle.spgemm(Z, B)
    assert C.nnz == 0 and C.nrows == 4 and C.ncols == 6
    C0 = oracle.spgemm(synth.HostCSR(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0), 0, 3), B)
    assert C0.nnz == 0 and len(C0.rp) == 1


def grid_coords(kind, m, n):
    idx = np.arange(n)
    if kind == 5:
        return np.stack([idx % m, idx // m], 1)
    return np.stack([idx % m, (idx // m) % m, idx // (m * m)], 1)


@pytest.mark.parametrize("kind,m", [(27, 3), (27, 4), (27, 5), (27, 6), (27, 7), (5, 4), (5, 10), (7, 4), (7, 6)])
def test_stencil_square_closed_forms(kind, m):
    S = synth.stencil(kind, m, 5)
    C = oracle.spgemm(S, S)
    n = S.nrows
    xyz = grid_coords(kind, m, n)
    # structure of S^2: grid points within distance 2 (Chebyshev for 27-point, Manhattan for 5/7-point)
    d = np.abs(xyz[:, None, :] - xyz[None, :, :])
    dist = d.max(-1) if kind == 27 else d.sum(-1)
    expect = dist <= 2
    got = np.zeros((n, n), bool)
    got[np.repeat(np.arange(n), np.diff(C.rp)), C.col] = True
    np.testing.assert_array_equal(got, expect)
    rowlen = np.diff(S.rp)
    products = int(rowlen[S.col].sum())
    if kind == 27:
        assert S.nnz == (3 * m - 2) ** 3
        assert C.nnz == (5 * m - 6) ** 3
        assert products == (9 * m - 10) ** 3


def test_identity_and_permutation_special_cases():
    A = synth.uniform(40, 30, 7, 11)
    I30 = synth.identity(30)
    I40 = synth.identity(40)
    assert_csr_equal(oracle.spgemm(A, I30), A)          # fma(a, 1, +0) == a
    assert_csr_equal(oracle.spgemm(I40, A), A)
    p = synth.perm(40, 12)
    P = synth.relabel(I40, p, None)                     # row p[u] of P is e_u
    PA = oracle.spgemm(P, A)
    assert_csr_equal(PA, synth.relabel(A, p, None))


def test_diagonal_scaling_is_exact():
    A = synth.uniform(25, 25, 6, 13)
    d = np.random.default_rng(3).uniform(-2, 2, 25)
    D = synth.HostCSR(np.arange(26, dtype=np.int64), np.arange(25, dtype=np.int32), d, 25, 25)
    C = oracle.spgemm(D, A)
    rows = np.repeat(np.arange(25), np.diff(A.rp))
    np.testing.assert_array_equal(C.col, A.col)
    np.testing.assert_array_equal(C.val, d[rows] * A.val)   # one correctly rounded product


def test_row_permutation_invariant_bitwise():
    A = synth.uniform(300, 200, 9, 21)
    B = synth.uniform(200, 250, 5, 22)
    p = synth.perm(300, 23)
    C = oracle.spgemm(A, B)
    CP = oracle.spgemm(synth.relabel(A, p, None), B)
    assert_csr_equal(CP, synth.relabel(C, p, None))


def test_symmetric_relabel_structure():
    S = synth.stencil(27, 6, 3)
    M, q = synth.symmetric_relabel(S, 4)
    CS = oracle.spgemm(S, S)
    CM = oracle.spgemm(M, M)
    relab = synth.relabel(CS, q, q)
    np.testing.assert_array_equal(CM.rp, relab.rp)
    np.testing.assert_array_equal(CM.col, relab.col)
    # values differ only by summation order: bound by n_terms * eps * sum|a*b|
    absS = synth.HostCSR(S.rp, S.col, np.abs(S.val), S.nrows, S.ncols)
    mag = synth.relabel(oracle.spgemm(absS, absS), q, q).val
    assert np.all(np.abs(CM.val - relab.val) <= 27 * 2.3e-16 * mag)


def test_multithreaded_equals_single():
    A = synth.uniform(500, 500, 12, 31)
    C1 = oracle.spgemm(A, A)
    C2 = oracle.spgemm_mt(A, A, 4)
    assert_csr_equal(C1, C2)


@pytest.mark.parametrize("seed", range(6))
def test_structure_count_equals_boolean_product(seed):
    # row counts of the boolean product, from an independent numpy boolean matmul; rectangular, empty rows
    rng = np.random.default_rng(500 + seed)
    n, m, p = (int(x) for x in rng.integers(1, 90, 3))
    Ap = rng.random((n, m)) < rng.choice([0.0, 0.05, 0.3], size=n)[:, None]
    Bp = rng.random((m, p)) < rng.choice([0.0, 0.1, 0.6], size=m)[:, None]
    A = synth.from_dense(np.where(Ap, 1.0, 0.0), Ap)
    B = synth.from_dense(np.where(Bp, 1.0, 0.0), Bp)
    want = ((Ap.astype(np.int64) @ Bp.astype(np.int64)) > 0).sum(axis=1)
    for nth in (1, 3):
        np.testing.assert_array_equal(oracle.spgemm_count(A, B, nth), want)
    if n > 2:
        np.testing.assert_array_equal(oracle.spgemm_count(A, B, 2, (1, n - 1)), want[1:n - 1])


@pytest.mark.parametrize("kind,m", [(27, 7), (7, 9), (5, 12)])
def test_structure_count_stencil_closed_forms(kind, m):
    S = synth.stencil(kind, m, 3)
    total = int(oracle.spgemm_count(S, S, 4).sum())
    closed = {27: (5 * m - 6) ** 3}
    if kind in closed:
        assert total == closed[kind]
    np.testing.assert_array_equal(oracle.spgemm_count(S, S, 2), np.diff(oracle.spgemm(S, S).rp))


def test_structure_count_power_law_equals_gustavson():
    R = synth.rmat(11, 16, 0.57, 0.19, 0.19, 3)
    np.testing.assert_array_equal(oracle.spgemm_count(R, R, 5), np.diff(oracle.spgemm(R, R).rp))


def test_rowstats_matches_full():
    A = synth.uniform(200, 200, 8, 41)
    C = oracle.spgemm(A, A)
    nnz, h, s = oracle.rowstats(A, A, (0, 200), 3)
    np.testing.assert_array_equal(nnz, np.diff(C.rp))
    for r in (0, 17, 199):
        b, e = C.rp[r], C.rp[r + 1]
        assert h[r] == oracle.hash_cols(C.col[b:e])
        acc = 0.0
        for v in C.val[b:e]:
            acc += v
        assert s[r] == acc


# ------------------------------------------------------------- Jaccard pins

def py_jaccard(A, i, j):
    a, b = set(A.row(i)[0].tolist()), set(B_row(A, j))
    un = len(a | b)
    return Fraction(len(a & b), un) if un else Fraction(0)


def B_row(A, j):
    return A.row(j)[0].tolist()


def test_jaccard_27pt_neighbour_values():
    m = 7
    S = synth.stencil(27, m, 1)

    def idx(x, y, z):
        return x + m * (y + m * z)

    c = idx(3, 3, 3)
    expect = {
        idx(4, 3, 3): Fraction(1, 2),    # face
        idx(4, 4, 3): Fraction(2, 7),    # edge diagonal
        idx(4, 4, 4): Fraction(4, 23),   # corner
        idx(5, 3, 3): Fraction(1, 5),    # two apart on one axis
    }
    for j, f in expect.items():
        ov, un = oracle.jaccard(S, c, j)
        assert Fraction(ov, un) == f == py_jaccard(S, c, j)
    # x boundary: (0,y,z) against (1,y,z) and (2,y,z)
    ov, un = oracle.jaccard(S, idx(0, 3, 3), idx(1, 3, 3))
    assert Fraction(ov, un) == Fraction(2, 3)
    ov, un = oracle.jaccard(S, idx(0, 3, 3), idx(2, 3, 3))
    assert Fraction(ov, un) == Fraction(1, 4)


def test_jaccard_random_vs_sets():
    A = synth.uniform(60, 40, 8, 5)
    rng = np.random.default_rng(0)
    for _ in range(200):
        i, j = rng.integers(0, 60, 2)
        ov, un = oracle.jaccard(A, int(i), int(j))
        assert Fraction(ov, un) == py_jaccard(A, int(i), int(j))


# ------------------------------------------------------------- plan pins

def csr_from_rows(rows, ncols):
    rp = np.zeros(len(rows) + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([c for r in rows for c in sorted(r)], np.int32)
    return synth.HostCSR(rp, col, np.ones(len(col)), len(rows), ncols)


def test_variable_plan_paper_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "variable_worked_example.json")))
    A = csr_from_rows(g["rows"], g["ncols"])
    for s in g["printed_similarities"]:
        ov, un = oracle.jaccard(A, *s["pair"])
        assert Fraction(ov, un) == Fraction(*s["value"])
    plan = oracle.plan_variable(A, tuple(g["jacc_th"]), g["max_cluster"])
    assert plan.clusters() == g["expected_clusters"]


def test_variable_plan_special_cases():
    A = synth.uniform(50, 40, 6, 7)
    # threshold 0: every row qualifies, so clusters are fixed blocks of max_cluster rows
    for K in (1, 3, 8):
        pv = oracle.plan_variable(A, (0, 1), K)
        pf = oracle.plan_fixed(50, K)
        np.testing.assert_array_equal(pv.perm, pf.perm)
        np.testing.assert_array_equal(pv.cl_row_ptr, pf.cl_row_ptr)
    # threshold above 1: only singletons
    pv = oracle.plan_variable(A, (11, 10), 8)
    assert pv.nclusters == 50
    # threshold exactly met joins (the listing breaks only on strictly smaller similarity)
    B = csr_from_rows([[0, 1], [0]], 2)                 # J = 1/2
    assert oracle.plan_variable(B, (1, 2), 8).clusters() == [[0, 1]]
    assert oracle.plan_variable(B, (51, 100), 8).clusters() == [[0], [1]]


@pytest.mark.parametrize("m", [4, 6, 10])
def test_variable_plan_natural_stencil_gives_x_pairs(m):
    S = synth.stencil(27, m, 2)
    plan = oracle.plan_variable(S, (3, 10), 8)
    assert plan.clusters() == [[2 * i, 2 * i + 1] for i in range(m ** 3 // 2)]
    Ac = oracle.cluster_build(S, plan)
    assert len(Ac.cl_col) == (2 * m - 2) * (3 * m - 2) ** 2
    assert len(Ac.cl_val) == 2 * len(Ac.cl_col)


def test_fixed_plan_and_perm_in():
    pf = oracle.plan_fixed(10, 4)
    assert pf.clusters() == [[0, 1, 2, 3], [4, 5, 6, 7], [8, 9]]
    pi = synth.perm(10, 1)
    pf = oracle.plan_fixed(10, 4, pi)
    np.testing.assert_array_equal(pf.perm, pi)
    assert oracle.plan_fixed(0, 4).nclusters == 0


def brute_topk(A, t, topk):
    n = A.nrows
    res = []
    for i in range(n):
        cands = []
        for j in range(n):
            if j == i:
                continue
            ov = len(set(A.row(i)[0].tolist()) & set(A.row(j)[0].tolist()))
            if ov == 0:
                continue
            J = py_jaccard(A, i, j)
            if J > t:
                cands.append((-J, j))
        cands.sort()
        res.append([j for _, j in cands[:topk]])
    return res


@pytest.mark.parametrize("seed,topk,d,t", [(1, 7, None, (3, 10)), (2, 3, None, (3, 10)), (3, 1, None, (3, 10)),
                                          (4, 15, None, (3, 10)), (5, 7, 4, (1, 3)), (6, 3, 6, (1, 2))])
def test_topk_candidates_bruteforce(seed, topk, d, t):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(20, 120))
    A = synth.uniform(n, 12 if d else 30, d or int(rng.integers(2, 9)), seed)
    cnt, nbr, ov, un = oracle.topk_candidates(A, t, topk)
    ref = brute_topk(A, Fraction(*t), topk)
    for i in range(n):
        assert nbr[i, :cnt[i]].tolist() == ref[i]


def test_hierarchical_hand_examples():
    g = json.load(open(os.path.join(GOLDEN, "hierarchical_hand_examples.json")))
    for ex in g["examples"]:
        A = csr_from_rows(ex["rows"], ex["ncols"])
        for case in ex["cases"]:
            for flags, key in ((oracle.SIM_ROOT, "expected_clusters_root"), (oracle.SIM_UNION, "expected_clusters_union")):
                plan = oracle.plan_hierarchical(A, tuple(case["jacc_th"]), case["max_cluster"], flags)
                assert plan.clusters() == case.get(key, case.get("expected_clusters")), case["trace"]


def test_hierarchical_similarity_readings_differ_on_hand_example():
    # the hand-worked example whose lifted pair passes the threshold only when the members' unions are
    # scored: the two readings of the merged-cluster similarity must give different plans
    g = json.load(open(os.path.join(GOLDEN, "hierarchical_hand_examples.json")))
    seen = 0
    for ex in g["examples"]:
        A = csr_from_rows(ex["rows"], ex["ncols"])
        for case in ex["cases"]:
            if "expected_clusters_union" in case and case["expected_clusters_union"] != case["expected_clusters_root"]:
                r = oracle.plan_hierarchical(A, tuple(case["jacc_th"]), case["max_cluster"], oracle.SIM_ROOT)
                u = oracle.plan_hierarchical(A, tuple(case["jacc_th"]), case["max_cluster"], oracle.SIM_UNION)
                assert r.clusters() != u.clusters()
                seen += 1
    assert seen >= 1


@pytest.mark.parametrize("seed", range(4))
def test_hierarchical_recovers_duplicate_groups(seed):
    rng = np.random.default_rng(seed)
    g, maxc = 40, 8
    base = synth.uniform(g, 5000, 20, 100 + seed)
    sizes = rng.integers(1, maxc + 1, g)
    rows = []
    grp = []
    for r in range(g):
        for _ in range(sizes[r]):
            rows.append(base.row(r)[0].tolist())
            grp.append(r)
    n = len(rows)
    shuffle = synth.perm(n, 200 + seed)
    srows = [None] * n
    sgrp = [None] * n
    for u in range(n):
        srows[shuffle[u]] = rows[u]
        sgrp[shuffle[u]] = grp[u]
    A = csr_from_rows(srows, 5000)
    for flags in (oracle.SIM_ROOT, oracle.SIM_UNION):
        plan = oracle.plan_hierarchical(A, (3, 10), maxc, flags)
        got = sorted(sorted(c) for c in plan.clusters())
        want = sorted(sorted(i for i in range(n) if sgrp[i] == r) for r in range(g))
        assert got == want


@pytest.mark.parametrize("maxc", [2, 4, 8, 16])
def test_hierarchical_invariants(maxc):
    M, S, q = synth.workload_stencil27(8, 2, 3)
    p1 = oracle.plan_hierarchical(M, (3, 10), maxc)
    p2 = oracle.plan_hierarchical(M, (3, 10), maxc)
    np.testing.assert_array_equal(p1.perm, p2.perm)                    # deterministic
    np.testing.assert_array_equal(p1.cl_row_ptr, p2.cl_row_ptr)
    assert sorted(p1.perm.tolist()) == list(range(M.nrows))            # a partition
    sizes = np.diff(p1.cl_row_ptr)
    assert sizes.min() >= 1 and sizes.max() <= maxc
    # threshold 1: no pair is strictly above it, so every row is alone
    p3 = oracle.plan_hierarchical(M, (1, 1), maxc)
    assert p3.nclusters == M.nrows
    # identity perm_in is the same as none
    p4 = oracle.plan_hierarchical(M, (3, 10), maxc, perm_in=np.arange(M.nrows, dtype=np.int32))
    np.testing.assert_array_equal(p1.perm, p4.perm)


def test_hierarchical_stencil_clusters_are_face_connected():
    # on the 27-point stencil only face neighbours exceed 0.3, so every merge joins face neighbours
    m = 8
    M, S, q = synth.workload_stencil27(m, 2, 3)
    qinv = np.empty_like(q)
    qinv[q] = np.arange(len(q))
    plan = oracle.plan_hierarchical(M, (3, 10), 8)
    xyz = grid_coords(27, m, m ** 3)
    for c in plan.clusters():
        pts = [xyz[qinv[r]] for r in c]
        # connected under face adjacency
        seen = {0}
        stack = [0]
        while stack:
            a = stack.pop()
            for b in range(len(pts)):
                if b not in seen and np.abs(pts[a] - pts[b]).sum() == 1:
                    seen.add(b)
                    stack.append(b)
        assert len(seen) == len(pts)
    assert plan.nclusters < M.nrows / 3


# ------------------------------------------------------------- CSR_Cluster pins

def cluster_to_csr(Ac):
    rows = {}
    for c in range(Ac.nclusters):
        b, e = Ac.cl_row_ptr[c], Ac.cl_row_ptr[c + 1]
        s = e - b
        cb, ce = Ac.cl_col_ptr[c], Ac.cl_col_ptr[c + 1]
        for l in range(s):
            r = int(Ac.perm[b + l])
            cols, vals = [], []
            for t in range(cb, ce):
                if (int(Ac.cl_mask[t]) >> l) & 1:
                    cols.append(int(Ac.cl_col[t]))
                    vals.append(Ac.cl_val[Ac.cl_val_ptr[c] + (t - cb) * s + l])
                else:
                    v = Ac.cl_val[Ac.cl_val_ptr[c] + (t - cb) * s + l]
                    assert v == 0.0 and not np.signbit(v)              # placeholder +0.0
            rows[r] = (cols, vals)
    rp = np.zeros(Ac.nrows + 1, np.int64)
    for r in range(Ac.nrows):
        rp[r + 1] = rp[r] + len(rows[r][0])
    col = np.array([c for r in range(Ac.nrows) for c in rows[r][0]], np.int32)
    val = np.array([v for r in range(Ac.nrows) for v in rows[r][1]])
    return synth.HostCSR(rp, col, val, Ac.nrows, Ac.ncols)


@pytest.mark.parametrize("planner", ["fixed", "variable", "hier", "hier_perm"])
def test_cluster_roundtrip(planner):
    A = synth.uniform(90, 70, 6, 8)
    if planner == "fixed":
        plan = oracle.plan_fixed(A.nrows, 5)
    elif planner == "variable":
        plan = oracle.plan_variable(A, (1, 10), 8)
    elif planner == "hier":
        plan = oracle.plan_hierarchical(A, (1, 10), 8)
    else:
        plan = oracle.plan_hierarchical(A, (1, 10), 16, perm_in=synth.perm(90, 3))
    Ac = oracle.cluster_build(A, plan)
    R = cluster_to_csr(Ac)
    np.testing.assert_array_equal(R.rp, A.rp)
    np.testing.assert_array_equal(R.col, A.col)
    np.testing.assert_array_equal(R.val, A.val)
    popcnt = sum(bin(int(x)).count("1") for x in Ac.cl_mask)
    assert popcnt == A.nnz
    for c in range(Ac.nclusters):                                     # union columns sorted
        seg = Ac.cl_col[Ac.cl_col_ptr[c]:Ac.cl_col_ptr[c + 1]]
        assert np.all(np.diff(seg) > 0)


def test_fixed8_natural_stencil_union_size_bruteforce():
    m = 10
    S = synth.stencil(27, m, 2)
    plan = oracle.plan_fixed(S.nrows, 8)
    Ac = oracle.cluster_build(S, plan)
    ncc = 0
    for c in plan.clusters():
        u = set()
        for r in c:
            u |= set(S.row(r)[0].tolist())
        ncc += len(u)
    assert len(Ac.cl_col) == ncc


# ------------------------------------------------------------- Alg. 1 pins

@pytest.mark.parametrize("planner", ["fixed4", "fixed16", "variable", "hier_root", "hier_union", "hier_perm"])
def test_clusterwise_equals_rowwise_bitwise(planner):
    M, S, q = synth.workload_stencil27(7, 2, 3)
    A = M
    if planner == "fixed4":
        plan = oracle.plan_fixed(A.nrows, 4)
    elif planner == "fixed16":
        plan = oracle.plan_fixed(A.nrows, 16, synth.perm(A.nrows, 9))
    elif planner == "variable":
        plan = oracle.plan_variable(A, (3, 10), 8)
    elif planner == "hier_root":
        plan = oracle.plan_hierarchical(A, (3, 10), 8, oracle.SIM_ROOT)
    elif planner == "hier_union":
        plan = oracle.plan_hierarchical(A, (3, 10), 8, oracle.SIM_UNION)
    else:
        plan = oracle.plan_hierarchical(A, (2, 10), 12, oracle.SIM_ROOT, perm_in=synth.perm(A.nrows, 5))
    Ac = oracle.cluster_build(A, plan)
    C = oracle.spgemm(A, A)
    Cc = oracle.cluster_spgemm(Ac, A)
    assert_csr_equal(C, Cc, bitwise=True)


def test_clusterwise_uniform_random_bitwise():
    A = synth.uniform(400, 300, 10, 3)
    B = synth.uniform(300, 500, 7, 4)
    plan = oracle.plan_hierarchical(A, (1, 20), 16)
    Cc = oracle.cluster_spgemm(oracle.cluster_build(A, plan), B)
    assert_csr_equal(oracle.spgemm(A, B), Cc, bitwise=True)


# ------------------------------------------------------------ row orderings

def _graph(n, edges):
    D = np.zeros((n, n))
    P = np.zeros((n, n), bool)
    for a, b in edges:
        P[a, b] = P[b, a] = True
        D[a, b] = D[b, a] = 1.0
    return synth.from_dense(D, P)


def _bandwidth(H, perm):
    inv = np.empty(H.nrows, np.int64)
    inv[perm] = np.arange(H.nrows)
    r = np.repeat(np.arange(H.nrows), np.diff(H.rp))
    return int(np.max(np.abs(inv[r] - inv[H.col]))) if len(H.col) else 0


def test_rcm_hand_example():
    g = json.load(open(os.path.join(GOLDEN, "rcm_hand_example.json")))
    H = _graph(6, g["edges"])
    assert oracle.order_rcm(H).tolist() == g["perm"]


def test_rcm_hand_example_pseudo_peripheral_start_and_degree_order():
    # the least-degree vertex is a leaf in the middle: the start moves to an end of the longest path, and
    # the hub's neighbours are visited by (degree, id), not by id
    g = json.load(open(os.path.join(GOLDEN, "rcm_hand_example_2.json")))
    H = _graph(g["n"], g["edges"])
    assert oracle.order_rcm(H).tolist() == g["perm"]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_rcm_recovers_a_shuffled_path(seed):
    # a path 0-1-...-(n-1) under a random labelling: RCM lays it out again, bandwidth 1
    n = 200
    q = synth.perm(n, seed)
    H = _graph(n, [(int(q[i]), int(q[i + 1])) for i in range(n - 1)])
    p = oracle.order_rcm(H)
    assert sorted(p.tolist()) == list(range(n))
    assert _bandwidth(H, p) == 1


@pytest.mark.parametrize("m", [5, 8, 13])
def test_rcm_grid_bandwidth(m):
    # 5-point grid: breadth-first levels from a corner are anti-diagonals, bandwidth m;
    # relabelled, the bandwidth stays within 2m (the labels only break ties)
    S = synth.stencil(5, m, 1)
    assert _bandwidth(S, oracle.order_rcm(S)) == m
    Q = synth.perm(m * m, 5)
    R = synth.relabel(S, Q, Q)
    assert _bandwidth(R, oracle.order_rcm(R)) <= 2 * m


def test_rcm_components_are_contiguous_and_isolated_vertices_kept():
    # two shuffled paths and isolated vertices: each component occupies one contiguous block
    edges = [(0, 5), (5, 2), (2, 7), (1, 4), (4, 9)]
    H = _graph(11, edges)
    p = oracle.order_rcm(H).tolist()
    assert sorted(p) == list(range(11))
    pos = {v: i for i, v in enumerate(p)}
    for comp in ([0, 5, 2, 7], [1, 4, 9]):
        ix = sorted(pos[v] for v in comp)
        assert ix == list(range(ix[0], ix[0] + len(comp)))
    assert _bandwidth(H, p) == 1


def test_degree_order():
    A = synth.from_dense(np.array([[1, 0, 0, 0], [1, 1, 1, 0], [0, 1, 1, 0], [1, 1, 1, 1.0]]))
    assert oracle.order_degree(A).tolist() == [3, 1, 2, 0]
    R = synth.rmat(9, 8, 0.57, 0.19, 0.19, 2)
    p = oracle.order_degree(R)
    ln = np.diff(R.rp)[p]
    assert np.all(ln[:-1] >= ln[1:]) and sorted(p.tolist()) == list(range(R.nrows))
    # equal lengths keep ascending ids
    for L in np.unique(ln):
        ids = p[ln == L]
        assert np.all(np.diff(ids) > 0)
