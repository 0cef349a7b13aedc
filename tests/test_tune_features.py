"""Host-side checks of the structure features and of the autotuner's table
(no GPU): closed values of the features on matrices whose structure is known,
and the table's choice rule."""
import numpy as np
import pytest

import paper_2507_21253_amd as hc
import synth
from paper_2507_21253_amd import tune


def test_features_closed_values_on_a_stencil():
    m = 12
    S = synth.stencil(27, m, 2)
    f = hc.features(S)
    n = m ** 3
    rl = np.diff(S.rp)
    assert f[0] == pytest.approx(np.log2(n + 1), rel=1e-6)
    assert f[1] == pytest.approx(np.log2((3 * m - 2) ** 3 + 1), rel=1e-6)
    assert f[2] == pytest.approx(rl.mean(), rel=1e-6)
    assert f[4] == pytest.approx(np.log2(28), rel=1e-6)
    # sum of products per row is sum_k |row k|^2 = (9m-10)^3
    assert f[10] == pytest.approx(np.log2((9 * m - 10) ** 3 + 1), rel=1e-6)
    assert f[23] == 0.0                                   # no empty rows
    assert sum(f[24:30]) == pytest.approx(1.0, abs=1e-6)  # work bins partition the rows
    assert f[30] == pytest.approx(np.log2(n + 1), rel=1e-6)


def test_features_uniform_rows_and_compression():
    U = synth.uniform(3000, 3000, 8, 5)
    f = hc.features(U)
    assert f[2] == 8.0 and f[3] == 0.0 and f[31] == 0.0   # every row has 8 entries
    assert 1.0 <= f[22] < 1.2                              # random columns barely collide
    E = synth.HostCSR(np.zeros(11, np.int64), np.zeros(0, np.int32), np.zeros(0), 10, 10)
    g = hc.features(E)
    assert g[23] == 1.0 and g[10] == 0.0


def test_features_similarity_of_neighbours():
    # natural-order 27-point rows: x-neighbours share 2/3 or 1/2 of their union; relabelling destroys it
    S = synth.stencil(27, 10, 2)
    M, _, _ = synth.workload_stencil27(10, 2, 3)
    fs, fm = hc.features(S), hc.features(M)
    assert fs[16] > 0.4 and fs[17] > 0.8
    assert fm[16] < 0.05 and fm[17] < 0.05
    # the best partner anywhere is found in both orders (a face neighbour, J >= 1/2)
    assert fs[21] >= 0.5 and fm[21] >= 0.5


NAN = float("nan")


def grid_run(plain=None, hc_times=None, nrows=10, nnz=10):
    """A run on the library's grid: plain {(sym, num): ms}, hc_times {(size, fill): ms}; the rest unmeasured."""
    r = hc.c_tune_run()
    r.nrows, r.nnz = nrows, nnz
    for i, sl in enumerate(hc.TUNE_SYM_FILLS):
        for j, nl in enumerate(hc.TUNE_NUM_FILLS):
            r.plain_ms[i][j] = (plain or {}).get((sl, nl), NAN)
    r.rcm_ms = NAN
    for i, mc in enumerate(hc.TUNE_CLUSTER_SIZES):
        for j, cl in enumerate(hc.TUNE_CL_FILLS):
            r.hc_ms[i][j] = (hc_times or {}).get((mc, cl), NAN)
    return r


def test_tune_table_choice_rule_and_roundtrip(tmp_path):
    t = hc.TuneTableNative()
    key = "rl2_cv0_cr2_sim2_loc0"
    t.add(key, grid_run({(70, 60): 2.0, (100, 60): 1.5}, {(2, 60): 1.3, (2, 70): 1.2, (4, 60): 1.8, (8, 60): 3.0}))
    e = t.get(key)
    assert (e["path"], e["max_cluster"], e["sym_load_pct"], e["load_pct"], e["tuned"]) == ("hc", 2, 100, 60, True)
    assert e["cl_load_pct"] == 70 and e["best_cluster_size"] == 2
    # a second matrix of the class where plain wins by far moves the choice; scores are sums of time / the
    # run's best: plain (100,60): 1.5/1.2 + 1.1/1.0 = 2.35 < hc2: 1.2/1.2 + 3.0/1.0 = 4.0
    t.add(key, grid_run({(70, 60): 1.0, (100, 60): 1.1}, {(2, 60): 3.0, (2, 70): 3.2, (4, 60): 4.0, (8, 60): 5.0}))
    e = t.get(key)
    assert e["path"] == "plain" and e["max_cluster"] == 0 and e["best_cluster_size"] == 2 and e["runs"] == 2
    # (70, 60): 2.0/1.2 + 1.0/1.0 = 2.67 against (100, 60): 2.35 -> the fills stay 100/60
    assert (e["sym_load_pct"], e["load_pct"]) == (100, 60)
    # fill of the clustered product: least summed relative time, 1.3/1.2 + 3.0/1.0 < 1.2/1.2 + 3.2/1.0
    assert e["cl_load_pct"] == 60
    # a candidate one run lacks is not a candidate: plain (50, 50) measured only by a third run
    t.add(key, grid_run({(50, 50): 0.1, (70, 60): 1.0, (100, 60): 1.0}, {(2, 60): 2.0}))
    assert (t.get(key)["sym_load_pct"], t.get(key)["load_pct"]) == (100, 60)

    p = tmp_path / "t.txt"
    t.save(str(p))
    u = hc.TuneTableNative.load(str(p))
    assert u.classes() == [key] and u.get(key) == t.get(key)
    for a, b in zip(u.runs(key), t.runs(key)):
        assert bytes(a) == bytes(b)                        # every double round-trips (NaN included)
    f = np.zeros(32, np.float32)
    assert u.lookup(f)["tuned"] is False                  # unknown class: library defaults
    assert (u.lookup(f)["sym_load_pct"], u.lookup(f)["load_pct"], u.lookup(f)["path"]) == (70, 60, "plain")
    with pytest.raises(hc.HcspError):
        t.add("bad key", grid_run({(70, 60): 1.0}))
    with pytest.raises(hc.HcspError):
        t.add(key, grid_run())                             # nothing measured


def test_matrix_class_buckets():
    f = np.zeros(32, np.float32)
    f[2], f[12], f[22], f[21], f[14] = 27.0, 0.2, 5.0, 0.5, 0.3
    assert tune.matrix_class(f) == "rl2_cv0_cr2_sim1_loc1"
    f[14] = 0.001                                          # columns near the diagonal
    assert tune.matrix_class(f) == "rl2_cv0_cr2_sim1_loc0"
    # edges belong to the bucket above them
    f[2], f[12], f[22], f[21], f[14] = 40.0, 2.0, 3.0, 0.6, 0.05
    assert tune.matrix_class(f) == "rl3_cv2_cr2_sim2_loc1"


def test_matrix_class_of_real_features():
    # the library's key equals the rule restated here (count of edges at or below the feature) on the
    # features of matrices of each family
    def restated(f):
        b = lambda x, edges: sum(e <= float(x) for e in edges)
        return "rl%d_cv%d_cr%d_sim%d_loc%d" % (b(f[2], (6, 16, 40)), b(f[12], (0.5, 2.0)), b(f[22], (1.3, 3.0)),
                                               b(f[21], (0.3, 0.6)), b(f[14], (0.05,)))
    mats = [synth.stencil(27, 10, 2), synth.workload_stencil27(10, 2, 3)[0], synth.uniform(2000, 2000, 8, 3),
            synth.stencil(5, 40, 4), synth.rmat(10, 16, 0.57, 0.19, 0.19, 5)]
    keys = set()
    for M in mats:
        f = hc.features(M)
        assert tune.matrix_class(f) == restated(f)
        keys.add(restated(f))
    assert len(keys) >= 3


def test_shipped_table_loads():
    t = tune.TuneTable.load()
    assert len(t.classes()) >= 5
    e = t.entry("rl2_cv0_cr2_sim1_loc1")                  # the relabelled 27-point stencils
    assert e["tuned"] and e["path"] == "hc" and e["max_cluster"] == 4


def test_mlp_model_file_roundtrip(tmp_path):
    rng = np.random.default_rng(3)
    params = rng.normal(size=hc.MLP_NPARAMS).astype(np.float32)
    norm = rng.uniform(0.5, 2, 2 * hc.NFEATURES).astype(np.float32)
    m = hc.MlpModel(params, norm, "paths plain,rcm")
    p = str(tmp_path / "m.mlp")
    m.save(p)
    q = hc.MlpModel.load(p)
    P, N, tag = q.get()
    assert tag == "paths plain,rcm"
    np.testing.assert_array_equal(P, params)               # float32 round-trips exactly
    np.testing.assert_array_equal(N, norm)
    z = hc.MlpModel()                                      # zeros, mu 0, sd 1
    P0, N0, t0 = z.get()
    assert not P0.any() and not N0[:32].any() and (N0[32:] == 1).all() and t0 == ""
    z.set(norm=norm)
    assert (z.get()[1] == norm).all()
    open(str(tmp_path / "bad.mlp"), "w").write("hcsp-mlp 1 32 64 4\n\n")
    with pytest.raises(hc.HcspError):
        hc.MlpModel.load(str(tmp_path / "bad.mlp"))
