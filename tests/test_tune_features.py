"""Host-side checks of the structure features and of the autotuner's table
(no GPU): closed values of the features on matrices whose structure is known,
and the table's choice rule."""
import json

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


def run(cls, times, best, path="plain", mc=0):
    return {"class": cls, "path": path, "max_cluster": mc, "best_cluster_size": 2, "sym_load_pct": 70,
            "load_pct": 60, "cl_load_pct": 70, "ms": best, "times_ms": times, "nrows": 10, "nnz": 10}


def test_tune_table_choice_rule_and_roundtrip(tmp_path):
    t = tune.TuneTable()
    times = {"plain_s70_n60": 2.0, "plain_s100_n60": 1.5, "hc2": 1.2, "hc4": 1.8, "hc8": 3.0,
             "hc2_n60": 1.3, "hc2_n70": 1.2}
    t.add(run("rl2_cv0_cr2_sim2", times, 1.2, "hc", 2))
    e = t.entries["rl2_cv0_cr2_sim2"]
    assert (e["path"], e["max_cluster"], e["sym_load_pct"], e["load_pct"]) == ("hc", 2, 100, 60)
    assert e["cl_load_pct"] == 70
    # a second matrix of the class where plain wins by far moves the choice
    t.add(run("rl2_cv0_cr2_sim2", {"plain_s70_n60": 1.0, "plain_s100_n60": 1.1, "hc2": 3.0, "hc4": 4.0,
                                   "hc8": 5.0, "hc2_n60": 3.0, "hc2_n70": 3.2}, 1.0))
    e = t.entries["rl2_cv0_cr2_sim2"]
    assert e["path"] == "plain" and e["best_cluster_size"] == 2
    # fill of the clustered product: least summed relative time, 1.3/1.2 + 3.0/1.0 < 1.2/1.2 + 3.2/1.0
    assert e["cl_load_pct"] == 60

    p = tmp_path / "t.json"
    t.save(str(p))
    u = tune.TuneTable.load(str(p))
    assert u.entries == json.loads(json.dumps(t.entries))
    f = np.zeros(32, np.float32)
    assert u.lookup(f)["tuned"] is False                  # unknown class: library defaults


def test_matrix_class_buckets():
    f = np.zeros(32, np.float32)
    f[2], f[12], f[22], f[21], f[14] = 27.0, 0.2, 5.0, 0.5, 0.3
    assert tune.matrix_class(f) == "rl2_cv0_cr2_sim1_loc1"
    f[14] = 0.001                                          # columns near the diagonal
    assert tune.matrix_class(f) == "rl2_cv0_cr2_sim1_loc0"
