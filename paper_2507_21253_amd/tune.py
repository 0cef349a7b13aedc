"""Autotuner: bin thresholds and cluster size per matrix class.

The paper fixes the clustering parameters (threshold 0.3, at most 8 rows per
cluster, Sec. "Hierarchical Clusters") and notes that the best cluster length
depends on the matrix (Sec. "Clustering Without Changing Order"); which
layout wins also depends on the sparsity pattern (Sec. "Evaluation").  Here
those choices are measured instead of fixed: for a matrix, every candidate is
timed with the library's own product on the GPU, and the winner is stored
per *matrix class* (a coarse bucket of the library's structure features) in
a JSON table that later products look up.

Tuned per class:
  * ``sym_load_pct`` -- symbolic hash-table fill bound (bin thresholds of the
    symbolic phase: which table size a unit's product count selects),
  * ``load_pct`` -- numeric table fill target (bin thresholds of the numeric
    phase),
  * ``path`` and ``max_cluster`` -- plain CSR, or CSR_Cluster from
    hierarchical clustering (Alg. 3, threshold 3/10) of the rows taken in
    reverse Cuthill-McKee order (the paper's reorder-then-cluster flow), with
    at most 2, 4 or 8 rows per cluster;
  * ``cl_load_pct`` -- the numeric fill target for the clustered product
    (a cluster's table carries a value column per member, so a different
    fill can pay).

The decision is steady-state product time (symbolic + nnz read-back +
numeric), the regime of repeated products over one structure that the
paper's clustering targets; preprocessing time is recorded beside it.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import (DeviceCSR, Product, SIM_ROOT, cluster_build, features, opts, order_rcm, permute_h,
               plan_hierarchical)

SYM_LOADS = (50, 70, 100)
NUM_LOADS = (50, 60, 70)
CL_LOADS = (50, 60, 70, 75, 80, 85)
MAX_CLUSTERS = (2, 4, 8)
DEFAULT = {"path": "plain", "max_cluster": 0, "sym_load_pct": 70, "load_pct": 60}
TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json")


def _bucket(x: float, edges) -> int:
    return int(np.searchsorted(np.asarray(edges, float), float(x), side="right"))


def matrix_class(f: np.ndarray) -> str:
    """Class key from the structure features: mean row length, spread of the per-row work, compression of
    products into output entries, the best similarity a row finds (what clustering can exploit), and
    whether columns lie near the diagonal (mean |col - row| / ncols: a row's output columns then come in
    runs, which changes the best hash-table fill)."""
    return "rl%d_cv%d_cr%d_sim%d_loc%d" % (_bucket(f[2], (6, 16, 40)), _bucket(f[12], (0.5, 2.0)),
                                           _bucket(f[22], (1.3, 3.0)), _bucket(f[21], (0.3, 0.6)),
                                           _bucket(f[14], (0.05,)))


def _time_ms(P: Product, reps: int) -> float:
    import torch
    P.run()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        P.run(check=False)
    e1.record(s)
    torch.cuda.synchronize()
    P.check()
    return e0.elapsed_time(e1) / reps


def tune_matrix(H, reps: int = 3, threads: int = 0) -> dict:
    """Times the candidates on the GPU for C = H*H and returns the winner with every measurement."""
    f = features(H)
    D = DeviceCSR.from_host(H)
    times = {}
    # stage 1: table fill bounds, on the plain path
    best = None
    for sl in SYM_LOADS:
        for nl in NUM_LOADS:
            ms = _time_ms(Product(D, D, opts(sym_load_pct=sl, load_pct=nl)), reps)
            times["plain_s%d_n%d" % (sl, nl)] = ms
            if best is None or ms < best[0]:
                best = (ms, sl, nl)
    _, sl, nl = best
    # stage 2: rows in RCM order; the plain product over them (for reference), then cluster size and the
    # clustered product's numeric fill (its tables carry a value column per member, so its best fill can
    # differ from the plain product's)
    prep = {}
    t = time.perf_counter()
    rcm = order_rcm(H)
    prep["rcm"] = time.perf_counter() - t
    times["rcm"] = _time_ms(Product(DeviceCSR.from_host(permute_h(H, rcm, None, threads)), D,
                                    opts(sym_load_pct=sl, load_pct=nl)), reps)
    for mc in MAX_CLUSTERS:
        t = time.perf_counter()
        plan = plan_hierarchical(H, (3, 10), mc, SIM_ROOT, nthreads=threads, perm_in=rcm)
        Dc = cluster_build(D, plan)
        prep["hc%d" % mc] = time.perf_counter() - t
        for cl in CL_LOADS:
            times["hc%d_n%d" % (mc, cl)] = _time_ms(Product(Dc, D, opts(sym_load_pct=sl, load_pct=cl)), reps)
        times["hc%d" % mc] = min(times["hc%d_n%d" % (mc, cl)] for cl in CL_LOADS)
        del Dc
    cand = [("plain", 0, best[0])] + [("hc", mc, times["hc%d" % mc]) for mc in MAX_CLUSTERS]
    best_hc = min(cand[1:], key=lambda c: c[2])
    cl_best = min((times["hc%d_n%d" % (best_hc[1], cl)], cl) for cl in CL_LOADS)
    path, mc, ms = min(cand, key=lambda c: c[2])
    return {"class": matrix_class(f), "path": path, "max_cluster": mc, "best_cluster_size": best_hc[1],
            "sym_load_pct": sl, "load_pct": nl, "cl_load_pct": cl_best[1], "ms": ms, "times_ms": times,
            "prep_s": prep,
            "features": [float(x) for x in f], "nrows": int(H.nrows), "nnz": int(H.nnz)}


class TuneTable:
    """Per-class choices, stored as JSON: {class: entry}; each entry keeps the tuned fields and the
    measurements of the matrices it was tuned on."""

    def __init__(self, entries: dict | None = None):
        self.entries = dict(entries or {})

    @staticmethod
    def load(path: str = TABLE_PATH) -> "TuneTable":
        if not os.path.exists(path):
            return TuneTable()
        with open(path) as fh:
            return TuneTable(json.load(fh)["classes"])

    def save(self, path: str = TABLE_PATH):
        with open(path, "w") as fh:
            json.dump({"classes": self.entries}, fh, indent=1, sort_keys=True)

    def add(self, r: dict):
        """Adds one tuned matrix; a class tuned on several matrices keeps the choice with the smallest sum
        of per-matrix times relative to each matrix's own best."""
        e = self.entries.setdefault(r["class"], {"runs": []})
        e["runs"].append({k: r[k] for k in ("path", "max_cluster", "best_cluster_size", "sym_load_pct",
                                            "load_pct", "cl_load_pct", "ms", "times_ms", "nrows", "nnz")})
        runs = e["runs"]
        keys = set.intersection(*[set(x["times_ms"]) for x in runs])
        score = {k: sum(x["times_ms"][k] / x["ms"] for x in runs) for k in keys}
        stage1 = min((k for k in score if k.startswith("plain_")), key=score.get)
        sl, nl = (int(v[1:]) for v in stage1.split("_")[1:])
        paths = {"plain": score[stage1]}
        paths.update({k: score[k] for k in score if k.startswith("hc") and "_" not in k})
        win = min(paths, key=paths.get)
        hcs = [k for k in paths if k.startswith("hc") and "_" not in k]
        # the clustered product's fill at the class's best size: least summed relative time
        bcs = int(min(hcs, key=paths.get)[2:]) if hcs else 2
        cl_keys = [k for k in score if k.startswith("hc%d_n" % bcs)]
        e["cl_load_pct"] = int(min(cl_keys, key=score.get).split("_n")[1]) if cl_keys else nl
        e.update({"sym_load_pct": sl, "load_pct": nl, "path": "plain" if win == "plain" else "hc",
                  "max_cluster": 0 if win == "plain" else int(win[2:]),
                  "best_cluster_size": int(min(hcs, key=paths.get)[2:]) if hcs else 2})

    def lookup(self, f: np.ndarray) -> dict:
        e = self.entries.get(matrix_class(f))
        if e is None:
            return dict(DEFAULT, best_cluster_size=2, cl_load_pct=DEFAULT["load_pct"], tuned=False)
        return {"path": e["path"], "max_cluster": e["max_cluster"], "best_cluster_size": e["best_cluster_size"],
                "sym_load_pct": e["sym_load_pct"], "load_pct": e["load_pct"],
                "cl_load_pct": e.get("cl_load_pct", e["load_pct"]), "tuned": True}

    def opts_for(self, f: np.ndarray):
        e = self.lookup(f)
        return opts(sym_load_pct=e["sym_load_pct"], load_pct=e["load_pct"])


def tuning_set():
    """Seeded matrices of the workload families (smaller instances of each, large enough to fill the GPU
    the way the full-size ones do), name -> HostCSR."""
    import synth
    out = {}
    out["stencil27_90_relabelled"] = synth.workload_stencil27(90, 20, 21)[0]
    out["stencil27_80_relabelled"] = synth.workload_stencil27(80, 23, 24)[0]
    out["stencil27_70"] = synth.stencil(27, 70, 22)
    out["stencil7_40"] = synth.stencil(7, 40, 23)
    out["stencil5_300"] = synth.stencil(5, 300, 24)
    for d in (4, 8, 16, 32):
        out["uniform_50000_d%d" % d] = synth.uniform(50000, 50000, d, 25 + d)
    out["rmat14"] = synth.rmat(14, 16, 0.57, 0.19, 0.19, 26)
    return out


def main():
    import argparse
    p = argparse.ArgumentParser(description="tune the library's options per matrix class on this GPU")
    p.add_argument("--out", default=TABLE_PATH)
    p.add_argument("--reps", type=int, default=10)
    a = p.parse_args()
    table = TuneTable()
    for name, H in tuning_set().items():
        t = time.perf_counter()
        r = tune_matrix(H, a.reps)
        table.add(r)
        print("%-26s %-18s -> %s mc=%d sym=%d num=%d  %.3f ms (%.1fs)" % (
            name, r["class"], r["path"], r["max_cluster"], r["sym_load_pct"], r["load_pct"], r["ms"],
            time.perf_counter() - t), flush=True)
    table.save(a.out)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
