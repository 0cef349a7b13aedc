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

import math
import os
import time

import numpy as np

from . import (TUNE_CL_FILLS, TUNE_CLUSTER_SIZES, TUNE_NUM_FILLS, TUNE_SYM_FILLS, DeviceCSR, Product, SIM_ROOT,
               TuneTableNative, c_tune_run, cluster_build, features, opts, order_rcm, permute_h, plan_hierarchical,
               tune_class)

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.txt")


def matrix_class(f: np.ndarray) -> str:
    """Class key from the structure features (the library's rule, include/hcsp.h): mean row length, spread of
    the per-row work, compression of products into output entries, the best similarity a row finds (what
    clustering can exploit), and whether columns lie near the diagonal."""
    return tune_class(f)


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
    """Times the library's candidate grid on the GPU for C = H*H; returns the class key, the run (the
    library's record of the measurements), and the preprocessing times."""
    f = features(H)
    D = DeviceCSR.from_host(H)
    run = c_tune_run()
    run.nrows, run.nnz = H.nrows, H.nnz
    nan = float("nan")
    for i in range(len(TUNE_SYM_FILLS)):
        for j in range(len(TUNE_NUM_FILLS)):
            run.plain_ms[i][j] = _time_ms(Product(D, D, opts(sym_load_pct=TUNE_SYM_FILLS[i],
                                                              load_pct=TUNE_NUM_FILLS[j])), reps)
    # the clustered candidates use the plain grid's best fills (stage 2)
    flat = [(run.plain_ms[i][j], i, j) for i in range(len(TUNE_SYM_FILLS)) for j in range(len(TUNE_NUM_FILLS))]
    _, si, ni = min(flat)
    sl, nl = TUNE_SYM_FILLS[si], TUNE_NUM_FILLS[ni]
    prep = {}
    t = time.perf_counter()
    rcm = order_rcm(H)
    prep["rcm"] = time.perf_counter() - t
    run.rcm_ms = _time_ms(Product(DeviceCSR.from_host(permute_h(H, rcm, None, threads)), D,
                                  opts(sym_load_pct=sl, load_pct=nl)), reps)
    for i, mc in enumerate(TUNE_CLUSTER_SIZES):
        t = time.perf_counter()
        plan = plan_hierarchical(H, (3, 10), mc, SIM_ROOT, nthreads=threads, perm_in=rcm)
        Dc = cluster_build(D, plan)
        prep["hc%d" % mc] = time.perf_counter() - t
        for j, cl in enumerate(TUNE_CL_FILLS):
            run.hc_ms[i][j] = _time_ms(Product(Dc, D, opts(sym_load_pct=sl, load_pct=cl)), reps)
        del Dc
    key = matrix_class(f)
    one = TuneTableNative()
    one.add(key, run)
    return {"class": key, "run": run, "choice": one.get(key), "prep_s": prep,
            "features": [float(x) for x in f], "nrows": int(H.nrows), "nnz": int(H.nnz)}


def run_ms(run: c_tune_run) -> float:
    """The run's best time over the plain grid and every cluster size."""
    ts = [run.plain_ms[i][j] for i in range(len(TUNE_SYM_FILLS)) for j in range(len(TUNE_NUM_FILLS))]
    ts += [run.hc_ms[i][j] for i in range(len(TUNE_CLUSTER_SIZES)) for j in range(len(TUNE_CL_FILLS))]
    return min(t for t in ts if math.isfinite(t) and t > 0)


class TuneTable:
    """Per-class runs and choices: the library's table (hcsp_tune_*), stored as its text file."""

    def __init__(self, native: TuneTableNative | None = None):
        self.native = native or TuneTableNative()

    @staticmethod
    def load(path: str = TABLE_PATH) -> "TuneTable":
        if not os.path.exists(path):
            return TuneTable()
        return TuneTable(TuneTableNative.load(path))

    def save(self, path: str = TABLE_PATH):
        self.native.save(path)

    def add(self, r: dict):
        """Adds one tuned matrix (a tune_matrix result) to its class."""
        self.native.add(r["class"], r["run"])

    def entry(self, key: str) -> dict:
        return self.native.get(key)

    def classes(self) -> list:
        return self.native.classes()

    def lookup(self, f: np.ndarray) -> dict:
        return self.native.lookup(f)

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
        c = r["choice"]
        print("%-26s %-22s -> %s mc=%d sym=%d num=%d  %.3f ms (%.1fs)" % (
            name, r["class"], c["path"], c["max_cluster"], c["sym_load_pct"], c["load_pct"], run_ms(r["run"]),
            time.perf_counter() - t), flush=True)
    table.save(a.out)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
