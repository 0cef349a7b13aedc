#!/usr/bin/env python3
"""Benchmark: clustered vs plain Gustavson SpGEMM on one MI355X.

Workload (default): C = M*M for M the 27-point stencil on a 100^3 grid with
values U(-1,1), symmetrically relabelled by a seeded random permutation so
the natural locality is gone.  The method recovers it: A's rows are put in
reverse Cuthill-McKee order, hierarchical clustering (Alg. 3, jacc_th 0.3,
at most 4 rows per cluster by default -- the autotuner's choice for this
matrix class; the paper uses 8) regroups similar rows into CSR_Cluster, and the product runs
cluster-wise (Alg. 1) against B = M.  The baseline is the plain row-wise
product of M in its given order.  One step = symbolic phase (binning, counts,
scan), the nnz read-back, and the numeric phase of the clustered product;
the plain-CSR product of the same matrix is timed the same way for the
comparison.  Clustering itself (host plan + device CSR_Cluster build) is
preprocessing, timed once and reported in units of one SpGEMM.

Prints one JSON line.  ``--mode copy`` runs only a plain device copy of known
size (the calibration run for hardware byte counters); ``--mode batch``,
``--mode tallskinny`` and ``--mode rmat`` measure the batched products, the
square x tall-skinny products and the power-law R-MAT product.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def csr_bytes(nrows: int, nnz: int) -> int:
    return 8 * (nrows + 1) + 12 * nnz


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--m", type=int, default=100, help="stencil grid side")
    p.add_argument("--max-cluster", type=int, default=0,
                   help="rows per cluster at most (0: the autotuner's choice for the matrix class, else 2)")
    p.add_argument("--sim", choices=["root", "union"], default="root")
    p.add_argument("--clustering", choices=["hierarchical", "variable", "fixed"], default="hierarchical",
                   help="plan: Alg. 3 (default), Alg. 2 (threshold 3/10) or fixed-length blocks")
    p.add_argument("--reorder", choices=["rcm", "degree", "random", "none"], default="rcm",
                   help="row order of A before clustering (A = M with rows permuted, B = M)")
    p.add_argument("--symmetric", action="store_true",
                   help="permute M symmetrically (rows and columns; B reordered too) instead of A's rows only")
    p.add_argument("--lanes", type=int, default=0)
    p.add_argument("--mode", choices=["bench", "copy", "batch", "tallskinny", "rmat"], default="bench",
                   help="bench: the stencil workload (the headline line); batch: 512 uneven products replayed "
                        "as one captured graph; tallskinny: the stencil times 10 BFS frontier matrices; copy: "
                        "device copy for counter calibration")
    p.add_argument("--sources", type=int, default=512, help="tallskinny: BFS sources (columns of B)")
    p.add_argument("--iterations", type=int, default=10, help="tallskinny: frontier matrices (BFS levels 1..)")
    p.add_argument("--batch-count", type=int, default=512)
    p.add_argument("--rmat-scale", type=int, default=20, help="rmat: scale of the full product (numeric in panels)")
    p.add_argument("--rmat-cluster-scale", type=int, default=18,
                   help="rmat: scale of the plain vs clustered comparison (C held whole)")
    p.add_argument("--panel-gb", type=float, default=32.0, help="rmat: C panel buffer size")
    p.add_argument("--win-chunk-log2", type=int, default=0,
                   help="rmat: log2 of the products per column chunk of rows too long for shared memory "
                        "(0: the library default)")
    p.add_argument("--load-pct", type=int, default=0, help="numeric table fill target (0: autotuned)")
    p.add_argument("--sym-load-pct", type=int, default=0, help="symbolic table fill bound (0: autotuned)")
    p.add_argument("--untuned", action="store_true", help="ignore the autotuner's table")
    p.add_argument("--margin", type=float, default=0.1, help="margin on the predicted compression ratio")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-extras", action="store_true",
                   help="only the three timed products (no GPU-assisted plan, CSR_Cluster output or learned legs; "
                        "for counter runs that attribute launches by their order)")
    p.add_argument("--cpu-threads", type=int, default=0)
    p.add_argument("--cpu-runs", type=int, default=10, help="timed runs of the CPU oracle (mean and median)")
    return p.parse_args()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_num_stencil27_100_relabelled.md")
KERNEL_SOURCES = ["paper_2507_21253_amd/csrc/hash.hip"]


def numeric_traffic(key: str, config: str):
    """HBM bytes of one numeric phase from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE, each scaled by the copy-kernel calibration), or None when the numeric kernels' sources
    changed since the counters were taken or they were taken on another configuration."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    m = re.search(r"traffic: clustered_numeric_bytes=(\d+) plain_numeric_bytes=(\d+) kernel_source=(\w+) "
                  r"config=(\S+)", open(TRAFFIC_PROFILE).read())
    if not m or m.group(3) != h.hexdigest()[:16] or m.group(4) != config:
        return None
    return int(m.group(1) if key == "clustered" else m.group(2))


def copy_bandwidth(torch, n=1 << 28, reps=5):
    """GB/s (read + write) of a plain device copy of 2 GiB of float64 on the current stream."""
    try:
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
    except RuntimeError:
        return None
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 16 * n / ms / 1e6


def copy_mode(args):
    import torch
    n = 1 << 28  # 2 GiB of float64
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    print(json.dumps({"mode": "copy", "bytes_read": 8 * n, "bytes_written": 8 * n, "ms": ms,
                      "gbs": 16 * n / ms / 1e6}), flush=True)


def tallskinny_mode(args):
    """Square x tall-skinny products (the paper's second workload): A = the relabelled 27-point stencil,
    B_L = its multi-source BFS frontier matrix after L steps (one column per source), L = 1..iterations.
    A is reordered (RCM rows) and clustered (hierarchical, the tuned size) once and reused for every B_L;
    each product is timed plain and clustered (symbolic, read-back, numeric), with library default table
    fills; the clustered C must equal the plain C bit for bit (the products' parity with the oracle is
    tested in tests/test_gpu_tallskinny.py)."""
    import torch
    import paper_2507_21253_amd as hc
    import synth
    m = args.m
    M, _, _ = synth.workload_stencil27(m, 2, 3)
    t = time.perf_counter()
    Bs = [synth.frontiers(M, args.sources, L, 12) for L in range(1, args.iterations + 1)]
    log("frontiers: %d sources, nnz %s (%.1fs)" % (args.sources, [B.nnz for B in Bs], time.perf_counter() - t))
    from paper_2507_21253_amd import tune
    tuned = (tune.TuneTable() if args.untuned else tune.TuneTable.load()).lookup(hc.features(M))
    mc = args.max_cluster or (tuned["best_cluster_size"] if tuned["tuned"] else 2)
    ncpu = len(os.sched_getaffinity(0))
    t = time.perf_counter()
    plan = hc.plan_hierarchical(M, (3, 10), mc, hc.SIM_ROOT, nthreads=ncpu, perm_in=hc.order_rcm(M))
    t_prep = time.perf_counter() - t
    Md = hc.DeviceCSR.from_host(M)
    Dc = hc.cluster_build(Md, plan)
    torch.cuda.synchronize()
    rl = np.diff(M.rp)
    rows = []
    tot = {"plain": 0.0, "clustered": 0.0}
    flops = 0
    for L, B in enumerate(Bs, 1):
        Bd = hc.DeviceCSR.from_host(B)
        products = int(np.diff(B.rp)[M.col].sum())
        flops += 2 * products
        P_pl, P_cl = hc.Product(Md, Bd), hc.Product(Dc, Bd)
        w_pl = time_product(P_pl, args.steps, args.warmup, torch)[0]
        w_cl = time_product(P_cl, args.steps, args.warmup, torch)[0]
        nnz = P_pl.info.nnz
        assert P_cl.info.nnz == nnz
        assert (torch.equal(P_cl.C_row_ptr, P_pl.C_row_ptr) and torch.equal(P_cl.C_col[:nnz], P_pl.C_col[:nnz])
                and torch.equal(P_cl.C_val[:nnz].view(torch.int64), P_pl.C_val[:nnz].view(torch.int64)))
        tot["plain"] += w_pl
        tot["clustered"] += w_cl
        rows.append({"iteration": L, "nnz_B": B.nnz, "products": products, "nnz_C": int(nnz),
                     "plain_ms": round(w_pl, 4), "clustered_ms": round(w_cl, 4)})
        log("L=%d nnz(B)=%d products=%d: plain %.3f ms, clustered %.3f ms" % (L, B.nnz, products, w_pl, w_cl))
        del P_pl, P_cl, Bd
    out = {"metric": "tall-skinny SpGEMM GFLOP/s (A x %d BFS frontier matrices)" % len(Bs),
           "value": round(flops / (tot["clustered"] * 1e-3) / 1e9, 3), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(tot["clustered"], 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "stencil27_%d^3_relabelled_x_bfs_frontiers" % m, "sources": args.sources,
                      "iterations": len(Bs), "max_cluster": mc, "reorder": "rcm rows of A",
                      "clustering": "hierarchical"},
           "plain_ms_total": round(tot["plain"], 4), "speedup_clustered_vs_plain": round(tot["plain"] / tot["clustered"], 3),
           "preprocessing_host_s": round(t_prep, 3),
           "preprocessing_in_products": round(t_prep * 1e3 / (tot["clustered"] / len(Bs)), 1),
           "per_iteration": rows}
    print(json.dumps(out), flush=True)

def rmat_panels(D, hc, torch, panel_entries, steps, warmup, wlog2=0):
    """C = A*A for an A too large to hold C: symbolic over all rows, C's row offsets read back, then the
    numeric phase in row panels of at most panel_entries entries written one after another into one
    reused buffer.  Returns (ms per product, symbolic ms, numeric ms, nnz(C), panels)."""
    o = hc.opts(win_chunk_log2=wlog2)
    ws = torch.empty(hc.spgemm_workspace(D, D, o), dtype=torch.uint8, device="cuda")
    crp = torch.empty(D.nrows + 1, dtype=torch.int64, device="cuda")
    info = hc.spgemm_symbolic(D, D, crp, ws, o)
    nnz = int(info.nnz)
    cap = int(min(panel_entries, max(nnz, 1)))
    col = torch.empty(cap, dtype=torch.int32, device="cuda")
    val = torch.empty(cap, dtype=torch.float64, device="cuda")

    def one():
        t0 = time.perf_counter()
        inf = hc.spgemm_symbolic(D, D, crp, ws, o)
        rp = crp.cpu().numpy()
        t1 = time.perf_counter()
        lo, np_ = 0, 0
        while lo < D.nrows:
            hi = int(np.searchsorted(rp, rp[lo] + cap, side="right")) - 1
            hi = max(hi, lo + 1)
            if rp[hi] - rp[lo] > cap:
                raise RuntimeError("row %d alone exceeds the panel buffer" % lo)
            hc.spgemm_numeric(D, D, inf, crp, col, val, ws,
                              hc.opts(unit_lo=lo, unit_hi=hi, out_base=int(rp[lo]), win_chunk_log2=wlog2),
                              capacity=cap)
            lo, np_ = hi, np_ + 1
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return (t2 - t0) * 1e3, (t1 - t0) * 1e3, (t2 - t1) * 1e3, np_

    for _ in range(warmup):
        one()
    runs = [one() for _ in range(steps)]
    del col, val, ws
    torch.cuda.empty_cache()
    return (float(np.mean([r[0] for r in runs])), float(np.mean([r[1] for r in runs])),
            float(np.mean([r[2] for r in runs])), nnz, runs[0][3])


def rmat_mode(args):
    """The power-law workload: R-MAT (edge factor 16, a=0.57, b=c=0.19, seed 4; self-loops dropped,
    symmetrised, de-duplicated, values 1.0), C = A*A.  At the full scale C does not fit one GPU (about 2.4e10
    entries), so the symbolic phase runs over all rows and the numeric phase in row panels (one reused
    buffer): each step is symbolic + read-back + every panel.  At a smaller scale, where C fits, plain CSR is
    compared with CSR_Cluster (rows in RCM order, hierarchical clusters with the candidate search on the GPU)."""
    import torch
    import paper_2507_21253_amd as hc
    import synth
    out = {}
    R = synth.workload_rmat(args.rmat_scale, 4)
    rl = np.diff(R.rp)
    products = int(rl[R.col].sum())
    D = hc.DeviceCSR.from_host(R)
    panel_entries = int(args.panel_gb * 1e9 / 12)
    ms, sym, num, nnz, npan = rmat_panels(D, hc, torch, panel_entries, max(1, min(args.steps, 3)),
                                          min(args.warmup, 1), args.win_chunk_log2)
    log("rmat%d: %d rows, nnz %d, products %d, nnz(C) %d: %.1f ms (symbolic %.1f, numeric %.1f in %d panels)"
        % (args.rmat_scale, R.nrows, R.nnz, products, nnz, ms, sym, num, npan))
    out.update({"metric": "SpGEMM GFLOP/s, R-MAT C = A*A (numeric in row panels)",
                "value": round(2 * products / (ms * 1e-3) / 1e9, 3), "unit": "GFLOP/s", "n_gpus": 1,
                "steps": max(1, min(args.steps, 3)), "warmup": min(args.warmup, 1), "ms_per_step": round(ms, 2),
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                "data": "synthetic",
                "config": {"workload": "rmat%d_ef16_A2" % args.rmat_scale, "nrows": R.nrows, "nnz_A": R.nnz,
                           "products": products, "nnz_C": nnz, "panels": npan, "panel_gb": args.panel_gb,
                           "win_chunk_log2": args.win_chunk_log2 or None},
                "phases_ms": {"symbolic_incl_readback": round(sym, 2), "numeric_all_panels": round(num, 2)}})
    del D
    torch.cuda.empty_cache()
    # plain vs clustered where C fits
    sc = args.rmat_cluster_scale
    R = synth.workload_rmat(sc, 4)
    rl = np.diff(R.rp)
    products = int(rl[R.col].sum())
    D = hc.DeviceCSR.from_host(R)
    ow = hc.opts(win_chunk_log2=args.win_chunk_log2)
    P = hc.Product(D, D, ow)
    w_pl, s_pl, n_pl = time_product(P, max(1, min(args.steps, 3)), 1, torch)
    nnz = P.info.nnz
    ref_rp, ref_col = P.C_row_ptr.clone(), P.C_col[:nnz].clone()
    ref_val = P.C_val[:nnz].view(torch.int64).clone()
    del P
    torch.cuda.empty_cache()
    mc = args.max_cluster or 2
    t = time.perf_counter()
    perm = hc.order_rcm(R)
    plan = hc.plan_hierarchical_gpu(R, D, (3, 10), mc, hc.SIM_ROOT, perm_in=perm)
    t_prep = time.perf_counter() - t
    Dc = hc.cluster_build(D, plan)
    Pc = hc.Product(Dc, D, ow)
    w_cl, s_cl, n_cl = time_product(Pc, max(1, min(args.steps, 3)), 1, torch)
    same = bool(Pc.info.nnz == nnz and torch.equal(Pc.C_row_ptr, ref_rp) and torch.equal(Pc.C_col[:nnz], ref_col)
                and torch.equal(Pc.C_val[:nnz].view(torch.int64), ref_val))
    log("rmat%d: plain %.1f ms (sym %.1f, num %.1f); clustered %.1f ms (sym %.1f, num %.1f), %d clusters, "
        "equal %s, plan %.1f s" % (sc, w_pl, s_pl, n_pl, w_cl, s_cl, n_cl, plan.nclusters, same, t_prep))
    out["clustered_comparison"] = {
        "workload": "rmat%d_ef16_A2" % sc, "products": products, "nnz_C": int(nnz),
        "plain_ms": round(w_pl, 2), "plain_gflops": round(2 * products / (w_pl * 1e-3) / 1e9, 3),
        "plain_phases_ms": [round(s_pl, 2), round(n_pl, 2)],
        "clustered_ms": round(w_cl, 2), "clustered_gflops": round(2 * products / (w_cl * 1e-3) / 1e9, 3),
        "clustered_phases_ms": [round(s_cl, 2), round(n_cl, 2)],
        "reorder": "rcm rows", "clustering": "hierarchical (candidates on the GPU)", "max_cluster": mc,
        "nclusters": int(plan.nclusters), "plan_s": round(t_prep, 2), "clustered_equals_plain_bitwise": same}
    print(json.dumps(out), flush=True)


def batch_mode(args):
    """512 independent products C_p = A_p*A_p (seeds 1000..1511: 2-D 5-point / 3-D 7-point stencils and
    uniform-random matrices with 4..32 entries per row, sizes log-uniform in [1e3, 2e5] rows), both phases
    for all of them in one launch sequence captured into a graph; one step = one replay."""
    import torch
    import paper_2507_21253_amd as hc
    import synth
    t = time.perf_counter()
    hosts = [synth.batch_problem(s)[1] for s in range(1000, 1000 + args.batch_count)]
    ds = [hc.DeviceCSR.from_host(H) for H in hosts]
    rows = sum(H.nrows for H in hosts)
    products = 0
    for H in hosts:
        products += int(np.diff(H.rp)[H.col].sum())
    log("batch: %d products, %d rows, %d A entries, %d products (%.1fs)"
        % (len(hosts), rows, sum(H.nnz for H in hosts), products, time.perf_counter() - t))
    # the autotuner's choice per matrix class: table options and, where it pays, hierarchical clusters;
    # products with equal choices form one batch, and all batches go into one graph
    from paper_2507_21253_amd import tune
    table = tune.TuneTable() if args.untuned else tune.TuneTable.load()
    groups = {}
    t = time.perf_counter()
    for H, d in zip(hosts, ds):
        e = table.lookup(hc.features(H))
        if args.load_pct or args.sym_load_pct:
            e = dict(e, path="plain", load_pct=args.load_pct or 60, sym_load_pct=args.sym_load_pct or 70)
        key = (e["path"], e["max_cluster"], e["sym_load_pct"], e["cl_load_pct"] if e["path"] == "hc" else e["load_pct"])
        A = d
        if e["path"] == "hc":
            A = hc.cluster_build(d, hc.plan_hierarchical(H, (3, 10), e["max_cluster"], hc.SIM_ROOT,
                                                         nthreads=len(os.sched_getaffinity(0)),
                                                         perm_in=hc.order_rcm(H)))
        groups.setdefault(key, []).append((A, d))
    t_prep = time.perf_counter() - t
    log("groups: %s (%.1fs)" % ({"%s/%d/s%d/n%d" % k: len(v) for k, v in groups.items()}, t_prep))
    order = [pair for k in groups for pair in groups[k]]
    bts = [hc.Batch(groups[k], hc.opts(sym_load_pct=k[2], load_pct=k[3])) for k in groups]
    for bt in bts:
        bt.run()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for bt in bts:
                bt.run(s)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    ms = e0.elapsed_time(e1) / args.steps
    nnz_by = {id(A): z for bt in bts for (A, _), z in zip(bt.pairs, bt.status())}
    nnz = np.array([nnz_by[id(A)] for A, _ in order])
    hosts_in_order = {id(d): H for H, d in zip(hosts, ds)}
    # the same products one at a time with the library defaults (symbolic, read-back, numeric each)
    Ps = [hc.Product(d, d) for _, d in order]
    for P in Ps:
        P.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for P in Ps:
        P.run(check=False)
    torch.cuda.synchronize()
    loop_ms = (time.perf_counter() - t0) * 1e3
    for P in Ps:
        P.check()
    assert all(int(P.info.nnz) == int(z) for P, z in zip(Ps, nnz))
    a_bytes = sum(csr_bytes(H.nrows, H.nnz) for H in hosts)
    c_bytes = sum(csr_bytes(hosts_in_order[id(d)].nrows, int(z)) for (_, d), z in zip(order, nnz))
    out = {"metric": "batched SpGEMM GFLOP/s (graph replay of one launch sequence)",
           "value": round(2 * products / (ms * 1e-3) / 1e9, 3), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "wall_ms_per_step": round(wall, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batch_%d_stencil5_stencil7_uniform" % len(hosts), "rows": rows,
                      "products": products, "nnz_C": int(nnz.sum())},
           "gbs_compulsory": round((2 * a_bytes + c_bytes) / (ms * 1e-3) / 1e9, 2),
           "one_at_a_time_ms": round(loop_ms, 3), "speedup_vs_one_at_a_time": round(loop_ms / ms, 3),
           "tuned_groups": {"%s/%d/s%d/n%d" % k: len(v) for k, v in groups.items()},
           "tuned_prep_s": round(t_prep, 2)}
    print(json.dumps(out), flush=True)


def time_product(P, steps, warmup, torch, detail=None):
    """Runs warmup + timed steps of symbolic+numeric; returns per-step wall ms and phase ms (means over the
    steps).  ``detail`` (a dict), when given, receives the per-step event times and their medians."""
    for _ in range(warmup):
        P.run()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(s)
        P.symbolic()
        ev[i][1].record(s)
        P.numeric()
        ev[i][2].record(s)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    P.check()                                  # errors the kernels recorded in the timed runs
    syms = [a.elapsed_time(b) for a, b, c in ev]
    nums = [b.elapsed_time(c) for a, b, c in ev]
    if detail is not None:
        detail.update({"step_ms_median": float(np.median([x + y for x, y in zip(syms, nums)])),
                       "symbolic_ms_median": float(np.median(syms)), "numeric_ms_median": float(np.median(nums)),
                       "numeric_ms": nums})
    return wall, float(np.mean(syms)), float(np.mean(nums))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (sharding is a design note); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.mode == "copy":
        copy_mode(args)
        return
    if args.mode == "batch":
        batch_mode(args)
        return
    if args.mode == "tallskinny":
        tallskinny_mode(args)
        return
    if args.mode == "rmat":
        rmat_mode(args)
        return
    import paper_2507_21253_amd as hc
    import synth

    m = args.m
    t = time.perf_counter()
    M, S, q = synth.workload_stencil27(m, 2, 3)
    log("inputs: %d rows, nnz %d (%.1fs)" % (M.nrows, M.nnz, time.perf_counter() - t))
    rowlen = np.diff(M.rp)
    products = int(rowlen[M.col].sum())
    flop = 2 * products

    # ---- the autotuner's choices for this matrix class (table options, cluster size)
    from paper_2507_21253_amd import tune
    tuned = (tune.TuneTable() if args.untuned else tune.TuneTable.load()).lookup(hc.features(M))
    if not args.max_cluster:
        args.max_cluster = tuned["best_cluster_size"] if tuned["tuned"] else 2
    log("tuner: %s" % tuned)

    # ---- preprocessing: reordering (host), hierarchical plan (host), CSR_Cluster (device).  With rows-only
    # reordering the plan works on M's rows in the new order (perm_in) and names original rows, so the
    # CSR_Cluster is built from M itself and C comes out in M's row order; a symmetric reordering needs the
    # reordered matrix (its columns change too).
    ncpu = len(os.sched_getaffinity(0))
    t = time.perf_counter()
    P = None
    if args.reorder != "none":
        P = (hc.order_rcm(M) if args.reorder == "rcm" else hc.order_degree(M) if args.reorder == "degree"
             else synth.perm(M.nrows, 17))  # random: a seeded uniform permutation
    t_reorder = time.perf_counter() - t
    R = M if P is None else hc.permute_h(M, P, P if args.symmetric else None, ncpu)  # the reordered baseline
    A_plan, perm_in = (R, None) if args.symmetric else (M, P)
    t = time.perf_counter()
    if args.clustering == "variable":
        plan = hc.plan_variable(A_plan, (3, 10), args.max_cluster, perm_in=perm_in)
    elif args.clustering == "fixed":
        plan = hc.plan_fixed(A_plan.nrows, args.max_cluster, perm_in)
    else:
        plan = hc.plan_hierarchical(A_plan, (3, 10), args.max_cluster,
                                    hc.SIM_UNION if args.sim == "union" else hc.SIM_ROOT, nthreads=ncpu,
                                    perm_in=perm_in)
    t_plan = time.perf_counter() - t
    log("reorder %s %.2fs; plan: %d clusters (%.2fs, %d threads)" % (args.reorder, t_reorder, plan.nclusters,
                                                                     t_plan, ncpu))
    Md = hc.DeviceCSR.from_host(M)
    Rd = Md if R is M else hc.DeviceCSR.from_host(R)
    Bd = Rd if args.symmetric else Md          # right operand: M, or the reordered M
    # the same plan with the candidate search (SpGEMM_TopK) on the GPU and only the merge loop on the host
    t_plan_gpu = None
    if args.clustering == "hierarchical" and not args.symmetric and not args.no_extras:
        hc.plan_hierarchical_gpu(M, Md, (3, 10), args.max_cluster, hc.SIM_UNION if args.sim == "union"
                                 else hc.SIM_ROOT, perm_in=perm_in)  # warm-up (allocations, code load)
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan_g = hc.plan_hierarchical_gpu(M, Md, (3, 10), args.max_cluster, hc.SIM_UNION if args.sim == "union"
                                          else hc.SIM_ROOT, perm_in=perm_in)
        t_plan_gpu = time.perf_counter() - t
        assert np.array_equal(plan_g.perm, plan.perm) and np.array_equal(plan_g.cl_row_ptr, plan.cl_row_ptr)
        log("plan with GPU candidate search: %.3fs (host plan %.3fs), same plan" % (t_plan_gpu, t_plan))
        del plan_g
        torch.cuda.empty_cache()
    Ad = Rd if args.symmetric else Md          # the matrix the CSR_Cluster is built from
    torch.cuda.synchronize()
    for _ in range(2):
        Dc = hc.cluster_build(Ad, plan)
    torch.cuda.synchronize()
    t = time.perf_counter()
    Dc = hc.cluster_build(Ad, plan)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t
    log("CSR_Cluster: ncc %d nslots %d max %d (%.3fs)" % (Dc.ncc, Dc.nslots, Dc.max_cluster, t_build))

    o = hc.opts(lanes=args.lanes, load_pct=args.load_pct or tuned["load_pct"],
                sym_load_pct=args.sym_load_pct or tuned["sym_load_pct"])
    o_cl = hc.opts(lanes=args.lanes, load_pct=args.load_pct or tuned["cl_load_pct"],
                   sym_load_pct=args.sym_load_pct or tuned["sym_load_pct"])
    P_cl = hc.Product(Dc, Bd, o_cl)
    P_pl = hc.Product(Md, Md, o)
    det_cl = {}
    wall_cl, sym_cl, num_cl = time_product(P_cl, args.steps, args.warmup, torch, det_cl)
    nnzC = P_cl.info.nnz
    wall_pl, sym_pl, num_pl = time_product(P_pl, args.steps, args.warmup, torch)
    assert P_pl.info.nnz == nnzC
    if not args.symmetric:
        # both products give C in M's row order: the clustered one must equal the plain one bit for bit
        same = (torch.equal(P_cl.C_row_ptr, P_pl.C_row_ptr) and torch.equal(P_cl.C_col[:nnzC], P_pl.C_col[:nnzC])
                and torch.equal(P_cl.C_val[:nnzC].view(torch.int64), P_pl.C_val[:nnzC].view(torch.int64)))
        assert same, "clustered and plain products differ"
    wall_ro = None
    if R is not M:
        P_ro = hc.Product(Rd, Bd, o)
        wall_ro, sym_ro, num_ro = time_product(P_ro, args.steps, args.warmup, torch)
        assert P_ro.info.nnz == nnzC
        del P_ro
    if m >= 3:
        assert nnzC == (5 * m - 6) ** 3, "nnz(C) differs from the closed form"
    # ---- the learned selector and nnz predictor, when a trained model is in the tree
    learned_out = None
    from paper_2507_21253_amd import learned
    if os.path.exists(learned.MODEL) and not args.no_extras:
        sel = learned.Selector.load()
        f = hc.features(M)[None, :]
        z = sel.logits(f)[0]
        ratio_pred = float(np.exp(z[len(learned.PATHS)]))
        ratio = min(1.0, ratio_pred * (1 + args.margin))
        PP = hc.PredictedProduct(Md, Md, ratio, o)
        for _ in range(args.warmup):
            PP.run()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            PP.run()
        torch.cuda.synchronize()
        wall_pp = (time.perf_counter() - t) * 1e3 / args.steps
        assert PP.nnz == nnzC
        # the predicted-size C equals the clustered product's C bit for bit (which the CPU leg below
        # compares with the oracle's C)
        pred_equal = bool(torch.equal(PP.C_row_ptr, P_cl.C_row_ptr) and torch.equal(PP.C_col[:nnzC], P_cl.C_col[:nnzC])
                          and torch.equal(PP.C_val[:nnzC].view(torch.int64), P_cl.C_val[:nnzC].view(torch.int64)))
        assert pred_equal, "predicted-size and clustered products differ"
        learned_out = {"selector_choice": learned.PATHS[int(np.argmax(z[:len(learned.PATHS)]))],
                       "ratio_predicted": round(ratio_pred, 4), "ratio_true": round(nnzC / products, 4),
                       "margin": args.margin, "predicted_size_product": {
                           "ms_per_step": round(wall_pp, 4), "gflops": round(flop / (wall_pp * 1e-3) / 1e9, 3),
                           "rows_recomputed_exactly": int(PP.n_overflow),
                           "equals_clustered_bitwise": pred_equal}}
        log("learned: %s" % learned_out)
        del PP

    # ---- C written in CSR_Cluster form on A's clusters (Alg. 1's output), same operands and options
    clout = None
    if not args.symmetric and not args.no_extras:
        CP = hc.ClusterProduct(Dc, Bd, o_cl)
        for _ in range(args.warmup):
            CP.run()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            Ccl = CP.run()
        torch.cuda.synchronize()
        wall_co = (time.perf_counter() - t) * 1e3 / args.steps
        clout = {"ms_per_step": round(wall_co, 4), "gflops": round(flop / (wall_co * 1e-3) / 1e9, 3),
                 "ncc": int(Ccl.ncc), "nslots": int(Ccl.nslots), "bytes_over_csr": round(Ccl.bytes() /
                                                                                        csr_bytes(M.nrows, nnzC), 3)}
        log("CSR_Cluster output: %s" % clout)
        del CP, Ccl

    log("clustered: %.3f ms/step (sym %.3f, num %.3f); plain: %.3f ms/step (sym %.3f, num %.3f); "
        "plain reordered: %s" % (wall_cl, sym_cl, num_cl, wall_pl, sym_pl, num_pl,
                                 "-" if wall_ro is None else "%.3f ms/step (sym %.3f, num %.3f)" % (wall_ro, sym_ro,
                                                                                                   num_ro)))

    bytes_A = csr_bytes(M.nrows, M.nnz)
    bytes_Acl = Dc.bytes()
    bytes_C = csr_bytes(M.nrows, nnzC)
    comp = 2 * bytes_A + bytes_C                     # compulsory traffic |A| + |B| + |C| (CSR sizes)
    comp_cl = bytes_Acl + bytes_A + bytes_C          # the same with A in its CSR_Cluster form
    gflops_cl = flop / (wall_cl * 1e-3) / 1e9
    gflops_pl = flop / (wall_pl * 1e-3) / 1e9
    # dominant kernel family: the numeric launches of one product; algorithmic bytes |A| + |B| + |C|
    ach = comp / (num_cl * 1e-3) / 1e9
    ach_step = comp / (wall_cl * 1e-3) / 1e9
    copy_gbs = copy_bandwidth(torch)
    traffic = numeric_traffic("clustered", "m%d_%s%s_mc%d_%s_s%d_n%d" % (
        m, args.reorder, "sym" if args.symmetric else "", args.max_cluster, args.sim, o_cl.sym_load_pct,
        o_cl.load_pct))

    cpu = None
    oracle_equal = None
    if not args.no_cpu:
        import oracle
        nth = args.cpu_threads or ncpu
        oracle.spgemm_mt(M, M, nth, structure_only=True)  # warm the pages
        runs = []
        for _ in range(args.cpu_runs):
            t = time.perf_counter()
            Cref = oracle.spgemm_mt(M, M, nth)
            runs.append(time.perf_counter() - t)
        # the timed clustered C against the oracle's C, entry by entry (row offsets, columns, value bits)
        oracle_equal = bool(np.array_equal(P_cl.C_row_ptr.cpu().numpy(), Cref.rp)
                            and np.array_equal(P_cl.C_col[:nnzC].cpu().numpy(), Cref.col)
                            and np.array_equal(P_cl.C_val[:nnzC].cpu().numpy().view(np.int64),
                                               Cref.val.view(np.int64)))
        assert oracle_equal, "the clustered product differs from the oracle"
        del Cref
        tcpu = float(np.mean(runs))
        # one thread on a bounded slice of the rows (the first 1/16)
        hi1 = M.nrows // 16
        flop1 = 2 * int(rowlen[M.col[:M.rp[hi1]]].sum())
        t = time.perf_counter()
        oracle.spgemm(M, M, (0, hi1))
        t1 = time.perf_counter() - t
        cpu = {"value": round(flop / tcpu / 1e9, 3), "unit": "GFLOP/s", "cores": nth, "kind": "oracle",
               "sample": "full C = M*M (count pass + fill pass), mean of %d runs, %.2f s each" % (len(runs), tcpu),
               "median_value": round(flop / float(np.median(runs)) / 1e9, 3),
               "cpu_model": cpu_model(),
               "single_thread": {"value": round(flop1 / t1 / 1e9, 3), "unit": "GFLOP/s",
                                 "sample": "rows [0, %d) of C = M*M on one thread, %.2f s" % (hi1, t1)}}

    out = {
        "metric": "SpGEMM GFLOP/s + achieved HBM GB/s, CSR_Cluster vs plain CSR on 1 MI355X",
        "value": round(gflops_cl, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_cl, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "stencil27_%d^3_relabelled_A2" % m, "nrows": M.nrows, "nnz_A": M.nnz,
                   "nnz_C": nnzC, "products": products, "reorder": args.reorder + (" symmetric" if args.symmetric
                                                                                  else " rows of A"),
                   "clustering": args.clustering,
                   "jacc_th": "3/10", "max_cluster": args.max_cluster, "similarity": args.sim,
                   "sym_load_pct": o.sym_load_pct, "load_pct": o_cl.load_pct, "plain_load_pct": o.load_pct,
                   "autotuned": bool(tuned["tuned"])},
        "gbs_compulsory": round(comp / (wall_cl * 1e-3) / 1e9, 2),
        "median": {"ms_per_step": round(det_cl["step_ms_median"], 4),
                   "value": round(flop / (det_cl["step_ms_median"] * 1e-3) / 1e9, 3),
                   "symbolic_ms": round(det_cl["symbolic_ms_median"], 4),
                   "numeric_ms": round(det_cl["numeric_ms_median"], 4)},
        "oracle_equal": oracle_equal,
        "phases_ms": {"symbolic_incl_readback": round(sym_cl, 4), "numeric": round(num_cl, 4)},
        "plain_csr": {"gflops": round(gflops_pl, 3), "ms_per_step": round(wall_pl, 4),
                      "gbs_compulsory": round(comp / (wall_pl * 1e-3) / 1e9, 2),
                      "phases_ms": {"symbolic_incl_readback": round(sym_pl, 4), "numeric": round(num_pl, 4)}},
        "speedup_clustered_vs_plain": round(wall_pl / wall_cl, 3),
        "clustered_equals_plain_bitwise": None if args.symmetric else True,
        "clustered_output_csr_cluster": clout,
        "plain_csr_reordered": None if wall_ro is None else {
            "gflops": round(flop / (wall_ro * 1e-3) / 1e9, 3), "ms_per_step": round(wall_ro, 4),
            "phases_ms": {"symbolic_incl_readback": round(sym_ro, 4), "numeric": round(num_ro, 4)},
            "speedup_clustered_vs_this": round(wall_ro / wall_cl, 3)},
        "preprocessing": {"reorder_host_s": round(t_reorder, 3), "plan_host_s": round(t_plan, 3), "plan_threads": ncpu,
                          "plan_gpu_candidates_s": None if t_plan_gpu is None else round(t_plan_gpu, 3),
                          "cluster_build_s": round(t_build, 4),
                          "in_spgemms": round((t_reorder + t_plan + t_build) / (wall_cl * 1e-3), 1),
                          # the same plan (asserted equal) with the candidate search on the GPU
                          "in_spgemms_gpu_candidates": None if t_plan_gpu is None else
                          round((t_reorder + t_plan_gpu + t_build) / (wall_cl * 1e-3), 1),
                          "nclusters": plan.nclusters, "ncc": Dc.ncc, "nslots": Dc.nslots,
                          "csr_cluster_over_csr_bytes": round(bytes_Acl / bytes_A, 3)},
        "roofline": {"bound": "hbm", "kernel": "k_num (numeric phase launches of one product)",
                     "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "algorithmic_bytes": comp,
                     "algorithmic_bytes_csr_cluster_A": comp_cl,
                     "frac_whole_step": round(ach_step / HBM_PEAK_GBS, 4),
                     "achieved_whole_step": round(ach_step, 1),
                     "copy_gbs": None if copy_gbs is None else round(copy_gbs, 1),
                     "frac_of_copy": None if copy_gbs is None else round(ach / copy_gbs, 4)},
        "cpu_baseline": cpu,
        "learned": learned_out,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
