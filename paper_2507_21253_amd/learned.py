"""Learned path selector and nnz predictor.

The paper leaves choosing the reordering and clustering for a matrix to
machine learning as future work (Sec. "Conclusion and Future Work"); here a
small network does it from the library's 32 structure features:

  * selector: which of four paths to run for C = A*A, the plain product and
    the paper's three clusterings --
      ``plain``     row-wise product in the given order,
      ``fixed8``    CSR_Cluster of fixed-length clusters of 8 consecutive
                    rows in the given order (Sec. "Fixed-length Clusters"),
      ``variable``  CSR_Cluster from variable-length clustering (Alg. 2,
                    threshold 3/10, at most 8 rows) in the given order,
      ``rcm_hc4``   CSR_Cluster from hierarchical clustering (Alg. 3,
                    threshold 3/10, at most 4 rows per cluster) of the rows
                    taken in reverse Cuthill-McKee order (reorder, then
                    cluster: the benchmark's method path);
    the label is the path with the least time per product once its
    preprocessing (host plan and orderings, device CSR_Cluster build) is
    spread over ``HORIZON`` = 20 products, the horizon the paper measures
    the amortization of its preprocessing against (Sec. "Evaluation",
    preprocessing overhead);
  * predictor: log(nnz(C) / products), from which output and accumulator
    sizes can be estimated before the symbolic phase
    (``capacity = products * exp(prediction) * (1 + margin)``); the exact
    symbolic phase remains the fallback and the measure of its error.

The network is trained on the GPU by the library's own forward,
back-propagation and Adam kernels (``hcsp_mlp_*``); labels are the library's
own timings on seeded synthetic matrices (``gen``).
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import (DeviceCSR, MLP_NACT, MLP_NDELTA, MLP_NPARAMS, MlpModel, Product, SIM_ROOT, cluster_build,
               features, mlp_forward, mlp_train_step, order_rcm, plan_fixed, plan_hierarchical, plan_variable)

PATHS = ("plain", "fixed8", "variable", "rcm_hc4")
HORIZON = 20
NIN, NH, NOUT = 32, 64, 5
# seeds from LARGE_FROM draw matrices of LARGE rows (the benchmark's size class)
LARGE_FROM = 20000
LARGE = (5e5, 1.1e6)
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "learned_set.npz")
MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "selector.mlp")


def _time_ms(P: Product, reps: int) -> float:
    import torch
    P.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s = torch.cuda.current_stream()
    e0.record(s)
    for _ in range(reps):
        P.run(check=False)
    e1.record(s)
    torch.cuda.synchronize()
    P.check()
    return e0.elapsed_time(e1) / reps


def label(H, reps: int = 3, threads: int = 0) -> dict:
    """Features, per-path product time (ms) and preprocessing time (s), nnz(C) and the product count."""
    import torch
    f = features(H)
    D = DeviceCSR.from_host(H)
    times, prep = {}, {}
    P = Product(D, D)
    times["plain"] = _time_ms(P, reps)
    prep["plain"] = 0.0
    nnz = int(P.info.nnz)
    del P

    def clustered(name, make_plan):
        torch.cuda.synchronize()
        t = time.perf_counter()
        Dc = cluster_build(D, make_plan())
        torch.cuda.synchronize()
        prep[name] = time.perf_counter() - t
        times[name] = _time_ms(Product(Dc, D), reps)

    clustered("fixed8", lambda: plan_fixed(H.nrows, 8))
    clustered("variable", lambda: plan_variable(H, (3, 10), 8))
    clustered("rcm_hc4", lambda: plan_hierarchical(H, (3, 10), 4, SIM_ROOT, nthreads=threads, perm_in=order_rcm(H)))
    rl = np.diff(H.rp)
    return {"features": f, "times": np.array([times[p] for p in PATHS]), "prep": np.array([prep[p] for p in PATHS]),
            "nnz": nnz, "products": int(rl[H.col].sum())}


def costs(times: np.ndarray, prep: np.ndarray) -> np.ndarray:
    """ms per product with the preprocessing spread over HORIZON products."""
    return times + prep * 1e3 / HORIZON


def targets(ds) -> tuple[np.ndarray, np.ndarray]:
    """(best path index, log compression ratio) per matrix."""
    y = np.argmin(costs(ds["times"], ds["prep"]), axis=1).astype(np.int32)
    t = np.log(np.maximum(ds["nnz"], 1) / np.maximum(ds["products"], 1)).astype(np.float32)
    return y, t


def gen(lo: int, hi: int, out: str, reps: int = 3):
    """Labels the matrices of seeds lo..hi-1 (synth.learned_problem) and writes them to ``out``."""
    import synth
    rows = {"seed": [], "name": [], "features": [], "times": [], "prep": [], "nnz": [], "products": [], "nrows": []}
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    for s in range(lo, hi):
        name, H = synth.learned_problem(s, *LARGE) if s >= LARGE_FROM else synth.learned_problem(s)
        r = label(H, reps, threads)
        for k in ("features", "times", "prep", "nnz", "products"):
            rows[k].append(r[k])
        rows["seed"].append(s)
        rows["name"].append(name)
        rows["nrows"].append(H.nrows)
        print("%d %-24s n=%7d best=%-8s %s (%.0fs)" % (s, name, H.nrows, PATHS[int(np.argmin(costs(r["times"], r["prep"])))],
                                                     " ".join("%.3f" % x for x in r["times"]), time.perf_counter() - t0),
              flush=True)
    np.savez_compressed(out, seed=np.array(rows["seed"], np.int64), name=np.array(rows["name"]),
             features=np.array(rows["features"], np.float32), times=np.array(rows["times"]),
             prep=np.array(rows["prep"]), nnz=np.array(rows["nnz"], np.int64),
             products=np.array(rows["products"], np.int64), nrows=np.array(rows["nrows"], np.int64))


def load(path: str = DATA) -> dict:
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def split(ds: dict) -> tuple[dict, dict]:
    """(training, held-out): seeds 12000..12199 of the main set and 20000..20029 of the large set are held out."""
    s = ds["seed"]
    m = ((s >= 12000) & (s < 12200)) | ((s >= LARGE_FROM) & (s < LARGE_FROM + 30))
    return {k: v[~m] for k, v in ds.items()}, {k: v[m] for k, v in ds.items()}


def init_params(seed: int) -> np.ndarray:
    """He-style initial weights (seeded), zero biases; layout W1 b1 W2 b2 W3 b3."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, np.sqrt(2 / NIN), NH * NIN), np.zeros(NH), rng.normal(0, np.sqrt(2 / NH), NH * NH),
             np.zeros(NH), rng.normal(0, np.sqrt(1 / NH), NOUT * NH), np.zeros(NOUT)]
    return np.concatenate(parts).astype(np.float32)


class Selector:
    """The network, its feature normalization, and GPU training / inference through the library."""

    def __init__(self, params: np.ndarray | None = None, mu=None, sd=None, seed: int = 1):
        self.params = init_params(seed) if params is None else np.asarray(params, np.float32)
        assert self.params.size == MLP_NPARAMS
        self.mu = np.zeros(NIN, np.float32) if mu is None else np.asarray(mu, np.float32)
        self.sd = np.ones(NIN, np.float32) if sd is None else np.asarray(sd, np.float32)

    def fit(self, F: np.ndarray, y: np.ndarray, t: np.ndarray, epochs: int = 1500, lr: float = 3e-3,
            lam: float = 1.0) -> list:
        """Full-batch Adam on the GPU; returns the loss every 100 steps."""
        import torch
        dev = torch.device("cuda")
        F = np.asarray(F, np.float32)
        self.mu = F.mean(axis=0)
        self.sd = np.maximum(F.std(axis=0), 1e-3).astype(np.float32)
        B = F.shape[0]
        P = torch.from_numpy(self.params.copy()).to(dev)
        norm = torch.from_numpy(np.concatenate([self.mu, self.sd])).to(dev)
        X = torch.from_numpy(F).to(dev)
        Y = torch.from_numpy(np.asarray(y, np.int32)).to(dev)
        T = torch.from_numpy(np.asarray(t, np.float32)).to(dev)
        Z = torch.empty(B, NOUT, dtype=torch.float32, device=dev)
        act = torch.empty(B, MLP_NACT, dtype=torch.float32, device=dev)
        delta = torch.empty(B, MLP_NDELTA, dtype=torch.float32, device=dev)
        loss = torch.empty(B, dtype=torch.float32, device=dev)
        g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=dev)
        m = torch.zeros(MLP_NPARAMS, dtype=torch.float32, device=dev)
        v = torch.zeros(MLP_NPARAMS, dtype=torch.float32, device=dev)
        hist = []
        for step in range(1, epochs + 1):
            mlp_train_step(P, norm, X, Y, T, lam, act, Z, delta, loss, g, m, v, step, lr)
            if step % 100 == 0 or step == 1:
                hist.append(float(loss.mean().item()))
        self.params = P.cpu().numpy()
        return hist

    def logits(self, F: np.ndarray) -> np.ndarray:
        import torch
        dev = torch.device("cuda")
        X = torch.from_numpy(np.asarray(F, np.float32)).to(dev)
        Z = torch.empty(X.shape[0], NOUT, dtype=torch.float32, device=dev)
        mlp_forward(torch.from_numpy(self.params).to(dev), torch.from_numpy(np.concatenate([self.mu, self.sd])).to(dev),
                    X, Z)
        return Z.cpu().numpy()

    def choose(self, F: np.ndarray) -> np.ndarray:
        return self.logits(F)[:, :len(PATHS)].argmax(axis=1)

    def log_ratio(self, F: np.ndarray) -> np.ndarray:
        return self.logits(F)[:, len(PATHS)]

    def save(self, path: str = MODEL):
        """The library's model file; the tag names the scored paths and the horizon of the labels."""
        MlpModel(self.params, np.concatenate([self.mu, self.sd]),
                 "paths %s horizon %d" % (",".join(PATHS), HORIZON)).save(path)

    @staticmethod
    def load(path: str = MODEL) -> "Selector":
        params, norm, tag = MlpModel.load(path).get()
        fields = tag.split()
        if len(fields) < 2 or fields[0] != "paths" or fields[1] != ",".join(PATHS):
            raise ValueError("%s scores paths %r, this module %r" % (path, tag, ",".join(PATHS)))
        return Selector(params, norm[:NIN], norm[NIN:])


def evaluate(sel: Selector, ds: dict) -> dict:
    """Per-product cost (ms, preprocessing spread over HORIZON) of the selector's choices on ``ds`` against
    fixed policies and the per-matrix best; prediction error of the log compression ratio."""
    c = costs(ds["times"], ds["prep"])
    y, t = targets(ds)
    pick = sel.choose(ds["features"])
    idx = np.arange(len(y))
    out = {"matrices": int(len(y)), "selector_ms": float(c[idx, pick].sum()), "best_ms": float(c.min(axis=1).sum()),
           "accuracy": float(np.mean(pick == y))}
    for k, p in enumerate(PATHS):
        out["always_%s_ms" % p] = float(c[:, k].sum())
    err = np.abs(sel.log_ratio(ds["features"]) - t)
    out["log_ratio_abs_err_median"] = float(np.median(err))
    out["log_ratio_abs_err_p90"] = float(np.quantile(err, 0.9))
    out["label_counts"] = {p: int(np.sum(y == k)) for k, p in enumerate(PATHS)}
    return out


def main():
    import argparse
    p = argparse.ArgumentParser(description="data set, training and evaluation of the learned path selector")
    sub = p.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("gen")
    g.add_argument("--lo", type=int, required=True)
    g.add_argument("--hi", type=int, required=True)
    g.add_argument("--out", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--data", nargs="+", default=[DATA])
    tr.add_argument("--out", default=MODEL)
    tr.add_argument("--epochs", type=int, default=1500)
    a = p.parse_args()
    if a.cmd == "gen":
        gen(a.lo, a.hi, a.out)
        return
    parts = [load(f) for f in a.data]
    ds = {k: np.concatenate([d[k] for d in parts]) for k in parts[0]}
    train, held = split(ds)
    y, t = targets(train)
    sel = Selector(seed=1)
    hist = sel.fit(train["features"], y, t, a.epochs)
    sel.save(a.out)
    print(json.dumps({"loss": hist[::3], "train": evaluate(sel, train), "held_out": evaluate(sel, held)}), flush=True)


if __name__ == "__main__":
    main()
