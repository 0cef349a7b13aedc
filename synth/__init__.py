"""Seeded synthetic input matrices, shared by the oracle tests and the GPU tests.

This module only makes inputs.  It contains none of the SpGEMM method's
arithmetic; the generators themselves live in ``synth.c`` (compiled with gcc
into ``libsynth.so`` next to this file) and every random draw comes from a
counter-based SplitMix64 stream keyed by (seed, purpose).

Workload recipes follow the shapes the paper evaluates on (square matrices
squared, Evaluation/Datasets and Workloads): uniform-random rows, 2D/3D
stencils (optionally symmetrically relabelled to destroy locality) and R-MAT
power-law graphs, plus the batch and training-set mixes built from them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libsynth.so`` with gcc (plain C, no GPU code)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        i64, i32, u64, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
        lib.synth_u64.argtypes = [u64, u64]
        lib.synth_u64.restype = u64
        lib.synth_key.argtypes = [u64, u64]
        lib.synth_key.restype = u64
        lib.synth_u01.argtypes = [u64, u64]
        lib.synth_u01.restype = dbl
        lib.synth_uniform.argtypes = [i64, i64, i32, u64, vp, vp, vp]
        lib.synth_uniform.restype = ctypes.c_int
        lib.synth_stencil_nnz.argtypes = [ctypes.c_int, i64]
        lib.synth_stencil_nnz.restype = i64
        lib.synth_stencil.argtypes = [ctypes.c_int, i64, u64, vp, vp, vp]
        lib.synth_stencil.restype = ctypes.c_int
        lib.synth_perm.argtypes = [i64, u64, vp]
        lib.synth_perm.restype = ctypes.c_int
        lib.synth_relabel.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.synth_relabel.restype = ctypes.c_int
        lib.synth_rmat.argtypes = [ctypes.c_int, i64, dbl, dbl, dbl, u64, vp, vp, i64]
        lib.synth_rmat.restype = i64
        lib.synth_frontiers.argtypes = [i64, vp, vp, i32, i32, u64, vp, vp, vp, i64]
        lib.synth_frontiers.restype = i64
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class HostCSR:
    """A CSR matrix in host memory: int64 row offsets, int32 sorted columns, float64 values."""

    rp: np.ndarray
    col: np.ndarray
    val: np.ndarray
    nrows: int
    ncols: int

    @property
    def nnz(self) -> int:
        return int(self.rp[-1]) if len(self.rp) else 0

    def row(self, i: int):
        b, e = int(self.rp[i]), int(self.rp[i + 1])
        return self.col[b:e], self.val[b:e]

    def bytes(self) -> int:
        """CSR footprint: 8 B per row offset plus 12 B per stored entry."""
        return 8 * (self.nrows + 1) + 12 * self.nnz


def u64(key: int, n: int) -> int:
    return int(_load().synth_u64(key, n))


def key(seed: int, tag: int) -> int:
    return int(_load().synth_key(seed, tag))


def u01(k: int, n: int) -> float:
    return float(_load().synth_u01(k, n))


def uniform(nrows: int, ncols: int, d: int, seed: int) -> HostCSR:
    """Exactly ``d`` distinct uniform-random columns per row (Floyd sampling), values U(-1,1)."""
    rp = np.empty(nrows + 1, np.int64)
    col = np.empty(nrows * d, np.int32)
    val = np.empty(nrows * d, np.float64)
    if _load().synth_uniform(nrows, ncols, d, seed, _p(rp), _p(col), _p(val)) != 0:
        raise ValueError("bad uniform() sizes")
    return HostCSR(rp, col, val, nrows, ncols)


def stencil(kind: int, m: int, seed: int) -> HostCSR:
    """2D 5-point (kind 5), 3D 7-point (7) or 3D 27-point (27) stencil on an m-grid, x fastest."""
    lib = _load()
    nnz = int(lib.synth_stencil_nnz(kind, m))
    if nnz < 0:
        raise ValueError("bad stencil kind/size")
    n = m * m if kind == 5 else m * m * m
    rp = np.empty(n + 1, np.int64)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    if lib.synth_stencil(kind, m, seed, _p(rp), _p(col), _p(val)) != 0:
        raise ValueError("stencil generation failed")
    return HostCSR(rp, col, val, n, n)


def perm(n: int, seed: int) -> np.ndarray:
    """Seeded uniform permutation of range(n) (Fisher-Yates)."""
    p = np.empty(n, np.int32)
    if _load().synth_perm(n, seed, _p(p)) != 0:
        raise ValueError("bad perm size")
    return p


def relabel(A: HostCSR, rmap: np.ndarray, cmap: np.ndarray | None) -> HostCSR:
    """Row ``u`` of A becomes row ``rmap[u]``; columns map through ``cmap`` (None keeps them)."""
    rmap = np.ascontiguousarray(rmap, np.int32)
    rp2 = np.empty_like(A.rp)
    col2 = np.empty_like(A.col)
    val2 = np.empty_like(A.val)
    cm = None
    if cmap is not None:
        cm = np.ascontiguousarray(cmap, np.int32)
    rc = _load().synth_relabel(A.nrows, _p(A.rp), _p(A.col), _p(A.val), _p(rmap),
                               _p(cm) if cm is not None else None, _p(rp2), _p(col2), _p(val2))
    if rc != 0:
        raise RuntimeError("relabel failed")
    ncols = A.ncols
    return HostCSR(rp2, col2, val2, A.nrows, ncols)


def symmetric_relabel(A: HostCSR, seed: int) -> tuple[HostCSR, np.ndarray]:
    """M = Q A Q^T for a seeded permutation q (old index v -> new index q[v]); returns (M, q)."""
    if A.nrows != A.ncols:
        raise ValueError("symmetric relabel needs a square matrix")
    q = perm(A.nrows, seed)
    return relabel(A, q, q), q


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 4) -> HostCSR:
    """R-MAT graph, self-loops dropped, symmetrised, de-duplicated, all values 1.0."""
    n = 1 << scale
    nedges = edge_factor * n
    rp = np.empty(n + 1, np.int64)
    cap = 2 * nedges
    col = np.empty(cap, np.int32)
    nnz = int(_load().synth_rmat(scale, nedges, a, b, c, seed, _p(rp), _p(col), cap))
    if nnz < 0:
        raise RuntimeError("rmat generation failed (%d)" % nnz)
    col = col[:nnz].copy()
    return HostCSR(rp, col, np.ones(nnz, np.float64), n, n)


def frontiers(A: HostCSR, nsrc: int, level: int, seed: int) -> HostCSR:
    """Multi-source BFS frontier matrix (n x nsrc) of the square graph A: column s holds the vertices at
    distance exactly ``level`` from source s (sources: a seeded sample of the vertices), values U(-1,1)."""
    n = A.nrows
    rp_a = np.ascontiguousarray(A.rp, np.int64)
    col_a = np.ascontiguousarray(A.col, np.int32)
    rp = np.empty(n + 1, np.int64)
    cap = max(1 << 20, 4 * nsrc)
    while True:
        col = np.empty(cap, np.int32)
        val = np.empty(cap, np.float64)
        nnz = int(_load().synth_frontiers(n, _p(rp_a), _p(col_a), nsrc, level, seed, _p(rp), _p(col), _p(val), cap))
        if nnz == -2:
            cap *= 4
            continue
        if nnz < 0:
            raise ValueError("bad frontiers() arguments")
        return HostCSR(rp, col[:nnz].copy(), val[:nnz].copy(), n, nsrc)


def identity(n: int) -> HostCSR:
    return HostCSR(np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.ones(n), n, n)


def from_dense(D: np.ndarray, pattern: np.ndarray | None = None) -> HostCSR:
    """CSR of a dense array; ``pattern`` (bool) marks stored entries, default D != 0."""
    D = np.asarray(D, np.float64)
    pat = (D != 0) if pattern is None else np.asarray(pattern, bool)
    rows, cols = np.nonzero(pat)
    rp = np.zeros(D.shape[0] + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int64)
    return HostCSR(rp, cols.astype(np.int32), D[rows, cols].astype(np.float64), D.shape[0], D.shape[1])


def to_dense(A: HostCSR) -> tuple[np.ndarray, np.ndarray]:
    """(values, pattern) dense arrays of a CSR matrix."""
    D = np.zeros((A.nrows, A.ncols))
    P = np.zeros((A.nrows, A.ncols), bool)
    rows = np.repeat(np.arange(A.nrows), np.diff(A.rp))
    D[rows, A.col] = A.val
    P[rows, A.col] = True
    return D, P


# ---------------------------------------------------------------- workload recipes

def workload_uniform_2000(seed: int = 1) -> HostCSR:
    """2,000 x 2,000, exactly 10 distinct uniform-random columns per row, U(-1,1)."""
    return uniform(2000, 2000, 10, seed)


def workload_stencil27(m: int = 100, seed: int = 2, relabel_seed: int | None = 3):
    """27-point stencil on m^3 (values seed ``seed``); with ``relabel_seed`` it is symmetrically
    relabelled by a seeded permutation.  Returns (M, S, q) where S is natural order."""
    S = stencil(27, m, seed)
    if relabel_seed is None:
        return S, S, np.arange(S.nrows, dtype=np.int32)
    M, q = symmetric_relabel(S, relabel_seed)
    return M, S, q


def workload_rmat(scale: int = 20, seed: int = 4) -> HostCSR:
    return rmat(scale, 16, 0.57, 0.19, 0.19, seed)


def batch_problem(seed: int, n_lo: float = 1e3, n_hi: float = 2e5) -> tuple[str, HostCSR]:
    """One matrix of the uneven batch mix: 2D 5-point, 3D 7-point or uniform-random (4..32 per row),
    size log-uniform in [n_lo, n_hi] rows, values U(-1,1)."""
    k = key(seed, 77)
    kind = int(u64(k, 0) % 3)
    n = int(round(math.exp(math.log(n_lo) + u01(k, 1) * (math.log(n_hi) - math.log(n_lo)))))
    if kind == 0:
        side = max(2, int(round(math.sqrt(n))))
        return "stencil5", stencil(5, side, seed)
    if kind == 1:
        side = max(2, int(round(n ** (1.0 / 3.0))))
        return "stencil7", stencil(7, side, seed)
    d = 4 + int(u64(k, 2) % 29)
    n = max(n, d)
    return "uniform", uniform(n, n, d, seed)


def learned_problem(seed: int, n_lo: float = 1e4, n_hi: float = 5e5) -> tuple[str, HostCSR]:
    """One matrix of the learned selector's data set: the generators above (2-D 5-point, 3-D 7-point and
    27-point stencils, uniform-random with 4..32 entries per row, R-MAT of scale 12..14 with edge factor
    8..16), size log-uniform in [n_lo, n_hi] rows, and in half of the cases a seeded symmetric relabelling
    (natural order destroyed).  Returns (name, M)."""
    k = key(seed, 91)
    kind = int(u64(k, 0) % 5)
    n = int(round(math.exp(math.log(n_lo) + u01(k, 1) * (math.log(n_hi) - math.log(n_lo)))))
    if kind == 0:
        name, A = "stencil5", stencil(5, max(2, int(round(math.sqrt(n)))), seed)
    elif kind == 1:
        name, A = "stencil7", stencil(7, max(2, int(round(n ** (1 / 3)))), seed)
    elif kind == 2:
        name, A = "stencil27", stencil(27, max(2, int(round((n / 2) ** (1 / 3)))), seed)
    elif kind == 3:
        d = 4 + int(u64(k, 2) % 29)
        name, A = "uniform%d" % d, uniform(n, n, d, seed)
    else:
        sc = 12 + int(u64(k, 3) % 3)
        ef = 8 + int(u64(k, 4) % 9)
        name, A = "rmat%d_%d" % (sc, ef), rmat(sc, ef, 0.57, 0.19, 0.19, seed)
    if u64(k, 5) & 1:
        A, _ = symmetric_relabel(A, seed + 1)
        name += "_relabelled"
    return name, A
