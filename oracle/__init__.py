"""CPU oracle for clustered SpGEMM — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg
may import this package.  The GPU library never loads it and shares no code
with it; the product path fails loudly when its own HIP library is missing
instead of falling back to anything here.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc and
``-ffp-contract=off`` into ``liboracle.so``); this file only marshals numpy
arrays.  Each wrapper names the paper passage its C function follows:

* ``spgemm`` / ``spgemm_mt`` / ``rowstats`` — Gustavson row-wise product
  (Background, "SpGEMM Kernel", Fig. 1): ascending-k fused multiply-add per
  output entry starting from +0.0, sorted output columns, numeric zeros kept.
* ``dense_product`` — brute-force dense triple loop (pin for the above).
* ``jaccard`` — row similarity (Variable-length Clusters).
* ``plan_fixed`` / ``plan_variable`` / ``plan_hierarchical`` / ``topk_candidates``
  — the three clustering schemes (Fixed-length Clusters, Alg. 2, Alg. 3).
* ``cluster_build`` — the CSR_Cluster layout (Access Pattern and Matrix Format).
* ``cluster_spgemm`` — the cluster-wise product (Alg. 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from synth import HostCSR

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

SIM_ROOT = 0
SIM_UNION = 1


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (host C only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        # HCSP_ORACLE_LIB: a build of a modified oracle.c, loaded instead (the
        # mutation test plants one mistake at a time and expects a pin to fail)
        alt = os.environ.get("HCSP_ORACLE_LIB")
        if not alt and not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(alt or _SO)
        i64, i32, u32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p
        lib.orc_spgemm.argtypes = [i64, vp, vp, vp, vp, vp, vp, i64, i64, vp, vp, vp, i64]
        lib.orc_spgemm.restype = i64
        lib.orc_spgemm_mt.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, ctypes.c_int]
        lib.orc_spgemm_mt.restype = i64
        lib.orc_spgemm_rowstats.argtypes = [i64, vp, vp, vp, vp, vp, vp, i64, i64, vp, vp, vp, ctypes.c_int]
        lib.orc_spgemm_rowstats.restype = ctypes.c_int
        lib.orc_spgemm_count.argtypes = [i64, vp, vp, vp, vp, i64, i64, vp, ctypes.c_int]
        lib.orc_spgemm_count.restype = ctypes.c_int
        lib.orc_hash_cols.argtypes = [vp, i64]
        lib.orc_hash_cols.restype = ctypes.c_uint64
        lib.orc_dense_product.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp, vp]
        lib.orc_dense_product.restype = ctypes.c_int
        lib.orc_jaccard.argtypes = [vp, vp, i64, i64, vp, vp]
        lib.orc_jaccard.restype = None
        lib.orc_plan_fixed.argtypes = [i64, i32, vp, vp, vp]
        lib.orc_plan_fixed.restype = i64
        lib.orc_plan_variable.argtypes = [i64, vp, vp, i64, i64, i32, vp, vp, vp]
        lib.orc_plan_variable.restype = i64
        lib.orc_topk_candidates.argtypes = [i64, i64, vp, vp, i64, i64, i32, vp, vp, vp, vp, vp]
        lib.orc_topk_candidates.restype = ctypes.c_int
        lib.orc_plan_hierarchical.argtypes = [i64, i64, vp, vp, i64, i64, i32, u32, vp, vp, vp]
        lib.orc_plan_hierarchical.restype = i64
        lib.orc_cluster_count.argtypes = [i64, vp, vp, vp, vp, vp, vp]
        lib.orc_cluster_count.restype = ctypes.c_int
        lib.orc_cluster_fill.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.orc_cluster_fill.restype = ctypes.c_int
        lib.orc_cluster_spgemm.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i64]
        lib.orc_cluster_spgemm.restype = i64
        lib.orc_order_rcm.argtypes = [i64, vp, vp, vp]
        lib.orc_order_rcm.restype = ctypes.c_int
        lib.orc_order_degree.argtypes = [i64, vp, vp]
        lib.orc_order_degree.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _ratio(t) -> tuple[int, int]:
    f = Fraction(t).limit_denominator(1 << 20) if not isinstance(t, tuple) else Fraction(*t)
    return f.numerator, f.denominator


# ------------------------------------------------------------------ products

def spgemm(A: HostCSR, B: HostCSR, rows: tuple[int, int] | None = None) -> HostCSR:
    """C = A*B (Gustavson, Fig. 1) over rows ``rows`` of A (default: all)."""
    lo, hi = rows if rows else (0, A.nrows)
    lib = _load()
    rp = np.empty(hi - lo + 1, np.int64)
    nnz = lib.orc_spgemm(B.ncols, _p(A.rp), _p(A.col), _p(A.val), _p(B.rp), _p(B.col), _p(B.val),
                         lo, hi, _p(rp), None, None, 0)
    if nnz < 0:
        raise RuntimeError("orc_spgemm count failed (%d)" % nnz)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    nnz2 = lib.orc_spgemm(B.ncols, _p(A.rp), _p(A.col), _p(A.val), _p(B.rp), _p(B.col), _p(B.val),
                          lo, hi, _p(rp), _p(col), _p(val), nnz)
    if nnz2 != nnz:
        raise RuntimeError("orc_spgemm fill failed (%d)" % nnz2)
    return HostCSR(rp, col, val, hi - lo, B.ncols)


def spgemm_mt(A: HostCSR, B: HostCSR, nthreads: int, structure_only: bool = False) -> HostCSR:
    """The same product on ``nthreads`` host threads (contiguous row ranges)."""
    lib = _load()
    rp = np.zeros(A.nrows + 1, np.int64)
    if structure_only:
        nnz = lib.orc_spgemm_mt(A.nrows, B.ncols, _p(A.rp), _p(A.col), _p(A.val), _p(B.rp), _p(B.col),
                                _p(B.val), _p(rp), None, None, 0, nthreads)
        if nnz < 0:
            raise RuntimeError("orc_spgemm_mt failed")
        return HostCSR(rp, np.empty(0, np.int32), np.empty(0), A.nrows, B.ncols)
    nnz = lib.orc_spgemm_mt(A.nrows, B.ncols, _p(A.rp), _p(A.col), _p(A.val), _p(B.rp), _p(B.col),
                            _p(B.val), _p(rp), None, None, 0, nthreads)
    if nnz < 0:
        raise RuntimeError("orc_spgemm_mt count failed")
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    rp[:] = 0
    nnz2 = lib.orc_spgemm_mt(A.nrows, B.ncols, _p(A.rp), _p(A.col), _p(A.val), _p(B.rp), _p(B.col),
                             _p(B.val), _p(rp), _p(col), _p(val), nnz, nthreads)
    if nnz2 != nnz:
        raise RuntimeError("orc_spgemm_mt fill failed")
    return HostCSR(rp, col, val, A.nrows, B.ncols)


def spgemm_count(A: HostCSR, B: HostCSR, nthreads: int = 1, rows: tuple[int, int] | None = None) -> np.ndarray:
    """Row counts of C = A*B (the structure: distinct columns per row) over rows ``rows`` of A (default all),
    on ``nthreads`` host threads, without forming C."""
    lo, hi = rows if rows else (0, A.nrows)
    out = np.zeros(A.nrows, np.int64)
    if _load().orc_spgemm_count(B.ncols, _p(A.rp), _p(A.col), _p(B.rp), _p(B.col), lo, hi, _p(out), nthreads):
        raise RuntimeError("orc_spgemm_count failed")
    return out[lo:hi]


def rowstats(A: HostCSR, B: HostCSR, rows: np.ndarray | tuple[int, int], nthreads: int = 1):
    """Per-row (nnz, FNV-1a hash of sorted columns, value sum in column order) of C = A*B without
    storing C.  ``rows`` is a (lo, hi) range or an array of row ids."""
    lib = _load()
    if isinstance(rows, tuple):
        lo, hi = rows
        nnz = np.zeros(A.nrows, np.int64)
        h = np.zeros(A.nrows, np.uint64)
        s = np.zeros(A.nrows, np.float64)
        rc = lib.orc_spgemm_rowstats(B.ncols, _p(A.rp), _p(A.col), _p(A.val), _p(B.rp), _p(B.col),
                                     _p(B.val), lo, hi, _p(nnz), _p(h), _p(s), nthreads)
        if rc:
            raise RuntimeError("rowstats failed")
        return nnz[lo:hi], h[lo:hi], s[lo:hi]
    rows = np.asarray(rows, np.int64)
    out_n, out_h, out_s = [], [], []
    for r in rows:
        C = spgemm(A, B, (int(r), int(r) + 1))
        out_n.append(C.nnz)
        out_h.append(hash_cols(C.col))
        out_s.append(float(np.sum(C.val)) if C.nnz else 0.0)
    return np.array(out_n, np.int64), np.array(out_h, np.uint64), np.array(out_s)


def hash_cols(cols: np.ndarray) -> int:
    c = np.ascontiguousarray(cols, np.int32)
    return int(_load().orc_hash_cols(_p(c), len(c)))


def dense_product(A: np.ndarray, Ap: np.ndarray, B: np.ndarray, Bp: np.ndarray):
    """Brute-force dense C, presence(C) with ascending-k fused multiply-add chains."""
    A = np.ascontiguousarray(A, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    Ap = np.ascontiguousarray(Ap, np.uint8)
    Bp = np.ascontiguousarray(Bp, np.uint8)
    n, m = A.shape
    p = B.shape[1]
    C = np.empty((n, p))
    Cp = np.empty((n, p), np.uint8)
    _load().orc_dense_product(n, m, p, _p(A), _p(Ap), _p(B), _p(Bp), _p(C), _p(Cp))
    return C, Cp.astype(bool)


# ------------------------------------------------------------------ similarity and plans

def jaccard(A: HostCSR, i: int, j: int) -> tuple[int, int]:
    """(|Si n Sj|, |Si u Sj|) of rows i and j."""
    ov = ctypes.c_int64()
    un = ctypes.c_int64()
    _load().orc_jaccard(_p(A.rp), _p(A.col), i, j, ctypes.byref(ov), ctypes.byref(un))
    return ov.value, un.value


@dataclass
class Plan:
    """Clusters as consecutive ranges of ``perm``: cluster c holds original rows
    perm[cl_row_ptr[c]:cl_row_ptr[c+1]]."""

    perm: np.ndarray
    cl_row_ptr: np.ndarray

    @property
    def nclusters(self) -> int:
        return len(self.cl_row_ptr) - 1

    def clusters(self):
        return [self.perm[self.cl_row_ptr[c]:self.cl_row_ptr[c + 1]].tolist() for c in range(self.nclusters)]


def _perm_in(perm_in, n):
    return None if perm_in is None else np.ascontiguousarray(perm_in, np.int32)


def plan_fixed(n: int, K: int, perm_in=None) -> Plan:
    pi = _perm_in(perm_in, n)
    perm = np.empty(n, np.int32)
    crp = np.empty(n + 1, np.int64)
    c = _load().orc_plan_fixed(n, K, _p(pi), _p(perm), _p(crp))
    if c < 0:
        raise ValueError("bad fixed plan arguments")
    return Plan(perm, crp[:c + 1].copy())


def plan_variable(A: HostCSR, jacc_th=(3, 10), max_cluster: int = 8, perm_in=None) -> Plan:
    num, den = _ratio(jacc_th)
    pi = _perm_in(perm_in, A.nrows)
    perm = np.empty(A.nrows, np.int32)
    crp = np.empty(A.nrows + 1, np.int64)
    c = _load().orc_plan_variable(A.nrows, _p(A.rp), _p(A.col), num, den, max_cluster, _p(pi), _p(perm), _p(crp))
    if c < 0:
        raise ValueError("bad variable plan arguments")
    return Plan(perm, crp[:c + 1].copy())


def topk_candidates(A: HostCSR, jacc_th=(3, 10), topk: int = 7, perm_in=None):
    """Per-row top-k partners of SpGEMM_TopK: (cnt[n], nbr[n,topk], ov[n,topk], un[n,topk])."""
    num, den = _ratio(jacc_th)
    n = A.nrows
    pi = _perm_in(perm_in, n)
    cnt = np.zeros(n, np.int32)
    nbr = np.full((n, topk), -1, np.int32)
    ov = np.zeros((n, topk), np.int64)
    un = np.zeros((n, topk), np.int64)
    rc = _load().orc_topk_candidates(n, A.ncols, _p(A.rp), _p(A.col), num, den, topk, _p(pi), _p(cnt),
                                     _p(nbr), _p(ov), _p(un))
    if rc:
        raise RuntimeError("topk failed")
    return cnt, nbr, ov, un


def plan_hierarchical(A: HostCSR, jacc_th=(3, 10), max_cluster: int = 8, flags: int = SIM_ROOT,
                      perm_in=None) -> Plan:
    num, den = _ratio(jacc_th)
    pi = _perm_in(perm_in, A.nrows)
    perm = np.empty(A.nrows, np.int32)
    crp = np.empty(A.nrows + 1, np.int64)
    c = _load().orc_plan_hierarchical(A.nrows, A.ncols, _p(A.rp), _p(A.col), num, den, max_cluster, flags,
                                      _p(pi), _p(perm), _p(crp))
    if c < 0:
        raise ValueError("hierarchical plan failed")
    return Plan(perm, crp[:c + 1].copy())


# ------------------------------------------------------------------ CSR_Cluster

@dataclass
class HostCluster:
    """CSR_Cluster in host memory (see ``orc_cluster_count`` for the layout)."""

    nrows: int
    ncols: int
    perm: np.ndarray
    cl_row_ptr: np.ndarray
    cl_col_ptr: np.ndarray
    cl_col: np.ndarray
    cl_mask: np.ndarray
    cl_val_ptr: np.ndarray
    cl_val: np.ndarray

    @property
    def nclusters(self) -> int:
        return len(self.cl_row_ptr) - 1

    def bytes(self) -> int:
        """Footprint: offsets (8 B each), perm (4 B/row), 4+2 B per union column, 8 B per slot."""
        ncl = self.nclusters
        return 8 * 3 * (ncl + 1) + 4 * self.nrows + 6 * len(self.cl_col) + 8 * len(self.cl_val)


def cluster_build(A: HostCSR, plan: Plan) -> HostCluster:
    lib = _load()
    ncl = plan.nclusters
    perm = np.ascontiguousarray(plan.perm, np.int32)
    crp = np.ascontiguousarray(plan.cl_row_ptr, np.int64)
    ccp = np.empty(ncl + 1, np.int64)
    cvp = np.empty(ncl + 1, np.int64)
    if lib.orc_cluster_count(ncl, _p(A.rp), _p(A.col), _p(perm), _p(crp), _p(ccp), _p(cvp)):
        raise ValueError("cluster sizes must be 1..16")
    cl_col = np.empty(int(ccp[-1]), np.int32)
    cl_mask = np.empty(int(ccp[-1]), np.uint16)
    cl_val = np.empty(int(cvp[-1]), np.float64)
    if lib.orc_cluster_fill(ncl, _p(A.rp), _p(A.col), _p(A.val), _p(perm), _p(crp), _p(ccp), _p(cvp),
                            _p(cl_col), _p(cl_mask), _p(cl_val)):
        raise RuntimeError("cluster fill failed")
    return HostCluster(A.nrows, A.ncols, perm, crp, ccp, cl_col, cl_mask, cvp, cl_val)


def cluster_spgemm(Ac: HostCluster, B: HostCSR) -> HostCSR:
    """Alg. 1 over a CSR_Cluster operand; C in A's original row order."""
    lib = _load()
    rp = np.zeros(Ac.nrows + 1, np.int64)
    args = (Ac.nrows, B.ncols, Ac.nclusters, _p(Ac.cl_row_ptr), _p(Ac.perm), _p(Ac.cl_col_ptr), _p(Ac.cl_col),
            _p(Ac.cl_mask), _p(Ac.cl_val_ptr), _p(Ac.cl_val), _p(B.rp), _p(B.col), _p(B.val))
    nnz = lib.orc_cluster_spgemm(*args, _p(rp), None, None, 0)
    if nnz < 0:
        raise RuntimeError("cluster_spgemm count failed")
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    rp[:] = 0
    nnz2 = lib.orc_cluster_spgemm(*args, _p(rp), _p(col), _p(val), nnz)
    if nnz2 != nnz:
        raise RuntimeError("cluster_spgemm fill failed")
    return HostCSR(rp, col, val, Ac.nrows, B.ncols)


def order_rcm(A: HostCSR) -> np.ndarray:
    """Reverse Cuthill-McKee order of the pattern of A + A^T (Sec. "Matrix Reordering"); perm[p] is the row
    placed at position p."""
    perm = np.empty(max(A.nrows, 1), np.int32)
    if A.nrows and _load().orc_order_rcm(A.nrows, _p(A.rp), _p(A.col), _p(perm)):
        raise RuntimeError("orc_order_rcm failed")
    return perm[:A.nrows]


def order_degree(A: HostCSR) -> np.ndarray:
    """Rows by descending length, ties by ascending id (Sec. "Matrix Reordering", degree order)."""
    perm = np.empty(max(A.nrows, 1), np.int32)
    if A.nrows and _load().orc_order_degree(A.nrows, _p(A.rp), _p(perm)):
        raise RuntimeError("orc_order_degree failed")
    return perm[:A.nrows]
