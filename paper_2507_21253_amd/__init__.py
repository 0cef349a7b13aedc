"""hcsp — clustered Gustavson SpGEMM for AMD Instinct MI355X (gfx950).

Thin Python binding over the C ABI of ``libhcsp.so`` (declared in
``include/hcsp.h``).  The functions below carry the C names without the
``hcsp_`` prefix and only marshal arguments: torch tensors supply device
memory and the current HIP stream, numpy arrays supply host memory for the
cluster plans.  Every step of the product runs in the library's own kernels;
there is no Python or CPU fallback, and a missing library raises.

Paper: "Improving SpGEMM Performance Through Matrix Reordering and
Cluster-wise Computation" (arXiv 2507.21253): row-wise Gustavson SpGEMM over
CSR and over the row-clustered CSR_Cluster format (Alg. 1), with clusters
from fixed-length, variable-length (Alg. 2) or hierarchical (Alg. 3)
clustering.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhcsp.so")

HCSP_OK = 0
STATUS = {0: "OK", -1: "E_INVALID", -2: "E_PTR", -3: "E_RANGE", -4: "E_UNSORTED", -5: "E_CAPACITY",
          -6: "E_HIP", -7: "E_NOMEM", -8: "E_UNSUPPORTED", -9: "E_OVERFLOW"}
OP_CSR, OP_CLUSTER = 0, 1
SIM_ROOT, SIM_UNION = 0, 1
F_SYNC_CHECK = 1
F_ONE_STREAM = 2
MAX_BINS = 96

i64, i32, u32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p


class c_csr(ctypes.Structure):
    _fields_ = [("nrows", i64), ("ncols", i64), ("nnz", i64), ("row_ptr", vp), ("col", vp), ("val", vp)]


class c_csr_cluster(ctypes.Structure):
    _fields_ = [("nrows", i64), ("ncols", i64), ("nclusters", i64), ("ncc", i64), ("nslots", i64),
                ("max_cluster", i32), ("reserved", i32), ("cl_row_ptr", vp), ("perm", vp), ("cl_col_ptr", vp),
                ("cl_col", vp), ("cl_mask", vp), ("cl_val_ptr", vp), ("cl_val", vp)]


class c_operand(ctypes.Structure):
    _fields_ = [("kind", i32), ("reserved", i32), ("csr", c_csr), ("cl", c_csr_cluster)]


class c_ratio(ctypes.Structure):
    _fields_ = [("num", i32), ("den", i32)]


class c_opts(ctypes.Structure):
    _fields_ = [("lanes", i32), ("flags", i32), ("unit_lo", i64), ("unit_hi", i64), ("out_base", i64),
                ("dense_slots", i32), ("load_pct", i32), ("sym_tmax_log2", i32), ("num_tmax", i32),
                ("sym_load_pct", i32), ("win_chunk_log2", i32)]


class c_sym_info(ctypes.Structure):
    _fields_ = [("nnz", i64), ("units", i64), ("sym_bin_count", i64 * MAX_BINS),
                ("num_bin_count", i64 * MAX_BINS), ("lanes", i32), ("valid", i32), ("load_pct", i32),
                ("win_chunk_log2", i32)]


class c_batch_item(ctypes.Structure):
    _fields_ = [("A", c_operand), ("B", c_csr)]


class c_batch_plan(ctypes.Structure):
    _fields_ = [("count", i32), ("kind", i32), ("units", i64), ("rows", i64), ("row_ptr_len", i64),
                ("max_ncols", i64), ("max_class", i32), ("prepared", i32), ("max_probes", i64),
                ("out_capacity", i64), ("ws_bytes", ctypes.c_size_t), ("opts", c_opts)]


TUNE_NSYM, TUNE_NNUM, TUNE_NMC, TUNE_NCL = 3, 3, 3, 6
TUNE_SYM_FILLS = (50, 70, 100)
TUNE_NUM_FILLS = (50, 60, 70)
TUNE_CLUSTER_SIZES = (2, 4, 8)
TUNE_CL_FILLS = (50, 60, 70, 75, 80, 85)


class c_tune_run(ctypes.Structure):
    _fields_ = [("nrows", i64), ("nnz", i64), ("plain_ms", (ctypes.c_double * TUNE_NNUM) * TUNE_NSYM),
                ("rcm_ms", ctypes.c_double), ("hc_ms", (ctypes.c_double * TUNE_NCL) * TUNE_NMC)]


class c_tune_choice(ctypes.Structure):
    _fields_ = [("tuned", i32), ("path", i32), ("max_cluster", i32), ("best_cluster_size", i32),
                ("sym_load_pct", i32), ("load_pct", i32), ("cl_load_pct", i32), ("runs", i32)]


# every symbol include/hcsp.h declares, with its ctypes signature
_SIGS = {
    "hcsp_version": ([], ctypes.c_char_p),
    "hcsp_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "hcsp_last_error": ([], ctypes.c_char_p),
    "hcsp_csr_check": ([ctypes.POINTER(c_csr), vp, ctypes.c_size_t, vp], ctypes.c_int),
    "hcsp_plan_fixed": ([i64, i32, vp, vp, vp, ctypes.POINTER(i64)], ctypes.c_int),
    "hcsp_plan_variable": ([ctypes.POINTER(c_csr), c_ratio, i32, vp, vp, vp, ctypes.POINTER(i64)], ctypes.c_int),
    "hcsp_plan_hierarchical": ([ctypes.POINTER(c_csr), c_ratio, i32, u32, i32, vp, vp, vp, ctypes.POINTER(i64)],
                               ctypes.c_int),
    "hcsp_plan_hierarchical_candidates": ([ctypes.POINTER(c_csr), c_ratio, i32, u32, vp, vp, vp, vp, vp, vp,
                                          ctypes.POINTER(i64)], ctypes.c_int),
    "hcsp_topk_candidates": ([ctypes.POINTER(c_csr), vp, vp, c_ratio, i32, vp, vp, vp, vp], ctypes.c_int),
    "hcsp_cluster_workspace": ([i64, i64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hcsp_cluster_count": ([ctypes.POINTER(c_csr), vp, vp, i64, vp, vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                            ctypes.POINTER(i32), vp, ctypes.c_size_t, vp], ctypes.c_int),
    "hcsp_cluster_fill": ([ctypes.POINTER(c_csr), ctypes.POINTER(c_csr_cluster), vp], ctypes.c_int),
    "hcsp_spgemm_workspace": ([ctypes.POINTER(c_operand), ctypes.POINTER(c_csr), ctypes.POINTER(c_opts),
                               ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hcsp_spgemm_symbolic": ([ctypes.POINTER(c_operand), ctypes.POINTER(c_csr), ctypes.POINTER(c_opts), vp,
                              ctypes.POINTER(c_sym_info), vp, ctypes.c_size_t, vp], ctypes.c_int),
    "hcsp_spgemm_numeric": ([ctypes.POINTER(c_operand), ctypes.POINTER(c_csr), ctypes.POINTER(c_opts),
                             ctypes.POINTER(c_sym_info), vp, vp, vp, i64, vp, ctypes.c_size_t, vp], ctypes.c_int),
    "hcsp_spgemm_status": ([vp, ctypes.c_size_t, vp], ctypes.c_int),
    "hcsp_spgemm_noalloc": ([ctypes.POINTER(c_operand), ctypes.POINTER(c_csr), ctypes.POINTER(c_opts), vp, vp, vp,
                             i64, ctypes.POINTER(i64), vp], ctypes.c_int),
    "hcsp_csr_transpose_workspace": ([i64, i64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hcsp_csr_transpose": ([ctypes.POINTER(c_csr), ctypes.POINTER(c_csr), vp, ctypes.c_size_t, vp], ctypes.c_int),
    "hcsp_cluster_output_layout": ([ctypes.POINTER(c_operand), ctypes.POINTER(c_csr), ctypes.POINTER(c_opts),
                                    ctypes.POINTER(c_sym_info), vp, vp, ctypes.POINTER(i64), ctypes.POINTER(i64), vp,
                                    ctypes.c_size_t, vp], ctypes.c_int),
    "hcsp_spgemm_numeric_cluster": ([ctypes.POINTER(c_operand), ctypes.POINTER(c_csr), ctypes.POINTER(c_opts),
                                     ctypes.POINTER(c_sym_info), ctypes.POINTER(c_csr_cluster), vp, ctypes.c_size_t,
                                     vp], ctypes.c_int),
    "hcsp_batch_plan_init": ([i32, ctypes.POINTER(c_batch_item), ctypes.POINTER(c_opts),
                              ctypes.POINTER(c_batch_plan)], ctypes.c_int),
    "hcsp_batch_prepare": ([ctypes.POINTER(c_batch_plan), ctypes.POINTER(c_batch_item), vp, ctypes.c_size_t, vp, vp,
                            vp], ctypes.c_int),
    "hcsp_spgemm_batched": ([ctypes.POINTER(c_batch_plan), vp, vp, vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
    "hcsp_batch_status": ([ctypes.POINTER(c_batch_plan), vp, ctypes.c_size_t, vp, vp], ctypes.c_int),
    "hcsp_features": ([ctypes.POINTER(c_csr), ctypes.POINTER(c_csr), vp], ctypes.c_int),
    "hcsp_order_rcm": ([ctypes.POINTER(c_csr), vp], ctypes.c_int),
    "hcsp_order_degree": ([ctypes.POINTER(c_csr), vp], ctypes.c_int),
    "hcsp_permute_h": ([ctypes.POINTER(c_csr), vp, vp, ctypes.POINTER(c_csr), i32], ctypes.c_int),
    "hcsp_spgemm_products": ([ctypes.POINTER(c_csr), ctypes.POINTER(c_csr), ctypes.POINTER(i64), vp, ctypes.c_size_t,
                              vp], ctypes.c_int),
    "hcsp_predicted_workspace": ([ctypes.POINTER(c_csr), ctypes.POINTER(c_csr), ctypes.POINTER(c_opts),
                                  ctypes.c_float, i64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hcsp_spgemm_predicted": ([ctypes.POINTER(c_csr), ctypes.POINTER(c_csr), ctypes.POINTER(c_opts), ctypes.c_float,
                               i64, vp, vp, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, ctypes.c_size_t,
                               vp], ctypes.c_int),
    "hcsp_predicted_rows_workspace": ([ctypes.POINTER(c_csr), ctypes.POINTER(c_csr), ctypes.POINTER(c_opts), i64,
                                       ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "hcsp_spgemm_predicted_rows": ([ctypes.POINTER(c_csr), ctypes.POINTER(c_csr), ctypes.POINTER(c_opts), vp, i64,
                                    vp, vp, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, ctypes.c_size_t,
                                    vp], ctypes.c_int),
    "hcsp_mlp_forward": ([vp, vp, vp, i32, vp, vp, vp], ctypes.c_int),
    "hcsp_mlp_backward": ([vp, vp, vp, vp, vp, i32, ctypes.c_float, vp, vp, vp, vp], ctypes.c_int),
    "hcsp_mlp_adam": ([vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp],
                      ctypes.c_int),
    "hcsp_mlp_train_step": ([vp, vp, vp, vp, vp, i32, ctypes.c_float, vp, vp, vp, vp, vp, vp, vp, i32,
                             ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp], ctypes.c_int),
    "hcsp_mlp_create": ([vp, vp, ctypes.c_char_p, ctypes.POINTER(vp)], ctypes.c_int),
    "hcsp_mlp_destroy": ([vp], ctypes.c_int),
    "hcsp_mlp_get": ([vp, vp, vp, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
    "hcsp_mlp_set": ([vp, vp, vp], ctypes.c_int),
    "hcsp_mlp_save": ([vp, ctypes.c_char_p], ctypes.c_int),
    "hcsp_mlp_load": ([ctypes.c_char_p, ctypes.POINTER(vp)], ctypes.c_int),
    "hcsp_tune_create": ([ctypes.POINTER(vp)], ctypes.c_int),
    "hcsp_tune_destroy": ([vp], ctypes.c_int),
    "hcsp_tune_class": ([vp, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
    "hcsp_tune_add": ([vp, ctypes.c_char_p, ctypes.POINTER(c_tune_run)], ctypes.c_int),
    "hcsp_tune_get": ([vp, ctypes.c_char_p, ctypes.POINTER(c_tune_choice)], ctypes.c_int),
    "hcsp_tune_lookup": ([vp, vp, ctypes.POINTER(c_tune_choice)], ctypes.c_int),
    "hcsp_tune_classes": ([vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(i32)], ctypes.c_int),
    "hcsp_tune_runs": ([vp, ctypes.c_char_p, ctypes.POINTER(c_tune_run), i32, ctypes.POINTER(i32)], ctypes.c_int),
    "hcsp_tune_save": ([vp, ctypes.c_char_p], ctypes.c_int),
    "hcsp_tune_load": ([ctypes.c_char_p, ctypes.POINTER(vp)], ctypes.c_int),
}
MLP_NPARAMS, MLP_NACT, MLP_NDELTA = 6597, 160, 133
NFEATURES = 32

_lib = None


class HcspError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__("%s: %s (%s)" % (where, STATUS.get(status, status), detail))
        self.status = status


def lib():
    """The loaded ``libhcsp.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhcsp.so is not built (run __graft_entry__.build() or "
                               "python paper_2507_21253_amd/build.py); there is no fallback")
        # torch first: its HIP runtime is then the one the library's HIP calls bind to, so torch's
        # streams and device memory are valid in the library
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != HCSP_OK:
        raise HcspError(rc, where, lib().hcsp_last_error().decode())


def _np(a):
    return None if a is None else a.ctypes.data_as(vp)


def _ratio(t) -> c_ratio:
    if isinstance(t, tuple):
        return c_ratio(int(t[0]), int(t[1]))      # passed as given; the library validates it
    f = Fraction(t).limit_denominator(1 << 20)
    return c_ratio(f.numerator, f.denominator)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return vp(s.cuda_stream)


def _tp(t):
    return None if t is None else vp(t.data_ptr())


# ------------------------------------------------------------------ matrices

@dataclass
class DeviceCSR:
    """CSR matrix in device memory (torch tensors): row_ptr int64, col int32, val float64."""

    row_ptr: "object"
    col: "object"
    val: "object"
    nrows: int
    ncols: int

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @staticmethod
    def from_host(H, device="cuda"):
        import torch
        return DeviceCSR(torch.from_numpy(np.ascontiguousarray(H.rp)).to(device),
                         torch.from_numpy(np.ascontiguousarray(H.col)).to(device),
                         torch.from_numpy(np.ascontiguousarray(H.val)).to(device), H.nrows, H.ncols)

    def to_host(self):
        from types import SimpleNamespace
        return SimpleNamespace(rp=self.row_ptr.cpu().numpy(), col=self.col.cpu().numpy(),
                               val=self.val.cpu().numpy(), nrows=self.nrows, ncols=self.ncols)

    def c(self) -> c_csr:
        return c_csr(self.nrows, self.ncols, self.nnz, _tp(self.row_ptr), _tp(self.col), _tp(self.val))


@dataclass
class DeviceCluster:
    """CSR_Cluster in device memory (see include/hcsp.h for the layout)."""

    nrows: int
    ncols: int
    nclusters: int
    ncc: int
    nslots: int
    max_cluster: int
    cl_row_ptr: "object"
    perm: "object"
    cl_col_ptr: "object"
    cl_col: "object"
    cl_mask: "object"
    cl_val_ptr: "object"
    cl_val: "object"

    def c(self) -> c_csr_cluster:
        return c_csr_cluster(self.nrows, self.ncols, self.nclusters, self.ncc, self.nslots, self.max_cluster, 0,
                             _tp(self.cl_row_ptr), _tp(self.perm), _tp(self.cl_col_ptr), _tp(self.cl_col),
                             _tp(self.cl_mask), _tp(self.cl_val_ptr), _tp(self.cl_val))

    def bytes(self) -> int:
        return 8 * 3 * (self.nclusters + 1) + 4 * self.nrows + 6 * self.ncc + 8 * self.nslots


def operand(A) -> c_operand:
    op = c_operand()
    if isinstance(A, DeviceCluster):
        op.kind = OP_CLUSTER
        op.cl = A.c()
    else:
        op.kind = OP_CSR
        op.csr = A.c()
    return op


def opts(**kw) -> c_opts:
    o = c_opts()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


# ------------------------------------------------------------------ C-ABI mirrors

def version() -> str:
    return lib().hcsp_version().decode()


def strerror(status: int) -> str:
    return lib().hcsp_strerror(status).decode()


def last_error() -> str:
    return lib().hcsp_last_error().decode()


def csr_check(A: DeviceCSR, ws=None, stream=None) -> int:
    """Validate a device CSR matrix; returns the status code (0 = valid)."""
    import torch
    if ws is None:
        ws = torch.empty(64, dtype=torch.uint8, device=A.row_ptr.device)
    m = A.c()
    return lib().hcsp_csr_check(ctypes.byref(m), _tp(ws), ws.numel(), _stream(stream))


def _host_csr(H) -> c_csr:
    rp = np.ascontiguousarray(H.rp, np.int64)
    col = np.ascontiguousarray(H.col, np.int32)
    H._keep = (rp, col)
    return c_csr(H.nrows, H.ncols, int(rp[-1]) if len(rp) else 0, _np(rp), _np(col), None)


@dataclass
class Plan:
    """Cluster plan: cluster c holds original rows perm[cl_row_ptr[c]:cl_row_ptr[c+1]]."""

    perm: np.ndarray
    cl_row_ptr: np.ndarray

    @property
    def nclusters(self) -> int:
        return len(self.cl_row_ptr) - 1


def plan_fixed(nrows: int, K: int, perm_in=None) -> Plan:
    pi = None if perm_in is None else np.ascontiguousarray(perm_in, np.int32)
    perm = np.empty(max(nrows, 1), np.int32)
    crp = np.empty(nrows + 1, np.int64)
    ncl = i64()
    _check(lib().hcsp_plan_fixed(nrows, K, _np(pi), _np(perm), _np(crp), ctypes.byref(ncl)), "plan_fixed")
    return Plan(perm[:nrows], crp[:ncl.value + 1].copy())


def plan_variable(A_host, jacc_th=(3, 10), max_cluster: int = 8, perm_in=None) -> Plan:
    m = _host_csr(A_host)
    pi = None if perm_in is None else np.ascontiguousarray(perm_in, np.int32)
    perm = np.empty(max(A_host.nrows, 1), np.int32)
    crp = np.empty(A_host.nrows + 1, np.int64)
    ncl = i64()
    _check(lib().hcsp_plan_variable(ctypes.byref(m), _ratio(jacc_th), max_cluster, _np(pi), _np(perm), _np(crp),
                                    ctypes.byref(ncl)), "plan_variable")
    return Plan(perm[:A_host.nrows], crp[:ncl.value + 1].copy())


def plan_hierarchical(A_host, jacc_th=(3, 10), max_cluster: int = 8, sim=SIM_ROOT, nthreads: int = 0,
                      perm_in=None) -> Plan:
    m = _host_csr(A_host)
    pi = None if perm_in is None else np.ascontiguousarray(perm_in, np.int32)
    perm = np.empty(max(A_host.nrows, 1), np.int32)
    crp = np.empty(A_host.nrows + 1, np.int64)
    ncl = i64()
    _check(lib().hcsp_plan_hierarchical(ctypes.byref(m), _ratio(jacc_th), max_cluster, sim, nthreads, _np(pi),
                                        _np(perm), _np(crp), ctypes.byref(ncl)), "plan_hierarchical")
    return Plan(perm[:A_host.nrows], crp[:ncl.value + 1].copy())


def csr_transpose(A: "DeviceCSR", values: bool = True, stream=None) -> "DeviceCSR":
    """A^T on the device (values gathered when ``values``; otherwise val is an empty tensor)."""
    import torch
    dev = A.row_ptr.device
    nb = ctypes.c_size_t()
    _check(lib().hcsp_csr_transpose_workspace(A.nrows, A.ncols, ctypes.byref(nb)), "csr_transpose_workspace")
    ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=dev)
    T = DeviceCSR(torch.empty(A.ncols + 1, dtype=torch.int64, device=dev),
                  torch.empty(A.nnz, dtype=torch.int32, device=dev),
                  torch.empty(A.nnz if values else 0, dtype=torch.float64, device=dev), A.ncols, A.nrows)
    a = A.c()
    t = T.c()
    if not values:
        t.val = None
    _check(lib().hcsp_csr_transpose(ctypes.byref(a), ctypes.byref(t), _tp(ws), ws.numel(), _stream(stream)),
           "csr_transpose")
    T._ws = ws  # kept alive until the asynchronous launches are done with it
    return T


def topk_candidates_gpu(A: "DeviceCSR", jacc_th=(3, 10), topk: int = 7, perm_in=None, stream=None):
    """SpGEMM_TopK(A, A^T) (Alg. 3) on the GPU: the overlap matrix A A^T is the library's own product of A's
    pattern (all values 1) with its transpose (formed on the device), then one wavefront per row keeps its
    topk best partners.  Returns host arrays in plan positions: (cnt[n], nbr[n, topk], ov[n, topk])."""
    import torch
    dev = A.row_ptr.device
    ones = torch.ones(A.nnz, dtype=torch.float64, device=dev)
    P = DeviceCSR(A.row_ptr, A.col, ones, A.nrows, A.ncols)
    Pt = csr_transpose(P, values=False, stream=stream)
    Pt.val = ones                      # the pattern's values are all 1 on both sides
    O = spgemm(P, Pt, stream=stream)
    n = A.nrows
    pos = None
    if perm_in is not None:
        pi = torch.from_numpy(np.ascontiguousarray(perm_in, np.int32)).to(dev)
        pos = torch.empty(n, dtype=torch.int32, device=dev)
        pos[pi.long()] = torch.arange(n, dtype=torch.int32, device=dev)
    cnt = torch.zeros(n, dtype=torch.int32, device=dev)
    nbr = torch.full((max(n, 1) * topk,), -1, dtype=torch.int32, device=dev)
    ov = torch.zeros(max(n, 1) * topk, dtype=torch.int64, device=dev)
    oc = O.c()
    _check(lib().hcsp_topk_candidates(ctypes.byref(oc), _tp(A.row_ptr), _tp(pos) if pos is not None else None,
                                      _ratio(jacc_th), topk, _tp(cnt), _tp(nbr), _tp(ov), _stream(stream)),
           "topk_candidates")
    return cnt.cpu().numpy(), nbr.cpu().numpy()[:n * topk].reshape(n, topk), ov.cpu().numpy()[:n * topk].reshape(n, topk)


def plan_hierarchical_candidates(A_host, jacc_th, max_cluster: int, sim, cnt, nbr, ov, perm_in=None) -> Plan:
    """hierarchical plan (Alg. 3) from given candidate lists (positions; topk = max_cluster - 1): only the
    merge loop runs on the host."""
    m = _host_csr(A_host)
    pi = None if perm_in is None else np.ascontiguousarray(perm_in, np.int32)
    perm = np.empty(max(A_host.nrows, 1), np.int32)
    crp = np.empty(A_host.nrows + 1, np.int64)
    ncl = i64()
    cnt = np.ascontiguousarray(cnt, np.int32)
    nbr = np.ascontiguousarray(nbr, np.int32)
    ov = np.ascontiguousarray(ov, np.int64)
    _check(lib().hcsp_plan_hierarchical_candidates(ctypes.byref(m), _ratio(jacc_th), max_cluster, sim, _np(pi),
                                                   _np(cnt), _np(nbr), _np(ov), _np(perm), _np(crp),
                                                   ctypes.byref(ncl)), "plan_hierarchical_candidates")
    return Plan(perm[:A_host.nrows], crp[:ncl.value + 1].copy())


def plan_hierarchical_gpu(A_host, A: "DeviceCSR", jacc_th=(3, 10), max_cluster: int = 8, sim=SIM_ROOT,
                          perm_in=None) -> Plan:
    """hierarchical plan with the candidate search on the GPU and the merge loop on the host; the same plan
    as plan_hierarchical."""
    if max_cluster <= 1:
        return plan_hierarchical(A_host, jacc_th, max_cluster, sim, perm_in=perm_in)
    cnt, nbr, ov = topk_candidates_gpu(A, jacc_th, max_cluster - 1, perm_in)
    return plan_hierarchical_candidates(A_host, jacc_th, max_cluster, sim, cnt, nbr, ov, perm_in)


def order_rcm(A_host) -> np.ndarray:
    """Reverse Cuthill-McKee order (position -> original row) of the pattern of A + A^T."""
    m = _host_csr(A_host)
    perm = np.empty(max(A_host.nrows, 1), np.int32)
    _check(lib().hcsp_order_rcm(ctypes.byref(m), _np(perm)), "order_rcm")
    return perm[:A_host.nrows]


def order_degree(A_host) -> np.ndarray:
    """Rows by descending length, ties by ascending id (position -> original row)."""
    m = _host_csr(A_host)
    perm = np.empty(max(A_host.nrows, 1), np.int32)
    _check(lib().hcsp_order_degree(ctypes.byref(m), _np(perm)), "order_degree")
    return perm[:A_host.nrows]


def permute_h(A_host, rperm=None, cperm=None, nthreads: int = 0):
    """Host copy of A with rows and columns reordered (new row r = old row rperm[r], new column c = old
    column cperm[c]); rows come out sorted.  Returns an object with rp, col, val, nrows, ncols."""
    from types import SimpleNamespace
    val = np.ascontiguousarray(A_host.val, np.float64)
    a = _host_csr(A_host)
    a.val = _np(val)
    rp = np.empty(A_host.nrows + 1, np.int64)
    col = np.empty(max(len(A_host.col), 1), np.int32)
    v = np.empty(max(len(A_host.col), 1), np.float64)
    o = c_csr(A_host.nrows, A_host.ncols, len(A_host.col), _np(rp), _np(col), _np(v))
    rpn = None if rperm is None else np.ascontiguousarray(rperm, np.int32)
    cpn = None if cperm is None else np.ascontiguousarray(cperm, np.int32)
    _check(lib().hcsp_permute_h(ctypes.byref(a), _np(rpn), _np(cpn), ctypes.byref(o),
                                nthreads or len(os.sched_getaffinity(0))), "permute_h")
    n = len(A_host.col)
    return SimpleNamespace(rp=rp, col=col[:n], val=v[:n], nrows=A_host.nrows, ncols=A_host.ncols, nnz=n)


def features(A_host, B_host=None) -> np.ndarray:
    """The library's structure-only features of the product A x B (B defaults to A), float32[32]."""
    B_host = A_host if B_host is None else B_host
    a = _host_csr(A_host)
    b = _host_csr(B_host)
    out = np.zeros(NFEATURES, np.float32)
    _check(lib().hcsp_features(ctypes.byref(a), ctypes.byref(b), _np(out)), "features")
    return out


def cluster_workspace(nrows: int, ncl: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().hcsp_cluster_workspace(nrows, ncl, ctypes.byref(b)), "cluster_workspace")
    return b.value


def cluster_count(A: DeviceCSR, perm_d, cl_row_ptr_d, ws, stream=None):
    """Returns (cl_col_ptr, cl_val_ptr, ncc, nslots, max_cluster)."""
    import torch
    ncl = cl_row_ptr_d.numel() - 1
    ccp = torch.empty(ncl + 1, dtype=torch.int64, device=cl_row_ptr_d.device)
    cvp = torch.empty(ncl + 1, dtype=torch.int64, device=cl_row_ptr_d.device)
    ncc, nslots, mx = i64(), i64(), i32()
    m = A.c()
    _check(lib().hcsp_cluster_count(ctypes.byref(m), _tp(perm_d), _tp(cl_row_ptr_d), ncl, _tp(ccp), _tp(cvp),
                                    ctypes.byref(ncc), ctypes.byref(nslots), ctypes.byref(mx), _tp(ws), ws.numel(),
                                    _stream(stream)), "cluster_count")
    return ccp, cvp, ncc.value, nslots.value, mx.value


def cluster_fill(A: DeviceCSR, out: DeviceCluster, stream=None):
    m = A.c()
    o = out.c()
    _check(lib().hcsp_cluster_fill(ctypes.byref(m), ctypes.byref(o), _stream(stream)), "cluster_fill")


def cluster_build(A: DeviceCSR, plan: Plan, stream=None) -> DeviceCluster:
    """CSR_Cluster of A on the device for a host plan (count, allocate, fill)."""
    import torch
    dev = A.row_ptr.device
    perm_d = torch.from_numpy(np.ascontiguousarray(plan.perm, np.int32)).to(dev)
    crp_d = torch.from_numpy(np.ascontiguousarray(plan.cl_row_ptr, np.int64)).to(dev)
    ws = torch.empty(cluster_workspace(A.nrows, plan.nclusters), dtype=torch.uint8, device=dev)
    ccp, cvp, ncc, nslots, mx = cluster_count(A, perm_d, crp_d, ws, stream)
    out = DeviceCluster(A.nrows, A.ncols, plan.nclusters, ncc, nslots, mx, crp_d, perm_d, ccp,
                        torch.empty(ncc, dtype=torch.int32, device=dev),
                        torch.empty(ncc, dtype=torch.int16, device=dev),
                        cvp, torch.empty(nslots, dtype=torch.float64, device=dev))
    cluster_fill(A, out, stream)
    return out


def spgemm_workspace(A, B: DeviceCSR, o: c_opts | None = None) -> int:
    op = operand(A)
    b = B.c()
    o = o or c_opts()
    n = ctypes.c_size_t()
    _check(lib().hcsp_spgemm_workspace(ctypes.byref(op), ctypes.byref(b), ctypes.byref(o), ctypes.byref(n)),
           "spgemm_workspace")
    return n.value


def spgemm_symbolic(A, B: DeviceCSR, C_row_ptr, ws, o: c_opts | None = None, stream=None) -> c_sym_info:
    op = operand(A)
    b = B.c()
    o = o or c_opts()
    info = c_sym_info()
    _check(lib().hcsp_spgemm_symbolic(ctypes.byref(op), ctypes.byref(b), ctypes.byref(o), _tp(C_row_ptr),
                                      ctypes.byref(info), _tp(ws), ws.numel(), _stream(stream)), "spgemm_symbolic")
    return info


def spgemm_status(ws, stream=None):
    """Raises HcspError if the kernels of the last numeric call on this workspace recorded an error."""
    _check(lib().hcsp_spgemm_status(_tp(ws), ws.numel(), _stream(stream)), "spgemm_status")


def spgemm_numeric(A, B: DeviceCSR, info: c_sym_info, C_row_ptr, C_col, C_val, ws, o: c_opts | None = None,
                   capacity: int | None = None, stream=None):
    op = operand(A)
    b = B.c()
    o = o or c_opts()
    cap = C_col.numel() if capacity is None else capacity
    _check(lib().hcsp_spgemm_numeric(ctypes.byref(op), ctypes.byref(b), ctypes.byref(o), ctypes.byref(info),
                                     _tp(C_row_ptr), _tp(C_col), _tp(C_val), cap, _tp(ws), ws.numel(),
                                     _stream(stream)), "spgemm_numeric")


NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024


def spgemm_noalloc(A, B: DeviceCSR, C_row_ptr, C_col, C_val, o: c_opts | None = None, stream=None) -> int:
    """The whole product into caller buffers with the library's static workspace (no device allocation in
    the library); returns nnz(C)."""
    op = operand(A)
    b = B.c()
    o = o or c_opts()
    nnz = i64()
    rc = lib().hcsp_spgemm_noalloc(ctypes.byref(op), ctypes.byref(b), ctypes.byref(o), _tp(C_row_ptr), _tp(C_col),
                                   _tp(C_val), C_col.numel(), ctypes.byref(nnz), _stream(stream))
    _check(rc, "spgemm_noalloc")
    return nnz.value


class Product:
    """Workspace and output buffers for repeated C = A x B with one structure (the paper's use case of
    many SpGEMMs on the same operands).  ``run()`` does symbolic, the nnz read-back, and numeric."""

    def __init__(self, A, B: DeviceCSR, o: c_opts | None = None):
        import torch
        self.A, self.B = A, B
        self.o = o or c_opts()
        dev = B.row_ptr.device
        self.ws = torch.empty(spgemm_workspace(A, B, self.o), dtype=torch.uint8, device=dev)
        self.C_row_ptr = torch.empty(A.nrows + 1, dtype=torch.int64, device=dev)
        self.C_col = torch.empty(0, dtype=torch.int32, device=dev)
        self.C_val = torch.empty(0, dtype=torch.float64, device=dev)
        self.info = None

    def symbolic(self, stream=None):
        import torch
        self.info = spgemm_symbolic(self.A, self.B, self.C_row_ptr, self.ws, self.o, stream)
        nnz = self.info.nnz
        if self.C_col.numel() < nnz:
            self.C_col = torch.empty(nnz, dtype=torch.int32, device=self.ws.device)
            self.C_val = torch.empty(nnz, dtype=torch.float64, device=self.ws.device)
        return nnz

    def numeric(self, stream=None):
        spgemm_numeric(self.A, self.B, self.info, self.C_row_ptr, self.C_col, self.C_val, self.ws, self.o,
                       capacity=self.info.nnz, stream=stream)

    def check(self, stream=None):
        """Raises if the last numeric phase recorded an error (synchronizes)."""
        spgemm_status(self.ws, stream)

    def run(self, stream=None, check: bool = True) -> DeviceCSR:
        """Both phases; with ``check`` the numeric phase's error word is read back (one more
        synchronization), else call ``check()`` after a series of runs."""
        nnz = self.symbolic(stream)
        self.numeric(stream)
        if check:
            self.check(stream)
        return DeviceCSR(self.C_row_ptr, self.C_col[:nnz], self.C_val[:nnz], self.A.nrows, self.B.ncols)


def spgemm(A, B: DeviceCSR, o: c_opts | None = None, stream=None) -> DeviceCSR:
    """C = A x B (A: DeviceCSR or DeviceCluster) with C in A's original row order."""
    return Product(A, B, o).run(stream)


class ClusterProduct:
    """Buffers for repeated C = A x B with a CSR_Cluster A and C in CSR_Cluster form on A's clusters (Alg. 1's
    output).  ``run()`` does the symbolic phase, the output layout (one read-back) and the numeric phase."""

    def __init__(self, A: DeviceCluster, B: DeviceCSR, o: c_opts | None = None):
        import torch
        self.P = Product(A, B, o)
        self.A, self.B = A, B
        dev = B.row_ptr.device
        self.colp = torch.empty(A.nclusters + 1, dtype=torch.int64, device=dev)
        self.valp = torch.empty(A.nclusters + 1, dtype=torch.int64, device=dev)
        self.col = torch.empty(0, dtype=torch.int32, device=dev)
        self.mask = torch.empty(0, dtype=torch.int16, device=dev)
        self.val = torch.empty(0, dtype=torch.float64, device=dev)

    def run(self, stream=None) -> DeviceCluster:
        import torch
        P, A, B = self.P, self.A, self.B
        P.symbolic(stream)
        ncc, nslots = i64(), i64()
        opa, opb = operand(A), B.c()
        _check(lib().hcsp_cluster_output_layout(ctypes.byref(opa), ctypes.byref(opb), ctypes.byref(P.o),
                                                ctypes.byref(P.info), _tp(self.colp), _tp(self.valp),
                                                ctypes.byref(ncc), ctypes.byref(nslots), _tp(P.ws), P.ws.numel(),
                                                _stream(stream)), "cluster_output_layout")
        if self.col.numel() < ncc.value:
            self.col = torch.empty(ncc.value, dtype=torch.int32, device=self.colp.device)
            self.mask = torch.empty(ncc.value, dtype=torch.int16, device=self.colp.device)
        if self.val.numel() < nslots.value:
            self.val = torch.empty(nslots.value, dtype=torch.float64, device=self.colp.device)
        C = DeviceCluster(A.nrows, B.ncols, A.nclusters, ncc.value, nslots.value, A.max_cluster, A.cl_row_ptr,
                          A.perm, self.colp, self.col[:ncc.value], self.mask[:ncc.value], self.valp,
                          self.val[:nslots.value])
        cc = C.c()
        _check(lib().hcsp_spgemm_numeric_cluster(ctypes.byref(opa), ctypes.byref(opb), ctypes.byref(P.o),
                                                 ctypes.byref(P.info), ctypes.byref(cc), _tp(P.ws), P.ws.numel(),
                                                 _stream(stream)), "spgemm_numeric_cluster")
        return C


def spgemm_cluster_out(A: DeviceCluster, B: DeviceCSR, o: c_opts | None = None, stream=None) -> DeviceCluster:
    """C = A x B for a CSR_Cluster A, with C in CSR_Cluster form on A's clusters (Alg. 1's output)."""
    return ClusterProduct(A, B, o).run(stream)


# ------------------------------------------------------------------ batches

def batch_plan_init(items, o: c_opts | None = None) -> c_batch_plan:
    plan = c_batch_plan()
    o = o or c_opts()
    _check(lib().hcsp_batch_plan_init(len(items), items, ctypes.byref(o), ctypes.byref(plan)), "batch_plan_init")
    return plan


def batch_prepare(plan: c_batch_plan, items, ws, stream=None):
    """Returns (out_offset, seg_offset), numpy int64 arrays of count+1 entries."""
    n = plan.count
    out_off = np.zeros(n + 1, np.int64)
    seg_off = np.zeros(n + 1, np.int64)
    _check(lib().hcsp_batch_prepare(ctypes.byref(plan), items, _tp(ws), ws.numel(), _np(out_off), _np(seg_off),
                                    _stream(stream)), "batch_prepare")
    return out_off, seg_off


def spgemm_batched(plan: c_batch_plan, C_row_ptr, C_col, C_val, ws, stream=None):
    _check(lib().hcsp_spgemm_batched(ctypes.byref(plan), _tp(C_row_ptr), _tp(C_col), _tp(C_val), _tp(ws), ws.numel(),
                                     _stream(stream)), "spgemm_batched")


def batch_status(plan: c_batch_plan, ws, stream=None) -> np.ndarray:
    nnz = np.zeros(max(plan.count, 1), np.int64)
    _check(lib().hcsp_batch_status(ctypes.byref(plan), _tp(ws), ws.numel(), _np(nnz), _stream(stream)),
           "batch_status")
    return nnz[:plan.count]


class Batch:
    """Many independent products C_p = A_p x B_p computed by one fixed launch sequence (capturable into a
    graph).  ``run()`` enqueues both phases for every product; ``status()`` synchronizes and returns each
    product's nnz; ``result(p)`` is product p's C as a DeviceCSR view of the flat outputs."""

    def __init__(self, pairs, o: c_opts | None = None, stream=None):
        import torch
        self.pairs = list(pairs)
        n = len(self.pairs)
        self.items = (c_batch_item * max(n, 1))()
        for p, (A, B) in enumerate(self.pairs):
            self.items[p].A = operand(A)
            self.items[p].B = B.c()
        self.plan = batch_plan_init(self.items, o)
        dev = self.pairs[0][1].row_ptr.device if n else torch.device("cuda")
        self.ws = torch.empty(max(self.plan.ws_bytes, 1), dtype=torch.uint8, device=dev)
        self.out_off, self.seg_off = batch_prepare(self.plan, self.items, self.ws, stream)
        self.C_row_ptr = torch.empty(max(self.plan.row_ptr_len, 1), dtype=torch.int64, device=dev)
        self.C_col = torch.empty(max(self.plan.out_capacity, 1), dtype=torch.int32, device=dev)
        self.C_val = torch.empty(max(self.plan.out_capacity, 1), dtype=torch.float64, device=dev)

    def run(self, stream=None):
        spgemm_batched(self.plan, self.C_row_ptr, self.C_col, self.C_val, self.ws, stream)

    def status(self, stream=None) -> np.ndarray:
        return batch_status(self.plan, self.ws, stream)

    def result(self, p: int, nnz: int | None = None) -> DeviceCSR:
        A, B = self.pairs[p]
        s0 = int(self.seg_off[p])
        rp = self.C_row_ptr[s0:s0 + A.nrows + 1]
        if nnz is None:
            nnz = int(rp[-1].item())
        o0 = int(self.out_off[p])
        return DeviceCSR(rp, self.C_col[o0:o0 + nnz], self.C_val[o0:o0 + nnz], A.nrows, B.ncols)


# ------------------------------------------------------------------ learned selector (device arrays)

def mlp_forward(params, norm, X, Z, act=None, stream=None):
    _check(lib().hcsp_mlp_forward(_tp(params), _tp(norm), _tp(X), X.shape[0], _tp(Z), _tp(act), _stream(stream)),
           "mlp_forward")


def mlp_backward(params, act, Z, y, t, lam, delta, loss, grad, stream=None):
    _check(lib().hcsp_mlp_backward(_tp(params), _tp(act), _tp(Z), _tp(y), _tp(t), Z.shape[0], float(lam),
                                   _tp(delta), _tp(loss), _tp(grad), _stream(stream)), "mlp_backward")


def mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().hcsp_mlp_adam(_tp(params), _tp(grad), _tp(m), _tp(v), int(step), float(lr), float(beta1),
                               float(beta2), float(eps), _stream(stream)), "mlp_adam")


def mlp_train_step(params, norm, X, y, t, lam, act, Z, delta, loss, grad, m, v, step, lr=1e-3, beta1=0.9,
                   beta2=0.999, eps=1e-8, stream=None):
    _check(lib().hcsp_mlp_train_step(_tp(params), _tp(norm), _tp(X), _tp(y), _tp(t), X.shape[0], float(lam), _tp(act),
                                     _tp(Z), _tp(delta), _tp(loss), _tp(grad), _tp(m), _tp(v), int(step), float(lr),
                                     float(beta1), float(beta2), float(eps), _stream(stream)), "mlp_train_step")


class MlpModel:
    """Host copy of the selector's model in the library (parameters, feature normalization, a one-line tag),
    saved and loaded by the library's model file."""

    def __init__(self, params=None, norm=None, tag: str = "", _handle=None):
        if _handle is not None:
            self._h = _handle
            return
        h = vp()
        p = None if params is None else np.ascontiguousarray(params, np.float32)
        nm = None if norm is None else np.ascontiguousarray(norm, np.float32)
        if p is not None and p.size != MLP_NPARAMS or nm is not None and nm.size != 2 * NFEATURES:
            raise ValueError("parameter or normalization size")
        _check(lib().hcsp_mlp_create(_np(p), _np(nm), tag.encode(), ctypes.byref(h)), "mlp_create")
        self._h = h

    @staticmethod
    def load(path: str) -> "MlpModel":
        h = vp()
        _check(lib().hcsp_mlp_load(path.encode(), ctypes.byref(h)), "mlp_load")
        return MlpModel(_handle=h)

    def save(self, path: str):
        _check(lib().hcsp_mlp_save(self._h, path.encode()), "mlp_save")

    def get(self):
        """(params float32[MLP_NPARAMS], norm float32[64] (mu then sd), tag)"""
        p = np.empty(MLP_NPARAMS, np.float32)
        nm = np.empty(2 * NFEATURES, np.float32)
        buf = ctypes.create_string_buffer(4096)
        _check(lib().hcsp_mlp_get(self._h, _np(p), _np(nm), buf, len(buf)), "mlp_get")
        return p, nm, buf.value.decode()

    def set(self, params=None, norm=None):
        p = None if params is None else np.ascontiguousarray(params, np.float32)
        nm = None if norm is None else np.ascontiguousarray(norm, np.float32)
        _check(lib().hcsp_mlp_set(self._h, _np(p), _np(nm)), "mlp_set")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.hcsp_mlp_destroy(h)
            self._h = None


# ------------------------------------------------------------------ autotuner table

def tune_class(f) -> str:
    """The autotuner's class key of a matrix from its structure features."""
    f = np.ascontiguousarray(f, np.float32)
    buf = ctypes.create_string_buffer(64)
    _check(lib().hcsp_tune_class(_np(f), buf, len(buf)), "tune_class")
    return buf.value.decode()


def _choice_dict(c: c_tune_choice) -> dict:
    return {"path": "hc" if c.path == 1 else "plain", "max_cluster": c.max_cluster,
            "best_cluster_size": c.best_cluster_size, "sym_load_pct": c.sym_load_pct, "load_pct": c.load_pct,
            "cl_load_pct": c.cl_load_pct, "tuned": bool(c.tuned), "runs": c.runs}


class TuneTableNative:
    """The library's autotuner table (per-class runs and the choice rule of include/hcsp.h)."""

    def __init__(self, _handle=None):
        if _handle is None:
            _handle = vp()
            _check(lib().hcsp_tune_create(ctypes.byref(_handle)), "tune_create")
        self._h = _handle

    @staticmethod
    def load(path: str) -> "TuneTableNative":
        h = vp()
        _check(lib().hcsp_tune_load(path.encode(), ctypes.byref(h)), "tune_load")
        return TuneTableNative(h)

    def save(self, path: str):
        _check(lib().hcsp_tune_save(self._h, path.encode()), "tune_save")

    def add(self, key: str, run: c_tune_run):
        _check(lib().hcsp_tune_add(self._h, key.encode(), ctypes.byref(run)), "tune_add")

    def get(self, key: str) -> dict:
        c = c_tune_choice()
        _check(lib().hcsp_tune_get(self._h, key.encode(), ctypes.byref(c)), "tune_get")
        return _choice_dict(c)

    def lookup(self, f) -> dict:
        f = np.ascontiguousarray(f, np.float32)
        c = c_tune_choice()
        _check(lib().hcsp_tune_lookup(self._h, _np(f), ctypes.byref(c)), "tune_lookup")
        return _choice_dict(c)

    def classes(self) -> list:
        n = i32()
        _check(lib().hcsp_tune_classes(self._h, None, 0, ctypes.byref(n)), "tune_classes")
        buf = ctypes.create_string_buffer(64 * (n.value + 1))
        _check(lib().hcsp_tune_classes(self._h, buf, len(buf), ctypes.byref(n)), "tune_classes")
        return [k for k in buf.value.decode().split("\n") if k]

    def runs(self, key: str) -> list:
        n = i32()
        _check(lib().hcsp_tune_runs(self._h, key.encode(), None, 0, ctypes.byref(n)), "tune_runs")
        arr = (c_tune_run * max(n.value, 1))()
        _check(lib().hcsp_tune_runs(self._h, key.encode(), arr, n.value, ctypes.byref(n)), "tune_runs")
        return [arr[i] for i in range(n.value)]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.hcsp_tune_destroy(h)
            self._h = None


# ------------------------------------------------------------------ predicted sizes

def spgemm_products(A: DeviceCSR, B: DeviceCSR, stream=None) -> int:
    import torch
    ws = torch.empty(8, dtype=torch.uint8, device=B.row_ptr.device)
    a, b = A.c(), B.c()
    out = i64()
    _check(lib().hcsp_spgemm_products(ctypes.byref(a), ctypes.byref(b), ctypes.byref(out), _tp(ws), 8,
                                      _stream(stream)), "spgemm_products")
    return out.value


class PredictedProduct:
    """C = A x B with row sizes predicted from a compression ratio (nnz(C)/products, margin included), or
    given per row (``cap_row``: host integers, one per row of A, each clamped to [1, the row's products]);
    rows the prediction does not hold are recomputed through the exact symbolic phase.  ``run()`` returns C;
    ``n_overflow`` is the number of rows recomputed."""

    def __init__(self, A: DeviceCSR, B: DeviceCSR, ratio: float | None, o: c_opts | None = None, capacity=None,
                 cap_row=None):
        import torch
        self.A, self.B, self.o = A, B, o or c_opts()
        self.ratio = float(min(1.0, max(ratio if ratio is not None else 1.0, 1e-6)))
        self.products = spgemm_products(A, B)
        a, b = A.c(), B.c()
        n = ctypes.c_size_t()
        dev = B.row_ptr.device
        self.cap_row = None
        if cap_row is not None:
            c = np.asarray(cap_row, dtype=np.int64)
            if c.shape != (A.nrows,) or np.any(c > np.iinfo(np.int32).max):
                raise ValueError("cap_row: one int32 capacity per row of A")
            self.cap_sum = int(np.maximum(c, 0).sum())
            self.cap_row = torch.from_numpy(c.astype(np.int32)).to(dev)
            _check(lib().hcsp_predicted_rows_workspace(ctypes.byref(a), ctypes.byref(b), ctypes.byref(self.o),
                                                       self.cap_sum, ctypes.byref(n)), "predicted_rows_workspace")
        else:
            _check(lib().hcsp_predicted_workspace(ctypes.byref(a), ctypes.byref(b), ctypes.byref(self.o),
                                                  self.ratio, self.products, ctypes.byref(n)), "predicted_workspace")
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
        self.C_row_ptr = torch.empty(A.nrows + 1, dtype=torch.int64, device=dev)
        cap = self.products if capacity is None else capacity
        self.C_col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        self.C_val = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
        self.nnz = self.n_overflow = None

    def run(self, stream=None) -> DeviceCSR:
        a, b = self.A.c(), self.B.c()
        nnz, novf = i64(), i64()
        if self.cap_row is not None:
            _check(lib().hcsp_spgemm_predicted_rows(ctypes.byref(a), ctypes.byref(b), ctypes.byref(self.o),
                                                    _tp(self.cap_row), self.cap_sum, _tp(self.C_row_ptr),
                                                    _tp(self.C_col), _tp(self.C_val), self.C_col.numel(),
                                                    ctypes.byref(nnz), ctypes.byref(novf), _tp(self.ws),
                                                    self.ws.numel(), _stream(stream)), "spgemm_predicted_rows")
        else:
            _check(lib().hcsp_spgemm_predicted(ctypes.byref(a), ctypes.byref(b), ctypes.byref(self.o), self.ratio,
                                               self.products, _tp(self.C_row_ptr), _tp(self.C_col), _tp(self.C_val),
                                               self.C_col.numel(), ctypes.byref(nnz), ctypes.byref(novf),
                                               _tp(self.ws), self.ws.numel(), _stream(stream)), "spgemm_predicted")
        self.nnz, self.n_overflow = nnz.value, novf.value
        return DeviceCSR(self.C_row_ptr, self.C_col[:self.nnz], self.C_val[:self.nnz], self.A.nrows, self.B.ncols)
