/*
 * hcsp — clustered Gustavson SpGEMM on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libhcsp.so.  Plain pointers and sizes only; no C++ exceptions
 * cross this boundary.  Every entry point returns an int status: HCSP_OK (0)
 * or a negative HCSP_E_* code; hcsp_last_error() then holds a one-line
 * description (thread-local).
 *
 * Problem (paper, Background "SpGEMM Kernel" and Fig. 1): C = A x B with all
 * three matrices sparse.  A may be given as plain CSR or in the paper's
 * row-clustered CSR_Cluster format (Sec. "Access Pattern and Matrix
 * Format"); B is CSR; C is always CSR in A's original row order.  The
 * product runs in the two phases the paper describes: a symbolic phase that
 * counts the non-zeros of every output row so C can be allocated, then a
 * numeric phase that fills C.
 *
 * Conventions
 *  - Matrices: int64 row offsets, int32 column indices strictly increasing
 *    within a row, float64 values.  nrows/ncols/nnz < 2^31 for column and
 *    row ids; offsets are 64-bit.
 *  - Suffix _d: device pointer (memory the caller allocated on the GPU, e.g.
 *    a torch tensor).  Suffix _h: host pointer.  Pointers inside hcsp_csr /
 *    hcsp_csr_cluster are device pointers unless an entry point says "host".
 *  - The library never allocates device memory.  Callers query workspace
 *    sizes, allocate, and pass buffers in.  Host-side plans allocate only
 *    host memory.
 *  - Everything runs on the given stream (hipStream_t passed as void*, NULL
 *    = the default stream).  Only calls documented as synchronizing wait
 *    for the stream.
 *  - Kernels never write outside the caller's buffers: output writes are
 *    bounds-checked against the capacities passed in; a violation is
 *    reported as HCSP_E_CAPACITY where the call synchronizes.
 *  - Arithmetic contract: each output value c_ij starts at +0.0 and takes
 *    its contributions a_ik * b_kj in ascending k, each with one fused
 *    multiply-add (the accumulation order the CPU reference uses); entries
 *    whose value cancels to 0.0 are kept, so the structure of C is the
 *    boolean product.  Output columns are sorted ascending.
 */
#ifndef HCSP_H
#define HCSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
enum {
    HCSP_OK = 0,
    HCSP_E_INVALID = -1,     /* bad argument: null pointer, negative size, mismatched shapes */
    HCSP_E_PTR = -2,         /* row offsets not starting at 0, not monotone or not ending at nnz */
    HCSP_E_RANGE = -3,       /* a column index outside [0, ncols) */
    HCSP_E_UNSORTED = -4,    /* column indices not strictly increasing within a row */
    HCSP_E_CAPACITY = -5,    /* a workspace or output buffer is too small */
    HCSP_E_HIP = -6,         /* the HIP runtime reported an error */
    HCSP_E_NOMEM = -7,       /* host memory allocation failed */
    HCSP_E_UNSUPPORTED = -8, /* shape or option outside what the library implements */
    HCSP_E_OVERFLOW = -9     /* a count does not fit its index type */
};

/* ------------------------------------------------------------------ types */

/* CSR matrix (paper, Background "Sparse Matrix Storage Formats": row-id,
 * col-id and value arrays).  row_ptr[nrows+1], col[nnz], val[nnz]. */
typedef struct hcsp_csr {
    int64_t nrows, ncols, nnz;
    int64_t *row_ptr;
    int32_t *col;
    double *val;
} hcsp_csr;

/*
 * CSR_Cluster (paper, "Access Pattern and Matrix Format" and its figure):
 * rows grouped into clusters whose non-zeros are stored together column by
 * column.  Variable-length form: cluster sizes are kept as offsets, so row
 * ids are implicit, plus an array of pointers into the value array.
 *   cl_row_ptr[nclusters+1]  cluster c holds positions cl_row_ptr[c] .. cl_row_ptr[c+1)-1
 *   perm[nrows]              position -> original row id of A
 *   cl_col_ptr[nclusters+1]  cluster c's union columns are cl_col[cl_col_ptr[c] ..)
 *   cl_col[ncc]              sorted union of the member rows' columns
 *   cl_mask[ncc]             bit l set iff member l stores that column (the
 *                            placeholder positions of the paper have bit 0)
 *   cl_val_ptr[nclusters+1]  cluster c's values start at cl_val[cl_val_ptr[c]]
 *   cl_val[nslots]           column-major per cluster: value of member l at union
 *                            column t is cl_val[cl_val_ptr[c] + t*s + l], +0.0 for
 *                            placeholders (s = cluster size)
 * Clusters hold 1..16 rows (the mask is 16 bits).  max_cluster is the
 * largest cluster size present.
 */
typedef struct hcsp_csr_cluster {
    int64_t nrows, ncols, nclusters, ncc, nslots;
    int32_t max_cluster;
    int32_t reserved;
    int64_t *cl_row_ptr;
    int32_t *perm;
    int64_t *cl_col_ptr;
    int32_t *cl_col;
    uint16_t *cl_mask;
    int64_t *cl_val_ptr;
    double *cl_val;
} hcsp_csr_cluster;

enum { HCSP_OP_CSR = 0, HCSP_OP_CLUSTER = 1 };

/* The left operand A: plain CSR (kind HCSP_OP_CSR, field csr) or CSR_Cluster
 * (kind HCSP_OP_CLUSTER, field cl). */
typedef struct hcsp_operand {
    int32_t kind;
    int32_t reserved;
    hcsp_csr csr;
    hcsp_csr_cluster cl;
} hcsp_operand;

/* Exact rational threshold num/den (den > 0), so similarity comparisons are
 * done in integers. */
typedef struct hcsp_ratio {
    int32_t num, den;
} hcsp_ratio;

/* Product options.  Zero-initialised means: defaults, whole matrix. */
enum {
    HCSP_F_SYNC_CHECK = 1,  /* numeric: synchronize and report out-of-range writes as HCSP_E_CAPACITY */
    HCSP_F_ONE_STREAM = 2   /* every launch on the caller's stream (by default the bins of a phase are
                               spread over side streams forked from it and joined back into it) */
};
typedef struct hcsp_opts {
    int32_t lanes;          /* lanes per row/cluster: 0 = automatic (one 64-lane wavefront) or 64 */
    int32_t flags;          /* HCSP_F_* */
    int64_t unit_lo;        /* numeric: first unit (row of a CSR A, cluster of a CSR_Cluster A) */
    int64_t unit_hi;        /* numeric: one past the last unit; <= 0 means all units */
    int64_t out_base;       /* numeric: C_col_d/C_val_d point at global entry out_base of C */
    int32_t dense_slots;    /* concurrent dense accumulators for units of a batch too long for shared
                               memory: 0 = as many as fit in 4 GiB (32..1024) */
    int32_t load_pct;       /* numeric hash-table fill target in percent: 0 = default (60) */
    int32_t sym_tmax_log2;  /* largest shared-memory symbolic table, log2 slots: 0 = default */
    int32_t num_tmax;       /* largest shared-memory numeric table, slots: 0 = default */
    int32_t sym_load_pct;   /* symbolic tables get >= products*100/sym_load_pct slots (products: the
                               unit's upper bound on distinct columns), 10..100: 0 = default (70) */
    int32_t win_chunk_log2; /* rows of units too long for shared memory (single products) are cut into
                               about products / 2^this column chunks (1..256), counted per chunk by the
                               symbolic phase and computed one workgroup per chunk by the numeric phase:
                               0 = default (18), else 4..30; the numeric call must use the symbolic
                               call's value */
} hcsp_opts;

#define HCSP_MAX_BINS 96

/* What the symbolic phase learned, handed to the numeric phase. */
typedef struct hcsp_sym_info {
    int64_t nnz;                       /* nnz(C) */
    int64_t units;                     /* rows (CSR A) or clusters (CSR_Cluster A) */
    int64_t sym_bin_count[HCSP_MAX_BINS];
    int64_t num_bin_count[HCSP_MAX_BINS];
    int32_t lanes;                     /* lanes per group actually used */
    int32_t valid;                     /* set to 1 by hcsp_spgemm_symbolic */
    int32_t load_pct;                  /* numeric table fill the bins were chosen for */
    int32_t win_chunk_log2;            /* column-chunk size the long rows were counted with */
} hcsp_sym_info;

/* -------------------------------------------------------------- library */

const char *hcsp_version(void);
const char *hcsp_strerror(int status);
/* Detail of the last error on this host thread ("" if none). */
const char *hcsp_last_error(void);

/*
 * Validate a device CSR matrix: row_ptr[0] == 0, non-decreasing,
 * row_ptr[nrows] == nnz (else HCSP_E_PTR); every column in [0, ncols)
 * (else HCSP_E_RANGE); strictly increasing within each row (else
 * HCSP_E_UNSORTED).  ws_d: >= 64 bytes of device scratch.  Synchronizes.
 */
int hcsp_csr_check(const hcsp_csr *A, void *ws_d, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------- cluster plans
 * Plans run on HOST copies of A (every pointer in A_h is a host pointer; val
 * may be NULL).  They work on A's rows in the order perm_in_h gives
 * (position p holds original row perm_in_h[p]; NULL = identity) and report
 * clusters as consecutive position ranges: cluster c holds original rows
 * perm_out_h[cl_row_ptr_h[c] .. cl_row_ptr_h[c+1]).  perm_out_h has nrows
 * entries and cl_row_ptr_h nrows+1; *ncl receives the cluster count.
 * max_cluster is 1..16.
 */

/* Fixed-length clusters (paper, "Fixed-length Clusters"): consecutive blocks
 * of K rows; the last block holds the remainder. */
int hcsp_plan_fixed(int64_t nrows, int32_t K, const int32_t *perm_in_h,
                    int32_t *perm_out_h, int64_t *cl_row_ptr_h, int64_t *ncl);

/* Variable-length clusters (paper, Alg. 2): a row joins the open cluster
 * while its Jaccard similarity to the cluster's first row is >= jacc_th and
 * the cluster has fewer than max_cluster rows. */
int hcsp_plan_variable(const hcsp_csr *A_h, hcsp_ratio jacc_th, int32_t max_cluster,
                       const int32_t *perm_in_h, int32_t *perm_out_h, int64_t *cl_row_ptr_h,
                       int64_t *ncl);

enum { HCSP_SIM_ROOT = 0, HCSP_SIM_UNION = 1 };
/*
 * Hierarchical clusters (paper, Alg. 3): candidate pairs from
 * SpGEMM_TopK(A, A^T) with topk = max_cluster-1 and similarity strictly above
 * jacc_th; a max-heap of candidates and a union-find forest; two roots merge
 * while the merged size stays within max_cluster; a popped non-root pair is
 * lifted to its roots and re-scored (HCSP_SIM_ROOT: the root rows' patterns;
 * HCSP_SIM_UNION: the union of each cluster's rows).  Clusters are ordered by
 * smallest member position, members ascending.  nthreads host threads
 * compute the candidate pairs (<= 0: all available).
 */
int hcsp_plan_hierarchical(const hcsp_csr *A_h, hcsp_ratio jacc_th, int32_t max_cluster,
                           uint32_t sim_flags, int32_t nthreads, const int32_t *perm_in_h,
                           int32_t *perm_out_h, int64_t *cl_row_ptr_h, int64_t *ncl);

/* ------------------------------------------------------ CSR_Cluster build
 * Device construction of the CSR_Cluster form of A (paper, the
 * A_CSR_CLUSTER(A_CSR, clusters) step of Alg. 2 and Alg. 3).
 * Step 1, hcsp_cluster_count: given perm_d[nrows] and cl_row_ptr_d[ncl+1]
 * (a plan copied to the device), writes cl_col_ptr_d[ncl+1] and
 * cl_val_ptr_d[ncl+1] and returns the sizes ncc, nslots and the largest
 * cluster size on the host.  Synchronizes.  ws_d needs
 * hcsp_cluster_workspace() bytes.
 * Step 2, hcsp_cluster_fill: with out->cl_col/cl_mask/cl_val allocated to
 * those sizes and the other out fields set (the pointer arrays from step 1),
 * fills the union columns, masks and values.  Asynchronous.
 */
int hcsp_cluster_workspace(int64_t nrows, int64_t ncl, size_t *bytes);
int hcsp_cluster_count(const hcsp_csr *A, const int32_t *perm_d, const int64_t *cl_row_ptr_d,
                       int64_t ncl, int64_t *cl_col_ptr_d, int64_t *cl_val_ptr_d,
                       int64_t *ncc_h, int64_t *nslots_h, int32_t *max_cluster_h,
                       void *ws_d, size_t ws_bytes, void *stream);
int hcsp_cluster_fill(const hcsp_csr *A, const hcsp_csr_cluster *out, void *stream);

/* ---------------------------------------------------------------- SpGEMM
 * hcsp_spgemm_workspace: device workspace bytes for C = A x B.  Host only.
 *
 * hcsp_spgemm_symbolic: the symbolic phase (paper, "SpGEMM Kernel").
 * Writes C_row_ptr_d[A.nrows+1] (offsets of C in A's original row order) and
 * fills *info (host).  Synchronizes twice: after binning, because the host
 * sizes each bin's launch (table size and grid) from the bin counts, and to
 * read nnz(C).  A product that must be captured into a graph runs through
 * hcsp_spgemm_batched (a batch of one), whose launches read the bin counts
 * from device memory.
 * Rows of units too long for shared memory are counted in (row, column
 * chunk) pairs whose counts the workspace keeps (room for 4 per row plus
 * 2^22); HCSP_E_CAPACITY if a product needs more (a larger
 * opts->win_chunk_log2 gives fewer chunks).
 *
 * hcsp_spgemm_numeric: the numeric phase.  C_col_d/C_val_d hold `capacity`
 * entries starting at global entry opts->out_base, so a caller can compute
 * C in panels of units (opts->unit_lo/unit_hi).  `info` must come from the
 * hcsp_spgemm_symbolic call on the same A, B, opts and workspace, and the
 * workspace must not have been touched since.  Asynchronous unless
 * HCSP_F_SYNC_CHECK is set.
 *
 * hcsp_spgemm_status: the errors the kernels of the last numeric call on
 * this workspace recorded (hcsp_spgemm_numeric, _numeric_cluster,
 * _predicted; the symbolic phase clears them): HCSP_E_CAPACITY when an
 * output write fell outside the capacity given (the write was dropped),
 * HCSP_E_INVALID when a row's count differs from the symbolic phase's (the
 * inputs changed in between) or the long rows' chunk counts are missing.
 * Reads 4 bytes at offset 0 of ws_d; synchronizes.
 */
int hcsp_spgemm_workspace(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts,
                          size_t *bytes);
int hcsp_spgemm_symbolic(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts,
                         int64_t *C_row_ptr_d, hcsp_sym_info *info, void *ws_d, size_t ws_bytes,
                         void *stream);
int hcsp_spgemm_numeric(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts,
                        const hcsp_sym_info *info, const int64_t *C_row_ptr_d, int32_t *C_col_d,
                        double *C_val_d, int64_t capacity, void *ws_d, size_t ws_bytes,
                        void *stream);
int hcsp_spgemm_status(const void *ws_d, size_t ws_bytes, void *stream);

/*
 * hcsp_spgemm_noalloc: for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The whole product C = A x B -- hcsp_spgemm_symbolic, the
 * nnz(C) read-back and hcsp_spgemm_numeric, with the same kernels and the
 * same result bit for bit -- with its workspace in a static device array of
 * HCSP_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends, instead of a caller-provided ws_d.  It calls no
 * hipMalloc/hipFree and creates no streams: every launch runs on `stream`
 * (HCSP_F_ONE_STREAM is implied; unit_lo/unit_hi/out_base are ignored, the
 * whole matrix is computed).
 *   C_row_ptr_d[A.nrows+1]    written (offsets of C in A's original row order)
 *   C_col_d/C_val_d           caller-allocated, `capacity` entries
 *   nnz_h                     (nullable) receives nnz(C), -1 if the symbolic
 *                             phase did not run
 * Errors: HCSP_E_CAPACITY when the product's workspace
 * (hcsp_spgemm_workspace) exceeds the static array (nothing runs; about
 * 5.1e5 rows for a square CSR A times a B of the same size on a device of
 * 256 compute units: 32 MiB of it are the long-row path's chunk counts and
 * carried positions) or when nnz(C) >
 * capacity (then only C_row_ptr_d and *nnz_h are written); the numeric
 * phase's own errors as hcsp_spgemm_status reports them.  Synchronizes.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents (each call clears what must start at zero): calls that
 * overlap on one device, from several host threads or streams, race.
 */
#define HCSP_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int hcsp_spgemm_noalloc(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts, int64_t *C_row_ptr_d,
                        int32_t *C_col_d, double *C_val_d, int64_t capacity, int64_t *nnz_h, void *stream);

/*
 * C in CSR_Cluster form (paper, Alg. 1, which writes C cluster by cluster):
 * for a CSR_Cluster A, C keeps A's clusters (cl_row_ptr and perm are A's),
 * and per cluster holds the sorted union of its member rows' output columns,
 * a member mask per union column and the member values column by column
 * (+0.0 where a member lacks the column), the layout of hcsp_csr_cluster.
 * Such a C can be the left operand of a further product without a new plan.
 *
 * hcsp_cluster_output_layout: after hcsp_spgemm_symbolic on the same A, B,
 * opts and workspace, writes cl_col_ptr_d[nclusters+1] and
 * cl_val_ptr_d[nclusters+1] (device) and returns ncc and nslots (host) so
 * the caller can allocate cl_col (int32 [ncc]), cl_mask (uint16 [ncc]) and
 * cl_val (double [nslots]).  Synchronizes.  HCSP_E_UNSUPPORTED when a
 * cluster's union did not fit a shared-memory table (its rows take the
 * column-window path, which writes CSR only).
 *
 * hcsp_spgemm_numeric_cluster: the numeric phase writing C as CSR_Cluster.
 * C: nrows, nclusters as A's, ncols = B.ncols, ncc and nslots from the
 * layout call (the capacities of its arrays), cl_col_ptr/cl_val_ptr as the
 * layout call wrote them; cl_row_ptr/perm are not read.  Same info and
 * workspace rules as hcsp_spgemm_numeric.  Synchronizes; HCSP_E_CAPACITY if
 * the arrays are too small, HCSP_E_INVALID if the counts changed.
 */
int hcsp_cluster_output_layout(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts,
                               const hcsp_sym_info *info, int64_t *cl_col_ptr_d, int64_t *cl_val_ptr_d,
                               int64_t *ncc_h, int64_t *nslots_h, void *ws_d, size_t ws_bytes, void *stream);
int hcsp_spgemm_numeric_cluster(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts,
                                const hcsp_sym_info *info, const hcsp_csr_cluster *C, void *ws_d,
                                size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- predicted sizes
 * A product without a symbolic phase in front: every row's output count is
 * predicted as capacity_i = min(p_i, ceil(p_i * ratio)), p_i the row's
 * product count (an upper bound on its count) and ratio a predicted
 * compression nnz(C)/products with margin (e.g. from the learned predictor);
 * the numeric phase runs with hash tables sized for capacity_i and writes
 * into a padded scratch.  (The learned predictor has one compression-ratio
 * head per matrix, so this entry takes one ratio and derives the per-row
 * capacities on the device; hcsp_spgemm_predicted_rows below takes them per
 * row.)  Rows whose keys do not fit are recomputed exactly:
 * the symbolic phase runs for those rows only (the exact fallback), then the
 * numeric phase.  Finally the predicted rows move to their exact places.  The
 * result is the same C as hcsp_spgemm_symbolic + hcsp_spgemm_numeric, bit
 * for bit.  CSR A only.
 *   hcsp_spgemm_products      products = sum over A's entries (i, k) of |B_k|
 *                             (device computation; ws_d >= 8 bytes;
 *                             synchronizes)
 *   hcsp_predicted_workspace  workspace bytes for (ratio, products); host only
 *   hcsp_spgemm_predicted     C_row_ptr_d[n+1] exact offsets, C_col_d/C_val_d
 *                             with capacity >= nnz(C) (else HCSP_E_CAPACITY
 *                             after nnz_h is set), nnz_h and n_overflow_h
 *                             (rows recomputed exactly; both nullable).
 *                             ratio in (0, 1].  Synchronizes. */
int hcsp_spgemm_products(const hcsp_csr *A, const hcsp_csr *B, int64_t *products_h, void *ws_d, size_t ws_bytes,
                         void *stream);
int hcsp_predicted_workspace(const hcsp_csr *A, const hcsp_csr *B, const hcsp_opts *opts, float ratio,
                             int64_t products, size_t *bytes);
int hcsp_spgemm_predicted(const hcsp_csr *A, const hcsp_csr *B, const hcsp_opts *opts, float ratio,
                          int64_t products, int64_t *C_row_ptr_d, int32_t *C_col_d, double *C_val_d,
                          int64_t capacity, int64_t *nnz_h, int64_t *n_overflow_h, void *ws_d, size_t ws_bytes,
                          void *stream);

/*
 * The same product with a capacity given per row instead of one ratio (a
 * per-row size predictor; exact counts from an earlier product with the same
 * pattern).  Row i's capacity is cap_row_d[i] clamped to [1, p_i]; the
 * result is again the C of the two-phase product bit for bit, and the rows
 * recomputed exactly are those whose count exceeds their capacity (or whose
 * table would not fit in shared memory).
 *   cap_row_d[A.nrows]             int32, device, read only
 *   cap_sum                        >= the sum of the positive cap_row_d[i]
 *                                  (sizes the padded scratch: cap_sum +
 *                                  A.nrows entries)
 *   hcsp_predicted_rows_workspace  workspace bytes for cap_sum; host only
 * Other arguments and synchronization as hcsp_spgemm_predicted.  Errors:
 * HCSP_E_INVALID when the clamped capacities need more scratch than cap_sum
 * declares (detected before any numeric launch; nothing is written but
 * C_row_ptr_d).
 */
int hcsp_predicted_rows_workspace(const hcsp_csr *A, const hcsp_csr *B, const hcsp_opts *opts, int64_t cap_sum,
                                  size_t *bytes);
int hcsp_spgemm_predicted_rows(const hcsp_csr *A, const hcsp_csr *B, const hcsp_opts *opts,
                               const int32_t *cap_row_d, int64_t cap_sum, int64_t *C_row_ptr_d, int32_t *C_col_d,
                               double *C_val_d, int64_t capacity, int64_t *nnz_h, int64_t *n_overflow_h, void *ws_d,
                               size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- orderings
 * Row orderings applied before row-wise or cluster-wise SpGEMM (paper, Sec.
 * "Matrix Reordering" and its table of reordering algorithms), on host
 * copies of A (A_h: host arrays).  perm_out_h[n] receives the order:
 * position p holds original row perm_out_h[p].  Host only; allocate host
 * memory only.
 *   hcsp_order_rcm     reverse Cuthill-McKee on the pattern of A + A^T
 *                      (square A): per connected component a
 *                      pseudo-peripheral start found from the least
 *                      (degree, id) unvisited vertex by repeated
 *                      breadth-first level structures; breadth-first visit
 *                      of neighbours by ascending (degree, id); the whole
 *                      sequence reversed.
 *   hcsp_order_degree  rows by descending length, ties by ascending id.
 * hcsp_permute_h: out = A with new row r = old row rperm_h[r] and new column
 * c = old column cperm_h[c] (NULL = identity), rows re-sorted by column;
 * out's arrays (host) are caller-allocated with A's sizes.  For a symmetric
 * reordering pass the same order twice: the product of the reordered
 * matrices is P C P^T.  nthreads host threads (<= 0: one). */
int hcsp_order_rcm(const hcsp_csr *A_h, int32_t *perm_out_h);
int hcsp_order_degree(const hcsp_csr *A_h, int32_t *perm_out_h);
int hcsp_permute_h(const hcsp_csr *A_h, const int32_t *rperm_h, const int32_t *cperm_h, hcsp_csr *out_h,
                   int32_t nthreads);

/*
 * hcsp_csr_transpose: At = A^T on the device (paper, Alg. 3 forms the
 * transpose of A for SpGEMM_TopK(A, A^T)).  At->nrows = A->ncols, At->ncols =
 * A->nrows, At->nnz = A->nnz; At->row_ptr[A->ncols+1] and At->col[nnz] are
 * caller-allocated and written with ascending columns per row; At->val is
 * written too when it is not NULL (then A->val must be set), else only the
 * pattern is formed.  ws_d: hcsp_csr_transpose_workspace(A->nrows, A->ncols)
 * bytes.  Asynchronous.
 */
int hcsp_csr_transpose_workspace(int64_t nrows, int64_t ncols, size_t *bytes);
int hcsp_csr_transpose(const hcsp_csr *A, hcsp_csr *At, void *ws_d, size_t ws_bytes, void *stream);

/*
 * hcsp_topk_candidates: the candidate search of the hierarchical plan
 * (paper, Alg. 3, SpGEMM_TopK) on the GPU.  O (device CSR, n x n) is the
 * overlap matrix A A^T of A's pattern: O_ij = number of columns rows i and j
 * share, e.g. the library's own product of A's pattern (all values 1) with
 * its transpose from hcsp_csr_transpose.  a_rp_d: A's row offsets (row
 * lengths |S_i|).  pos_d[n]: position of each row in the plan order (the
 * inverse of perm_in; NULL = identity).  For every row i, the partners j != i
 * with J = O_ij / (|S_i| + |S_j| - O_ij) strictly above jacc_th, best first
 * by (J descending, position ascending), at most topk (1..15) of them, go to
 * position p = pos(i): cnt_d[p] partners, their positions in
 * nbr_d[p*topk ..] and overlaps in ov_d[p*topk ..] (int64).  Exact integer
 * comparisons.  Asynchronous.
 *
 * hcsp_plan_hierarchical_candidates: hcsp_plan_hierarchical with the
 * candidate lists given (host copies of hcsp_topk_candidates' outputs, topk =
 * max_cluster - 1): only the merge loop runs on the host; same result.
 */
int hcsp_topk_candidates(const hcsp_csr *O, const int64_t *a_rp_d, const int32_t *pos_d, hcsp_ratio jacc_th,
                         int32_t topk, int32_t *cnt_d, int32_t *nbr_d, int64_t *ov_d, void *stream);
int hcsp_plan_hierarchical_candidates(const hcsp_csr *A_h, hcsp_ratio jacc_th, int32_t max_cluster,
                                      uint32_t sim_flags, const int32_t *perm_in_h, const int32_t *cnt_h,
                                      const int32_t *nbr_h, const int64_t *ov_h, int32_t *perm_out_h,
                                      int64_t *cl_row_ptr_h, int64_t *ncl);

/* ---------------------------------------------------------------- features
 * HCSP_NFEATURES structure-only features of the product A x B from host
 * copies of the patterns (A_h, B_h: host arrays; values are not read), for
 * the autotuner's matrix classes and the learned path selector.  The paper
 * finds that the gain of clustering and reordering depends on the sparsity
 * pattern (Sec. "Evaluation") and proposes learning the choice (Sec.
 * "Conclusion and Future Work"); the feature list itself is this library's:
 *   0 log2(n+1)           1 log2(nnz+1)          2 mean row length
 *   3 std row length      4 log2(max row len+1)  5..9 log2(row length+1) at
 *   the 10/25/50/75/90% quantiles                10 log2(sum of products+1)
 *   11 log2(mean products per row+1)             12 coefficient of variation
 *   of products per row   13 log2(max products per row+1)
 *   14/15 mean/std of |col - row| / ncols        16 mean Jaccard of rows
 *   (i, i+1) over <= 4096 evenly spaced i        17/18 fraction of those
 *   pairs with J >= 0.3 / 0.5                    19 column compression of
 *   the pairs with J >= 0.3: (|S_i|+|S_i+1|)/|S_i u S_i+1|
 *   20 padding of fixed-length clusters of 8: 8|union|/sum|S_i| over <= 512
 *   blocks               21 mean over <= 256 sampled rows of the best
 *   Jaccard with any row sharing a column (<= 64 rows per column)
 *   22 products / distinct output columns over the sampled rows
 *   23 fraction of empty rows  24..29 fraction of rows whose product count
 *   is < 64, < 256, < 1024, < 4096, < 16384, larger  30 log2(B.ncols+1)
 *   31 fraction of rows longer than twice the mean
 * out[HCSP_NFEATURES] receives float32 values.  Host only. */
#define HCSP_NFEATURES 32
int hcsp_features(const hcsp_csr *A_h, const hcsp_csr *B_h, float *out);

/* ---------------------------------------------------------------- learned selector
 * A 32-64-64-5 multilayer perceptron in float32 that, from the structure
 * features above, scores the product paths (logits z[0..3]) and predicts the
 * log compression ratio log(nnz(C) / products) (z[4]); it is trained on the
 * GPU with these kernels.  The paper proposes learning the reordering and
 * clustering choice as future work (Sec. "Conclusion and Future Work"); the
 * model is this library's.
 *   x_n = (x - mu) / sd;  h1 = relu(W1 x_n + b1);  h2 = relu(W2 h1 + b2);
 *   z = W3 h2 + b3;
 *   loss = mean_b(-log softmax(z_b[0..3])[y_b]) + lam * mean_b((z_b[4] - t_b)^2)
 * Device arrays (float32 unless noted):
 *   params_d[HCSP_MLP_NPARAMS]  W1 (64x32 row-major), b1 (64), W2 (64x64),
 *                               b2 (64), W3 (5x64), b3 (5)
 *   norm_d[2*32]                mu then sd of the features
 *   X_d[B*32], Z_d[B*5]
 *   act_d[B*HCSP_MLP_NACT]      per sample: x_n (32), W1 x_n + b1 (64),
 *                               W2 h1 + b2 (64); written by forward when not
 *                               NULL, read by backward
 *   y_d[B] (int32 class), t_d[B] (target log ratio), loss_d[B] (per-sample
 *   loss), delta_d[B*HCSP_MLP_NDELTA] (scratch), grad_d[HCSP_MLP_NPARAMS]
 * hcsp_mlp_adam applies one Adam step (step >= 1, bias-corrected) to params
 * with moment arrays m_d, v_d[HCSP_MLP_NPARAMS] (zero before step 1).  All
 * three run on the stream and never synchronize. */
#define HCSP_MLP_NIN 32
#define HCSP_MLP_NH 64
#define HCSP_MLP_NOUT 5
#define HCSP_MLP_NCLS 4
#define HCSP_MLP_NPARAMS 6597
#define HCSP_MLP_NACT 160
#define HCSP_MLP_NDELTA 133
int hcsp_mlp_forward(const float *params_d, const float *norm_d, const float *X_d, int32_t B, float *Z_d,
                     float *act_d, void *stream);
int hcsp_mlp_backward(const float *params_d, const float *act_d, const float *Z_d, const int32_t *y_d,
                      const float *t_d, int32_t B, float lam, float *delta_d, float *loss_d, float *grad_d,
                      void *stream);
int hcsp_mlp_adam(float *params_d, const float *grad_d, float *m_d, float *v_d, int32_t step, float lr, float beta1,
                  float beta2, float eps, void *stream);

/*
 * hcsp_mlp_train_step: one full-batch training step on the device -- forward
 * (act_d required), back-propagation and one Adam step with the arrays and
 * meanings above.  Never synchronizes.
 *
 * The model on the host (hcsp_mlp, opaque): the parameters, the feature
 * normalization (mu then sd) and a one-line tag (e.g. the path names the
 * selector head scores).  The library allocates host memory only.
 *   hcsp_mlp_create   copies params_h[HCSP_MLP_NPARAMS] (NULL: zeros) and
 *                     norm_h[2*HCSP_MLP_NIN] (NULL: mu 0, sd 1); tag NULL = ""
 *   hcsp_mlp_get/set  copy out / in (NULL arguments are skipped); get's tag
 *                     buffer needs the tag's length + 1 bytes
 *   hcsp_mlp_save/load  a text file (layer sizes, tag, normalization and
 *                     parameters to 9 significant digits: exact for float32);
 *                     load refuses a file of another shape
 *   hcsp_mlp_destroy  frees it (NULL is a no-op)
 */
typedef struct hcsp_mlp hcsp_mlp;
int hcsp_mlp_train_step(float *params_d, const float *norm_d, const float *X_d, const int32_t *y_d, const float *t_d,
                        int32_t B, float lam, float *act_d, float *Z_d, float *delta_d, float *loss_d, float *grad_d,
                        float *m_d, float *v_d, int32_t step, float lr, float beta1, float beta2, float eps,
                        void *stream);
int hcsp_mlp_create(const float *params_h, const float *norm_h, const char *tag, hcsp_mlp **out);
int hcsp_mlp_destroy(hcsp_mlp *m);
int hcsp_mlp_get(const hcsp_mlp *m, float *params_h, float *norm_h, char *tag, size_t len);
int hcsp_mlp_set(hcsp_mlp *m, const float *params_h, const float *norm_h);
int hcsp_mlp_save(const hcsp_mlp *m, const char *path);
int hcsp_mlp_load(const char *path, hcsp_mlp **out);

/* ---------------------------------------------------------------- autotuner
 * Tuned options per matrix class.  The paper fixes the clustering parameters
 * (similarity threshold 0.3, at most 8 rows per cluster, Sec. "Hierarchical
 * Clusters") and notes that the best cluster length depends on the matrix
 * (Sec. "Clustering Without Changing Order"); here they are measured per
 * class of matrices instead.  Host only; the library allocates host memory
 * only.
 *
 * Class of a matrix: five of the structure features (hcsp_features) cut at
 * fixed edges -- mean row length (feature 2; edges 6, 16, 40), coefficient of
 * variation of the products per row (12; 0.5, 2), products per distinct output
 * column of the sampled rows (22; 1.3, 3), the best similarity a row finds
 * (21; 0.3, 0.6) and mean |col - row| / ncols (14; 0.05) -- as the key
 * "rl<a>_cv<b>_cr<c>_sim<d>_loc<e>", each digit the number of edges at or
 * below the feature's value (hcsp_tune_class; key buffer >= 32 bytes).
 *
 * A run is one matrix's measured product times (ms per product: symbolic
 * phase, nnz read-back and numeric phase; NaN or <= 0 = not measured) on a
 * fixed grid:
 *   plain_ms[i][j]  plain CSR, symbolic fill {50,70,100}[i] (opts.sym_load_pct),
 *                   numeric fill {50,60,70}[j] (opts.load_pct)
 *   rcm_ms          plain CSR over reverse Cuthill-McKee rows (recorded, not
 *                   used by the choice)
 *   hc_ms[i][j]     CSR_Cluster of hierarchical clusters (Alg. 3, threshold
 *                   3/10) of at most {2,4,8}[i] rows over RCM rows, numeric
 *                   fill {50,60,70,75,80,85}[j]
 * Choice of a class, over the candidates every one of its runs measured: a
 * candidate's score is the sum over the runs of its time divided by the run's
 * best time (over the plain grid and every cluster size at its best fill);
 * sym_load_pct/load_pct are the best-scoring plain candidate's fills; each
 * cluster size scores with its best fill per run, and the best-scoring size is
 * best_cluster_size, its best-scoring fill cl_load_pct; the path is that
 * cluster size (path 1, max_cluster) if it scores strictly lower than the
 * plain candidate, else plain (path 0, max_cluster 0).  Ties go to the first
 * candidate in grid order.  A class without runs gets the library defaults:
 * tuned 0, plain, fills 70 and 60, best_cluster_size 2, cl_load_pct 60.
 *
 *   hcsp_tune_create/destroy  an empty table / free it (NULL is a no-op)
 *   hcsp_tune_add      appends a run to a class (key from hcsp_tune_class)
 *   hcsp_tune_get      the choice of the class with that key
 *   hcsp_tune_lookup   the choice of the class of a matrix's features
 *   hcsp_tune_classes  the class keys, one per line (keys may be NULL to get
 *                      the count only)
 *   hcsp_tune_runs     a class's runs (*count set; runs NULL: the count only;
 *                      HCSP_E_CAPACITY if more than cap)
 *   hcsp_tune_save/load  a text file: header with the grid shape, per class a
 *                      line "class <key> <runs>" and one line per run (17
 *                      significant digits, "nan" where not measured)
 */
#define HCSP_TUNE_NSYM 3
#define HCSP_TUNE_NNUM 3
#define HCSP_TUNE_NMC 3
#define HCSP_TUNE_NCL 6
typedef struct hcsp_tune_run {
    int64_t nrows, nnz;
    double plain_ms[HCSP_TUNE_NSYM][HCSP_TUNE_NNUM];
    double rcm_ms;
    double hc_ms[HCSP_TUNE_NMC][HCSP_TUNE_NCL];
} hcsp_tune_run;
typedef struct hcsp_tune_choice {
    int32_t tuned;             /* 0: no runs for the class (defaults) */
    int32_t path;              /* 0 plain CSR, 1 hierarchical clusters over RCM rows */
    int32_t max_cluster;       /* rows per cluster of the chosen path (0 for plain) */
    int32_t best_cluster_size; /* best-scoring cluster size */
    int32_t sym_load_pct;      /* opts.sym_load_pct */
    int32_t load_pct;          /* opts.load_pct, plain CSR */
    int32_t cl_load_pct;       /* opts.load_pct, CSR_Cluster of best_cluster_size rows */
    int32_t runs;              /* runs of the class */
} hcsp_tune_choice;
typedef struct hcsp_tune_table hcsp_tune_table;
int hcsp_tune_create(hcsp_tune_table **out);
int hcsp_tune_destroy(hcsp_tune_table *t);
int hcsp_tune_class(const float *features, char *key, size_t len);
int hcsp_tune_add(hcsp_tune_table *t, const char *key, const hcsp_tune_run *run);
int hcsp_tune_get(const hcsp_tune_table *t, const char *key, hcsp_tune_choice *out);
int hcsp_tune_lookup(const hcsp_tune_table *t, const float *features, hcsp_tune_choice *out);
int hcsp_tune_classes(const hcsp_tune_table *t, char *keys, size_t len, int32_t *count);
int hcsp_tune_runs(const hcsp_tune_table *t, const char *key, hcsp_tune_run *runs, int32_t cap, int32_t *count);
int hcsp_tune_save(const hcsp_tune_table *t, const char *path);
int hcsp_tune_load(const char *path, hcsp_tune_table **out);

/* ---------------------------------------------------------------- batches
 * Many independent products C_p = A_p x B_p of uneven sizes in one fixed
 * sequence of launches: the units (rows or clusters) of all products are
 * numbered consecutively, binned together, and every bin is processed by
 * one persistent launch whose wavefronts take slices of the bin.  Bin sizes
 * stay in device memory, so hcsp_spgemm_batched never synchronizes, copies
 * or allocates: it can be captured into a HIP graph and replayed.  (The
 * paper's row-wise product, Background "SpGEMM Kernel"; the batching is this
 * library's own.)
 *
 * Outputs are flat: product p's row offsets are the nrows_p + 1 entries of
 * C_row_ptr_d starting at seg_offset[p] (= sum over q < p of nrows_q + 1),
 * local to the product (starting at 0); its columns and values start at
 * out_offset[p] of C_col_d / C_val_d, where out_offset is the prefix sum of
 * the per-product upper bounds sum_i sum_{k in A_i} |B_k|, so they never
 * overflow.
 *
 * Use: hcsp_batch_plan_init (host only: sizes) -> allocate plan->ws_bytes
 * -> hcsp_batch_prepare (uploads the descriptors, computes the bounds;
 * synchronizes) -> allocate plan->out_capacity entries for C_col_d / C_val_d
 * and plan->row_ptr_len for C_row_ptr_d -> hcsp_spgemm_batched, any number
 * of times (capturable) -> hcsp_batch_status (per-product nnz and errors;
 * synchronizes).  The items' device arrays must stay valid and keep their
 * structure between prepare and the last batched call.
 */
typedef struct hcsp_batch_item {
    hcsp_operand A; /* device arrays; all items of a batch have the same kind */
    hcsp_csr B;     /* device arrays */
} hcsp_batch_item;

typedef struct hcsp_batch_plan {
    int32_t count;        /* products */
    int32_t kind;         /* HCSP_OP_CSR or HCSP_OP_CLUSTER */
    int64_t units;        /* rows (CSR) or clusters, over all products */
    int64_t rows;         /* rows of A over all products */
    int64_t row_ptr_len;  /* rows + count: entries of C_row_ptr_d */
    int64_t max_ncols;    /* widest B */
    int32_t max_class;    /* member-count class of the widest cluster (0 for CSR) */
    int32_t prepared;     /* set by hcsp_batch_prepare */
    int64_t max_probes;   /* largest per-unit product count (prepare) */
    int64_t out_capacity; /* entries of C_col_d / C_val_d (prepare) */
    size_t ws_bytes;      /* workspace bytes (plan_init) */
    hcsp_opts opts;       /* options the plan was made with */
} hcsp_batch_plan;

/* Host only: checks the items (host copies of the descriptors, device
 * arrays inside) and fills count, kind, units, rows, row_ptr_len,
 * max_ncols, max_class and ws_bytes.  opts may be NULL. */
int hcsp_batch_plan_init(int32_t count, const hcsp_batch_item *items_h, const hcsp_opts *opts,
                         hcsp_batch_plan *plan);
/* Uploads the descriptors into the workspace and computes every product's
 * output bound; fills plan->max_probes, plan->out_capacity and, when not
 * NULL, out_offset_h[count+1] and seg_offset_h[count+1].  Synchronizes. */
int hcsp_batch_prepare(hcsp_batch_plan *plan, const hcsp_batch_item *items_h, void *ws_d, size_t ws_bytes,
                       int64_t *out_offset_h, int64_t *seg_offset_h, void *stream);
/* Symbolic and numeric phases of every product.  Never synchronizes,
 * copies from the host or allocates (capture-safe).  Errors are recorded
 * per product in the workspace and reported by hcsp_batch_status. */
int hcsp_spgemm_batched(const hcsp_batch_plan *plan, int64_t *C_row_ptr_d, int32_t *C_col_d, double *C_val_d,
                        void *ws_d, size_t ws_bytes, void *stream);
/* nnz_h[count] (nullable) receives nnz(C_p); returns HCSP_E_CAPACITY or
 * HCSP_E_INVALID if a product of the last batched call flagged an error.
 * Synchronizes. */
int hcsp_batch_status(const hcsp_batch_plan *plan, void *ws_d, size_t ws_bytes, int64_t *nnz_h, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HCSP_H */
