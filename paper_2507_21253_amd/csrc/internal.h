// Host-side internals of libhcsp: error reporting, bin geometry, workspace
// layout and the kernel-launch interface between the host runtime and the
// gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/hcsp.h"

namespace hcsp {

// ------------------------------------------------------------ error reporting
void set_error(const std::string &msg);
void clear_error();
int fail(int code, const std::string &msg);

#define HCSP_HIP(call)                                                                 \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::hcsp::fail(HCSP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------ bin geometry
// Units (rows of a CSR A, clusters of a CSR_Cluster A) are sorted into bins
// before each phase.  A bin fixes the cluster-size class (S = 1, 2, 4, 8, 16)
// and the shared-memory table size, so one launch handles units of one
// shape.  Bin 0 holds units with no work; the last bin holds units too big
// for shared memory (the column-window path in single products, the dense
// global-memory path in batches).
constexpr int kSClasses = 5;                 // S = 1 << sclass
constexpr int kSymLog2Min = 6;               // symbolic tables: 64 .. 2^kSymLog2Max slots
constexpr int kSymLog2Max = 14;
constexpr int kSymT = kSymLog2Max - kSymLog2Min + 1;
constexpr int kNumT = 14;                    // numeric table sizes, see kNumTable
constexpr int kBinEmpty = 0;
constexpr int kSymBins = 2 + kSClasses * kSymT;   // + empty + global
constexpr int kNumBins = 2 + kSClasses * kNumT;
constexpr int kSymGlobal = kSymBins - 1;
constexpr int kNumGlobal = kNumBins - 1;
// numeric probe tail past the hashed range: short for small tables (space),
// longer for large ones, whose runs near the end would otherwise wrap
__host__ __device__ constexpr int num_tail(int T) { return T <= 256 ? 16 : 32; }
// keys a numeric table of T slots holds at most: a unit goes to the smallest
// table with U * 100 <= T * load_pct
__host__ __device__ constexpr int num_vcap(int T, int load_pct) { return (int)((int64_t)T * load_pct / 100); }
constexpr int kBinBlocks = 4096;            // blocks of the binning kernels
static_assert(kSymBins <= HCSP_MAX_BINS && kNumBins <= HCSP_MAX_BINS, "bin count");

__host__ __device__ inline int num_table(int t)
{
    // 64, 96, 128, 192, ... : powers of two and their 3/2 multiples
    return (t & 1) ? (3 << (5 + (t >> 1))) : (64 << (t >> 1));
}

__host__ __device__ inline int sclass_of(int s)
{
    return s <= 1 ? 0 : s <= 2 ? 1 : s <= 4 ? 2 : s <= 8 ? 3 : 4;
}

// Shared-memory bytes of one wavefront's tables (layouts in hash.hip).
int64_t sym_wave_bytes(int mask_bytes, int T);  // mask bytes per slot: 0 for one-row units
// mask bytes per slot of a member-count class (0: one row, 1: up to 8 rows, 2: 16)
inline int mask_bytes_of_class(int sc) { return sc == 0 ? 0 : (sc <= 3 ? 1 : 2); }
int64_t num_wave_bytes(bool cl, int sclass, int T, int load_pct);

// Tuning derived from hcsp_opts.
struct Tune {
    int G;               // lanes per unit (one wavefront)
    int load_pct;        // numeric table fill target
    int sym_load_pct;    // symbolic table fill bound (percent of the product count)
    int sym_tmax_log2;   // largest symbolic table
    int num_tmax;        // largest numeric table
    int dense_slots;     // concurrent dense accumulators
    int win_log2;        // column-window path: products per column chunk, log2
    int64_t lds_budget;  // shared memory per workgroup we plan for
    bool one_stream;     // every launch on the caller's stream (no side streams)
};

// ------------------------------------------------------------ workspace
struct Workspace {
    // per unit
    int64_t *probes;     // sum of |B_k| over the unit's columns
    int32_t *keylo, *keyhi;
    int32_t *ucount;     // distinct output columns of the unit (symbolic result)
    uint8_t *bin;        // current bin of the unit
    int32_t *order_sym, *order_num;
    // counters
    int64_t *sym_count;  // [HCSP_MAX_BINS]
    int64_t *num_count;
    int32_t *bin_hist;   // [kBinBlocks][HCSP_MAX_BINS] per-block bin counts, then scatter offsets
    uint32_t *err;       // error flags
    int64_t *scan_tmp;   // block sums of the scan
    // dense path
    uint32_t *dense_bits;
    double *dense_vals;
    int64_t dense_words; // 32-bit words per bitmap
    int dense_slots;
    // column-window path (rows of units too long for shared memory): the
    // distinct output columns of each (row, chunk) pair of the symbolic
    // window launch [win_cap]; per unit its first pair there [nunits]; per
    // unit of a window launch its first pair [nunits + 1]
    int32_t *chunk_cnt;
    int64_t *sym_base;
    int64_t *win_base;
    int64_t win_cap;
    // per wavefront of the numeric window launch (win_cur_slots of them), two
    // arrays of kWinCurMax positions in B (where each item's row of B reaches
    // the next window)
    int32_t *win_cur;
    int64_t win_cur_slots;
    // single products: the length of each row of B, saturated at 65535 (a
    // 2-byte array that the work estimate gathers from instead of pairs of
    // 8-byte row offsets; it stays in L2)
    uint16_t *b_len;
    size_t bytes;
};

// windows: single products, whose units too long for shared memory take the
// column-window path (chunk counts, no dense accumulators); otherwise
// (batches) dense_slots dense accumulators
size_t layout_workspace(int64_t nunits, int64_t nrows, int64_t ncols, int64_t brows, int dense_slots, bool windows,
                        char *base, Workspace *ws);

// ------------------------------------------------------------ batches
// One product of a batch as the kernels see it (device copy).  Units of all
// products are numbered consecutively (unit_base); C row offsets of product
// p occupy nrows+1 entries from seg_base of one flat array, and its columns
// and values start at out_base of the flat output arrays.
struct BatchProb {
    const int64_t *a_rp;
    const int32_t *a_col;
    const double *a_val;
    const int64_t *cl_row_ptr;
    const int32_t *perm;
    const int64_t *cl_col_ptr;
    const int32_t *cl_col;
    const uint16_t *cl_mask;
    const int64_t *cl_val_ptr;
    const double *cl_val;
    const int64_t *b_rp;
    const int32_t *b_col;
    const double *b_val;
    int64_t unit_base, nunits, seg_base, nrows, out_base, cap, ncols;
};

// ------------------------------------------------------------ kernel interface
struct SpArgs {
    // A as CSR
    const int64_t *a_rp;
    const int32_t *a_col;
    const double *a_val;
    // A as CSR_Cluster
    const int64_t *cl_row_ptr;
    const int32_t *perm;
    const int64_t *cl_col_ptr;
    const int32_t *cl_col;
    const uint16_t *cl_mask;
    const int64_t *cl_val_ptr;
    const double *cl_val;
    // B
    const int64_t *b_rp;
    const int32_t *b_col;
    const double *b_val;
    // units of this launch
    const int32_t *order;
    int64_t bin_begin, count;
    int32_t *keylo, *keyhi;    // smallest / largest output column of each unit (symbolic writes)
    int32_t *ucount;
    // C
    int64_t *c_rp;
    int32_t *c_col;
    double *c_val;
    int64_t cap, out_base;
    int64_t unit_lo, unit_hi;
    uint32_t *err;
    // geometry
    int G, T, log2T, group_bytes;
    int vcap;  // numeric, clusters of several rows: value entries per table (keys at most)
    // dense path
    uint32_t *dense_bits;
    double *dense_vals;
    int64_t dense_words;
    int64_t ncols;
    // column-window path: per-unit product counts, per-(unit, chunk) counts,
    // per-row first (row, chunk) pair of the launch
    const int64_t *probes;
    int32_t *chunk_cnt;
    int64_t *sym_base;
    int64_t *win_base;
    int64_t win_cap;
    int32_t *win_cur;
    int win_log2;
    // batch launches: the products, their unit bases [nprob+1], the bin's
    // unit count and start in device memory, per-product error words
    const BatchProb *batch;
    const int64_t *batch_units;
    int nprob, bin;
    const int64_t *dcount, *dbegin;
    uint32_t *errs;
    // predicted sizes: padded row starts (numeric writes there and stores its
    // row count, or -1 when the prediction was too small, into c_rp)
    const int64_t *pad_off;
    // numeric output in CSR_Cluster form with A's clusters (null oc_col: CSR
    // output): per cluster its sorted union columns, their member masks and
    // the member values column by column (+0.0 where a member lacks the column)
    const int64_t *oc_col_ptr, *oc_val_ptr;
    int32_t *oc_col;
    uint16_t *oc_mask;
    double *oc_val;
    int64_t oc_ncc, oc_nslots;  // capacities of oc_col/oc_mask and oc_val
};

// error flag bits
enum : uint32_t {
    kErrCapacity = 1u,
    kErrCount = 2u,
    kErrPtr = 4u,
    kErrRange = 8u,
    kErrUnsorted = 16u,
    kErrWindows = 32u,  // more (row, chunk) pairs than the workspace holds counts for
};

// launchers (kernels.hip)
// batch = true: persistent launches over a batch (unit ids are batch-wide,
// the bin's count and start are read from device memory)
hipError_t launch_sym(int sclass, bool cluster, bool batch, const SpArgs &a, int blocks, int threads, size_t lds,
                      hipStream_t s);
hipError_t launch_num(int sclass, bool cluster, bool batch, const SpArgs &a, int blocks, int threads, size_t lds,
                      hipStream_t s);
hipError_t launch_sym_dense(bool cluster, bool batch, const SpArgs &a, int blocks, hipStream_t s);
// numeric with predicted sizes (CSR rows): bounded probing, padded output
hipError_t launch_num_pred(const SpArgs &a, int blocks, int threads, size_t lds, hipStream_t s);
hipError_t launch_num_dense(bool cluster, bool batch, const SpArgs &a, int blocks, hipStream_t s);
// column-window path for units too long for shared memory: bitmaps of each
// row's output columns (a cluster's member rows one by one), one workgroup
// per unit (symbolic) or per (row, chunk) of the output columns (numeric),
// persistent over the bin; a unit of ub products gets about ub / 2^win_log2
// chunks per row
constexpr int kWinChunksMax = 256;
// items of a window row whose positions in B are carried from one window to
// the next (later items are found by binary search in every window)
constexpr int kWinCurMax = 1024;
// wavefronts of a workgroup of the bitmap kernels: symbolic (one unit per
// workgroup; its bitmap takes most of a compute unit's shared memory, so more
// wavefronts hide more of the latency of walking the products) and numeric
// (a row, or a column chunk of one, per workgroup; each wavefront also holds
// a window of values, so fewer of them fit beside the bitmap)
constexpr int kSymBmWaves = 16;
constexpr int kNumBmWaves = 8;
constexpr int kWinLog2Default = 18;
__host__ __device__ inline int win_nchunks(int64_t ub, int log2)
{
    const int64_t n = (ub + ((int64_t)1 << log2) - 1) >> log2;
    return (int)(n < 1 ? 1 : (n > kWinChunksMax ? kWinChunksMax : n));
}
hipError_t launch_win_prep(bool sym, bool cluster, const SpArgs &a, hipStream_t s);
int64_t sym_bm_bytes();
int64_t num_bm_bytes();
hipError_t launch_sym_bm(bool cluster, const SpArgs &a, int blocks, hipStream_t s);
hipError_t launch_num_bm(bool cluster, const SpArgs &a, int blocks, hipStream_t s);

// launchers (util.hip)
struct BinArgs {
    const int64_t *a_rp;
    const int32_t *a_col;
    const int64_t *cl_row_ptr;
    const int32_t *perm;
    const int64_t *cl_col_ptr;
    const int32_t *cl_col;
    const int64_t *b_rp;
    const int32_t *b_col;
    const uint16_t *b_len;  // nullable: B's row lengths, saturated at 65535
    int64_t nunits;
    Workspace ws;
    int64_t *c_rp;
    int sym_tmax_log2;
    int num_tmax_by_class[kSClasses];
    int load_pct;
    int sym_load_pct;
    // batch: unit ids are batch-wide; c_rp is the flat row-offset array
    const BatchProb *batch;
    const int64_t *batch_units;
    int nprob;
    // restriction to the units with active[u] != 0 (nullable: all units)
    const uint8_t *active;
    // predicted sizes: row capacity min(products, ceil(products * ratio)), or the
    // given one clamped to [1, products], into pad[]
    float ratio;
    const int32_t *cap_row;  // per-row capacities instead of the ratio (nullable)
    int64_t *pad;
    const int2 *b_span;  // predicted sizes: first and last column of each row of B (nullable)
};
hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
// Up to four device scalars (8- or 4-byte words, the latter zero-extended)
// gathered into dst[0..n), so that the host reads them back with the bin
// counts in one copy.
struct GatherWords {
    const void *src[4];
    int32_t bytes[4];
    int32_t n;
};
hipError_t launch_gather_words(int64_t *dst, const GatherWords &g, hipStream_t s);
// The symbolic phase's first launch: out[k] = min(rp[k+1] - rp[k], 65535)
// for k < n (B's row lengths), and zeros into the first nz words of z0 and
// of z1, into *err and into *z2.
hipError_t launch_sym_start(const int64_t *rp, int64_t n, uint16_t *out, int64_t *z0, int64_t *z1, int nz,
                            uint32_t *err, int64_t *z2, hipStream_t s);
hipError_t launch_work(bool cluster, const BinArgs &a, hipStream_t s);
hipError_t launch_numbin(bool cluster, const BinArgs &a, hipStream_t s);
// batches
// CSR_Cluster output layout: per cluster its union count and union count x
// members, [nunits] = 0 (exclusive scans then give the offsets and totals);
// a unit counted by column chunks (count INT32_MAX) sets *err.
hipError_t launch_cl_out_counts(const int32_t *ucount, const int64_t *cl_row_ptr, int64_t nunits, int64_t *colp,
                                int64_t *valp, uint32_t *err, hipStream_t s);
// SpGEMM_TopK: per row of the overlap matrix O (rows: original ids) the
// topk best partners above num/den; outputs at the row's position
hipError_t launch_topk(const int64_t *o_rp, const int32_t *o_col, const double *o_val, const int64_t *a_rp,
                       const int32_t *pos, int64_t n, int64_t num, int64_t den, int topk, int32_t *cnt, int32_t *nbr,
                       int64_t *nov, hipStream_t s);
hipError_t launch_max_i64(const int64_t *x, int64_t n, int64_t *out, hipStream_t s);
// predicted sizes
hipError_t launch_products(const hcsp_csr &A, const hcsp_csr &B, int64_t *out, hipStream_t s);
hipError_t launch_work_pred(const BinArgs &a, hipStream_t s);
// span[k] = (first, last) column of row k of B; (INT_MAX, -1) for an empty row
hipError_t launch_row_span(const int64_t *rp, const int32_t *col, int64_t n, int2 *span, hipStream_t s);
hipError_t launch_mark_overflow(const int64_t *c_rp, int64_t n, uint8_t *active, int64_t *count, hipStream_t s);
hipError_t launch_copy_rows(const int64_t *pad_off, const int32_t *scol, const double *sval, const int64_t *c_rp,
                            const uint8_t *active, int64_t n, int32_t *C_col, double *C_val, int64_t cap,
                            uint32_t *err, hipStream_t s);
hipError_t launch_bin_begin(const int64_t *counts, int nbins, int64_t *begin, hipStream_t s);
hipError_t launch_batch_bound(const BatchProb *batch, int nprob, bool cluster, int64_t *ub, hipStream_t s);
hipError_t launch_batch_seg_tail(const BatchProb *batch, int nprob, int64_t *flat, hipStream_t s);
hipError_t launch_batch_seg_rebase(const BatchProb *batch, const int64_t *segs, int nprob, int64_t *flat,
                                   int64_t nflat, int64_t *base, int64_t *nnz, hipStream_t s);
hipError_t launch_scatter(const uint8_t *bin, int64_t n, int32_t *hist, int nbins, int64_t *counts, int32_t *order,
                          hipStream_t s);
int bin_blocks(int64_t nunits);
hipError_t launch_scan_exclusive(int64_t *data, int64_t n, int64_t *tmp, hipStream_t s);
size_t scan_tmp_elems(int64_t n);
hipError_t launch_csr_check(const hcsp_csr &A, uint32_t *flags, hipStream_t s);

// launchers (transpose.hip): A^T of a device CSR matrix (values when At.val is set)
struct TrWs {
    int64_t *cursor;    // [ncols] next free slot of each row of A^T
    int32_t *mid, *lng; // [ncols] rows of A^T for the two larger sorts
    uint32_t *counts;   // [0] mid rows, [1] long rows
    uint32_t *bits;     // bitmaps over A's rows, one per long-row block
    int64_t words;      // 32-bit words per bitmap
    int64_t *scan_tmp;
};
size_t layout_transpose(int64_t nrows, int64_t ncols, char *base, TrWs *w);
hipError_t launch_transpose(const hcsp_csr &A, const hcsp_csr &At, const TrWs &w, hipStream_t s);

// launchers (cluster.hip)
hipError_t launch_cluster_count(const hcsp_csr &A, const int32_t *perm, const int64_t *cl_row_ptr, int64_t ncl,
                                int64_t *cl_col_cnt, int64_t *cl_val_cnt, int32_t *maxsize, hipStream_t s);
hipError_t launch_cluster_fill(const hcsp_csr &A, const hcsp_csr_cluster &out, hipStream_t s);

}  // namespace hcsp
