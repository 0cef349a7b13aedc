// C ABI of libhcsp: argument checks, workspace layout, bin dispatch and the
// two-phase SpGEMM orchestration (symbolic, then numeric) on one HIP stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace hcsp {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
void clear_error() { g_err.clear(); }
int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static int64_t num_bm_blocks();

size_t layout_workspace(int64_t nunits, int64_t nrows, int64_t ncols, int64_t brows, int dense_slots, bool windows,
                        char *base, Workspace *ws)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        off = align_up(off, 256);
        void *p = base ? (void *)(base + off) : nullptr;
        off += bytes;
        return p;
    };
    const size_t nu = (size_t)std::max<int64_t>(nunits, 1);
    ws->err = (uint32_t *)take(256);  // first: hcsp_spgemm_status reads it at offset 0
    ws->probes = (int64_t *)take(8 * nu);
    ws->keylo = (int32_t *)take(4 * nu);
    ws->keyhi = (int32_t *)take(4 * nu);
    ws->ucount = (int32_t *)take(4 * nu);
    ws->bin = (uint8_t *)take(nu);
    ws->order_sym = (int32_t *)take(4 * nu);
    ws->order_num = (int32_t *)take(4 * nu);
    ws->sym_count = (int64_t *)take(8 * HCSP_MAX_BINS);
    ws->num_count = (int64_t *)take(8 * HCSP_MAX_BINS);
    ws->bin_hist = (int32_t *)take(4 * (size_t)kBinBlocks * HCSP_MAX_BINS);
    ws->scan_tmp = (int64_t *)take(8 * scan_tmp_elems(std::max(nrows, nunits) + 1));
    ws->dense_words = (std::max<int64_t>(ncols, 1) + 31) / 32;
    ws->dense_slots = windows ? 0 : dense_slots;
    ws->dense_bits = (uint32_t *)take(4 * (size_t)ws->dense_words * ws->dense_slots);
    ws->dense_vals = (double *)take(8 * (size_t)std::max<int64_t>(ncols, 1) * ws->dense_slots);
    // counts of the symbolic window launch's (row, chunk) pairs: room for 4
    // per row plus 4M (chunks follow the products, about products / 2^16 per
    // unit; a launch that needs more fails with HCSP_E_CAPACITY)
    ws->win_cap = windows ? 4 * std::max<int64_t>(nrows, nunits) + (1 << 22) : 0;
    ws->chunk_cnt = (int32_t *)take(4 * (size_t)ws->win_cap);
    ws->sym_base = (int64_t *)take(windows ? 8 * nu : 0);
    ws->win_base = (int64_t *)take(windows ? 8 * (nu + 1) : 0);
    ws->win_cur_slots = windows ? num_bm_blocks() * kNumBmWaves : 0;
    ws->win_cur = (int32_t *)take(4 * 2 * (size_t)kWinCurMax * (size_t)ws->win_cur_slots);
    ws->b_len = (uint16_t *)take(windows ? 2 * (size_t)std::max<int64_t>(brows, 1) : 0);
    ws->bytes = align_up(off, 256);
    return ws->bytes;
}

// Compute units of the current device (queried once per device).
static int cu_count()
{
    static std::mutex mu;
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (!cache[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cache[dev] = v;
    }
    return cache[dev];
}

// Shared memory per workgroup the bins may plan for (queried once per device).
static int64_t lds_limit()
{
    static std::mutex mu;
    static int64_t cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
    std::lock_guard<std::mutex> lk(mu);
    if (!cache[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 64 * 1024;
        cache[dev] = std::min<int64_t>(v, 160 * 1024);
    }
    return cache[dev];
}

// Side streams for the bins of a phase.  The bin with the most work runs on
// the caller's stream, launched first (its start is the phase's critical
// path; queueing the other launches first delayed it by their host time),
// the others on side streams forked from it and joined back before the
// phase's next step, so that the few long units of a small bin overlap the
// large bin instead of running alone after it.  Created once
// per device (default priority, non-blocking); where they cannot be created
// every bin runs on the caller's stream.  The lock keeps one call's fork and
// join events from being re-recorded by another host thread in between.
constexpr int kSide = 3;
struct SideStreams {
    hipStream_t st[kSide];
    hipEvent_t fork, join[kSide];
    bool ok;
};

static std::mutex g_side_mu;

static SideStreams *side_streams()
{
    static SideStreams cache[64];
    static bool tried[64] = {false};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    SideStreams &x = cache[dev];
    if (!tried[dev]) {
        tried[dev] = true;
        x.ok = hipEventCreateWithFlags(&x.fork, hipEventDisableTiming) == hipSuccess;
        for (int i = 0; i < kSide && x.ok; ++i)
            x.ok = hipStreamCreateWithFlags(&x.st[i], hipStreamNonBlocking) == hipSuccess &&
                   hipEventCreateWithFlags(&x.join[i], hipEventDisableTiming) == hipSuccess;
    }
    return x.ok ? &x : nullptr;
}

// Runs launch(b, stream) for every bin b with work[b] > 0: the largest on s
// (first), the others on the side streams.  The side streams are
// joined back into s also when a launch fails; returns the first error.
template <class F>
static int run_bins(hipStream_t s, const std::vector<int64_t> &work, bool one_stream, F launch)
{
    int big = -1, nb = 0;
    for (int b = 0; b < (int)work.size(); ++b) {
        if (work[b] <= 0) continue;
        ++nb;
        if (big < 0 || work[b] > work[big]) big = b;
    }
    std::lock_guard<std::mutex> lk(g_side_mu);
    SideStreams *x = nb > 1 && !one_stream ? side_streams() : nullptr;
    if (x && hipEventRecord(x->fork, s) != hipSuccess) x = nullptr;
    bool used[kSide] = {false, false, false};
    int k = 0, rc = HCSP_OK;
    if (big >= 0) rc = launch(big, s);
    for (int b = 0; b < (int)work.size() && rc == HCSP_OK; ++b) {
        if (work[b] <= 0 || b == big) continue;
        hipStream_t t = s;
        if (x) {
            const int i = k++ % kSide;
            if (!used[i]) {
                if (hipStreamWaitEvent(x->st[i], x->fork, 0) != hipSuccess) {
                    rc = fail(HCSP_E_HIP, "hipStreamWaitEvent failed");
                    break;
                }
                used[i] = true;
            }
            t = x->st[i];
        }
        rc = launch(b, t);
    }
    for (int i = 0; i < kSide; ++i) {
        if (!used[i]) continue;
        if ((hipEventRecord(x->join[i], x->st[i]) != hipSuccess || hipStreamWaitEvent(s, x->join[i], 0) != hipSuccess) &&
            rc == HCSP_OK)
            rc = fail(HCSP_E_HIP, "joining a side stream failed");
    }
    return rc;
}

static int make_tune(const hcsp_opts *o, const hcsp_csr *B, bool need_device, Tune *t)
{
    hcsp_opts z;
    std::memset(&z, 0, sizeof z);
    if (!o) o = &z;
    if (o->lanes != 0 && o->lanes != 64) return fail(HCSP_E_INVALID, "opts.lanes must be 0 or 64");
    t->G = 64;
    t->one_stream = (o->flags & HCSP_F_ONE_STREAM) != 0;
    t->load_pct = o->load_pct ? o->load_pct : 60;
    if (t->load_pct < 10 || t->load_pct > 95) return fail(HCSP_E_INVALID, "opts.load_pct must be in 10..95");
    t->sym_load_pct = o->sym_load_pct ? o->sym_load_pct : 70;
    if (t->sym_load_pct < 10 || t->sym_load_pct > 100) return fail(HCSP_E_INVALID, "opts.sym_load_pct must be in 10..100");
    t->lds_budget = need_device ? lds_limit() : 64 * 1024;
    int sym = kSymLog2Max;
    while (sym > kSymLog2Min && sym_wave_bytes(2, 1 << sym) > t->lds_budget) --sym;
    if (o->sym_tmax_log2) sym = std::max(kSymLog2Min + 1, std::min(sym, (int)o->sym_tmax_log2));
    t->sym_tmax_log2 = sym;
    t->num_tmax = o->num_tmax ? o->num_tmax : (1 << 30);
    // dense accumulators: by default as many as fit in 4 GiB, between 32 and 1024
    const int64_t per_slot = 8 * std::max<int64_t>(B->ncols, 1) + 4 * ((B->ncols + 31) / 32);
    t->dense_slots = o->dense_slots ? o->dense_slots
                                    : (int)std::max<int64_t>(32, std::min<int64_t>(1024, (4ll << 30) / per_slot));
    if (t->dense_slots < 4) t->dense_slots = 4;
    t->dense_slots &= ~3;
    t->win_log2 = o->win_chunk_log2 ? o->win_chunk_log2 : kWinLog2Default;
    if (t->win_log2 < 4 || t->win_log2 > 30) return fail(HCSP_E_INVALID, "opts.win_chunk_log2 must be 0 or in 4..30");
    // and never more than 16 GiB
    while (t->dense_slots > 4 && (int64_t)t->dense_slots * per_slot > (16ll << 30)) t->dense_slots -= 4;
    return HCSP_OK;
}

static void num_tmax_classes(const Tune &tu, bool cl, int out[kSClasses])
{
    for (int sc = 0; sc < kSClasses; ++sc) {
        int best = 0;
        for (int t = 0; t < kNumT; ++t) {
            const int T = num_table(t);
            if (T <= tu.num_tmax && num_wave_bytes(cl, sc, T, tu.load_pct) <= tu.lds_budget) best = T;
        }
        out[sc] = best;
    }
}

static int check_csr_shape(const hcsp_csr *M, const char *name, bool need_val)
{
    if (!M) return fail(HCSP_E_INVALID, std::string(name) + " is null");
    if (M->nrows < 0 || M->ncols < 0 || M->nnz < 0)
        return fail(HCSP_E_INVALID, std::string(name) + ": negative size");
    if (M->nrows >= INT32_MAX || M->ncols >= INT32_MAX)
        return fail(HCSP_E_OVERFLOW, std::string(name) + ": row/column ids must fit int32");
    if (!M->row_ptr || (M->nnz > 0 && (!M->col || (need_val && !M->val))))
        return fail(HCSP_E_INVALID, std::string(name) + ": null array");
    return HCSP_OK;
}

struct OpView {
    bool cluster;
    int64_t nrows, ncols, nunits;
};

static int check_operands(const hcsp_operand *A, const hcsp_csr *B, OpView *v)
{
    if (!A || !B) return fail(HCSP_E_INVALID, "null operand");
    int rc = check_csr_shape(B, "B", true);
    if (rc) return rc;
    if (A->kind == HCSP_OP_CSR) {
        rc = check_csr_shape(&A->csr, "A", true);
        if (rc) return rc;
        v->cluster = false;
        v->nrows = A->csr.nrows;
        v->ncols = A->csr.ncols;
        v->nunits = A->csr.nrows;
    } else if (A->kind == HCSP_OP_CLUSTER) {
        const hcsp_csr_cluster &c = A->cl;
        if (c.nrows < 0 || c.nclusters < 0 || c.ncc < 0 || c.nslots < 0)
            return fail(HCSP_E_INVALID, "A (cluster): negative size");
        if (c.nrows >= INT32_MAX || c.ncols >= INT32_MAX || c.nclusters >= INT32_MAX)
            return fail(HCSP_E_OVERFLOW, "A (cluster): ids must fit int32");
        if (c.max_cluster < 0 || c.max_cluster > 16) return fail(HCSP_E_UNSUPPORTED, "clusters hold at most 16 rows");
        if (!c.cl_row_ptr || !c.perm && c.nrows > 0 || !c.cl_col_ptr || !c.cl_val_ptr ||
            (c.ncc > 0 && (!c.cl_col || !c.cl_mask)) || (c.nslots > 0 && !c.cl_val))
            return fail(HCSP_E_INVALID, "A (cluster): null array");
        v->cluster = true;
        v->nrows = c.nrows;
        v->ncols = c.ncols;
        v->nunits = c.nclusters;
    } else {
        return fail(HCSP_E_INVALID, "unknown operand kind");
    }
    if (v->ncols != B->nrows) return fail(HCSP_E_INVALID, "A.ncols != B.nrows");
    if (B->nnz >= (1ll << 29))
        return fail(HCSP_E_UNSUPPORTED, "B must have fewer than 2^29 entries (32-bit byte offsets)");
    return HCSP_OK;
}

static SpArgs base_args(const hcsp_operand *A, const hcsp_csr *B, const Workspace &ws, const Tune &tu)
{
    SpArgs a;
    std::memset(&a, 0, sizeof a);
    if (A->kind == HCSP_OP_CSR) {
        a.a_rp = A->csr.row_ptr;
        a.a_col = A->csr.col;
        a.a_val = A->csr.val;
    } else {
        a.cl_row_ptr = A->cl.cl_row_ptr;
        a.perm = A->cl.perm;
        a.cl_col_ptr = A->cl.cl_col_ptr;
        a.cl_col = A->cl.cl_col;
        a.cl_mask = A->cl.cl_mask;
        a.cl_val_ptr = A->cl.cl_val_ptr;
        a.cl_val = A->cl.cl_val;
    }
    a.b_rp = B->row_ptr;
    a.b_col = B->col;
    a.b_val = B->val;
    a.keylo = ws.keylo;
    a.keyhi = ws.keyhi;
    a.ucount = ws.ucount;
    a.err = ws.err;
    a.G = tu.G;
    a.dense_bits = ws.dense_bits;
    a.dense_vals = ws.dense_vals;
    a.dense_words = ws.dense_words;
    a.probes = ws.probes;
    a.chunk_cnt = ws.chunk_cnt;
    a.sym_base = ws.sym_base;
    a.win_base = ws.win_base;
    a.win_cap = ws.win_cap;
    a.win_cur = ws.win_cur;
    a.win_log2 = tu.win_log2;
    a.ncols = B->ncols;
    a.unit_lo = 0;
    a.unit_hi = INT64_MAX;
    return a;
}

static BinArgs bin_args(const hcsp_operand *A, const hcsp_csr *B, const Workspace &ws, const Tune &tu,
                        int64_t nunits, int64_t *c_rp)
{
    BinArgs b;
    std::memset(&b, 0, sizeof b);
    if (A->kind == HCSP_OP_CSR) {
        b.a_rp = A->csr.row_ptr;
        b.a_col = A->csr.col;
    } else {
        b.cl_row_ptr = A->cl.cl_row_ptr;
        b.perm = A->cl.perm;
        b.cl_col_ptr = A->cl.cl_col_ptr;
        b.cl_col = A->cl.cl_col;
    }
    b.b_rp = B->row_ptr;
    b.b_col = B->col;
    b.nunits = nunits;
    b.ws = ws;
    b.c_rp = c_rp;
    b.sym_tmax_log2 = tu.sym_tmax_log2;
    num_tmax_classes(tu, A->kind == HCSP_OP_CLUSTER, b.num_tmax_by_class);
    b.load_pct = tu.load_pct;
    b.sym_load_pct = tu.sym_load_pct;
    return b;
}

// Launch geometry for one bin: one wavefront per unit, one to four per block,
// whichever lets the most wavefronts share a compute unit's 160 KiB of LDS
// (ties go to the larger block).
// Wavefronts per block: the most resident wavefronts per compute unit, ties
// to the larger block; one wavefront per block (single) when units take
// uneven time, so that a finished wavefront frees its shared memory at once
// instead of when the slowest of its block ends.
static void geometry(int64_t wave_bytes, int64_t count, int *blocks, int *threads, size_t *lds,
                     bool single = false)
{
    const int64_t cu_lds = 160 * 1024, wb = std::max<int64_t>(wave_bytes, 1);
    int64_t wpb = 1, best = -1;
    for (int64_t w = single ? 1 : 4; w >= 1; w >>= 1) {
        const int64_t resident = std::min<int64_t>(32, cu_lds / (w * wb) * w);
        if (w * wb <= cu_lds && resident > best) {
            best = resident;
            wpb = w;
        }
    }
    *threads = (int)(wpb * 64);
    *lds = (size_t)(wpb * wave_bytes);
    *blocks = (int)((count + wpb - 1) / wpb);
}

// Workgroups of a numeric launch over rows too long for shared memory (as
// many as fit on the device).
static int64_t num_bm_blocks()
{
    return std::max<int64_t>(1, (160 * 1024) / num_bm_bytes()) * cu_count();
}

static int ensure_lds(size_t lds, int64_t budget)
{
    if ((int64_t)lds > budget) return fail(HCSP_E_UNSUPPORTED, "shared-memory table larger than the device allows");
    return HCSP_OK;
}

// Batch workspace: descriptors and per-product data, then the same per-unit
// arrays and counters as a single product (over the batch's units).
struct BatchWs {
    BatchProb *probs;
    int64_t *units, *segs;     // [count+1] unit and row-offset segment bases
    int64_t *ub, *nnz, *seg_base, *maxp;
    uint32_t *errs;
    int64_t *sym_begin, *num_begin;
    Workspace w;
};

static size_t layout_batch(int32_t count, int64_t units, int64_t row_ptr_len, int64_t max_ncols, int dense_slots,
                           char *base, BatchWs *b)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        off = align_up(off, 256);
        void *p = base ? (void *)(base + off) : nullptr;
        off += bytes;
        return p;
    };
    const size_t n = (size_t)std::max(count, 1);
    b->probs = (BatchProb *)take(sizeof(BatchProb) * n);
    b->units = (int64_t *)take(8 * (n + 1));
    b->segs = (int64_t *)take(8 * (n + 1));
    b->ub = (int64_t *)take(8 * n);
    b->nnz = (int64_t *)take(8 * n);
    b->seg_base = (int64_t *)take(8 * n);
    b->maxp = (int64_t *)take(8);
    b->errs = (uint32_t *)take(4 * n);
    b->sym_begin = (int64_t *)take(8 * HCSP_MAX_BINS);
    b->num_begin = (int64_t *)take(8 * HCSP_MAX_BINS);
    off = align_up(off, 256);
    const size_t rest = layout_workspace(units, row_ptr_len, max_ncols, 0, dense_slots, false, base ? base + off : nullptr, &b->w);
    return off + rest;
}

static BinArgs batch_bin_args(const hcsp_batch_plan &plan, const BatchWs &ws, const Tune &tu, int64_t *c_rp)
{
    BinArgs b;
    std::memset(&b, 0, sizeof b);
    b.nunits = plan.units;
    b.ws = ws.w;
    b.c_rp = c_rp;
    b.sym_tmax_log2 = tu.sym_tmax_log2;
    num_tmax_classes(tu, plan.kind == HCSP_OP_CLUSTER, b.num_tmax_by_class);
    b.load_pct = tu.load_pct;
    b.sym_load_pct = tu.sym_load_pct;
    b.batch = ws.probs;
    b.batch_units = ws.units;
    b.nprob = plan.count;
    return b;
}

}  // namespace hcsp

using namespace hcsp;

static int numeric_bins(SpArgs &a, const hcsp_sym_info *info, bool cluster, const Tune &tu, const Workspace &ws,
                        hipStream_t s);

extern "C" {

const char *hcsp_version(void) { return "hcsp 0.1 (gfx950)"; }

const char *hcsp_strerror(int status)
{
    switch (status) {
    case HCSP_OK: return "ok";
    case HCSP_E_INVALID: return "invalid argument";
    case HCSP_E_PTR: return "malformed row offsets";
    case HCSP_E_RANGE: return "column index out of range";
    case HCSP_E_UNSORTED: return "columns not strictly increasing within a row";
    case HCSP_E_CAPACITY: return "buffer too small";
    case HCSP_E_HIP: return "HIP runtime error";
    case HCSP_E_NOMEM: return "host out of memory";
    case HCSP_E_UNSUPPORTED: return "unsupported";
    case HCSP_E_OVERFLOW: return "index overflow";
    default: return "unknown status";
    }
}

const char *hcsp_last_error(void) { return g_err.c_str(); }

int hcsp_csr_check(const hcsp_csr *A, void *ws_d, size_t ws_bytes, void *stream)
{
    clear_error();
    if (!A || !A->row_ptr) return fail(HCSP_E_INVALID, "null matrix");
    if (A->nrows < 0 || A->ncols < 0 || A->nnz < 0) return fail(HCSP_E_INVALID, "negative size");
    if (A->nnz > 0 && !A->col) return fail(HCSP_E_INVALID, "null column array");
    if (!ws_d || ws_bytes < 64) return fail(HCSP_E_CAPACITY, "csr_check needs 64 bytes of workspace");
    hipStream_t s = (hipStream_t)stream;
    uint32_t *flags = (uint32_t *)ws_d;
    HCSP_HIP(launch_fill_u32(flags, 1, 0u, s));
    HCSP_HIP(launch_csr_check(*A, flags, s));
    uint32_t h = 0;
    HCSP_HIP(hipMemcpyAsync(&h, flags, 4, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));
    if (h & kErrPtr) return fail(HCSP_E_PTR, "row offsets are not a valid CSR offset array");
    if (h & kErrRange) return fail(HCSP_E_RANGE, "a column index is outside [0, ncols)");
    if (h & kErrUnsorted) return fail(HCSP_E_UNSORTED, "columns are not strictly increasing within a row");
    return HCSP_OK;
}

int hcsp_cluster_workspace(int64_t nrows, int64_t ncl, size_t *bytes)
{
    clear_error();
    if (!bytes || nrows < 0 || ncl < 0) return fail(HCSP_E_INVALID, "bad arguments");
    *bytes = align_up(8 * scan_tmp_elems(ncl + 1), 256) + 256;
    return HCSP_OK;
}

int hcsp_cluster_count(const hcsp_csr *A, const int32_t *perm_d, const int64_t *cl_row_ptr_d, int64_t ncl,
                       int64_t *cl_col_ptr_d, int64_t *cl_val_ptr_d, int64_t *ncc_h, int64_t *nslots_h,
                       int32_t *max_cluster_h, void *ws_d, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc = check_csr_shape(A, "A", true);
    if (rc) return rc;
    if (ncl < 0 || (ncl > 0 && (!perm_d || !cl_row_ptr_d)) || !cl_col_ptr_d || !cl_val_ptr_d || !ncc_h ||
        !nslots_h)
        return fail(HCSP_E_INVALID, "bad arguments");
    size_t need = 0;
    hcsp_cluster_workspace(A->nrows, ncl, &need);
    if (!ws_d || ws_bytes < need) return fail(HCSP_E_CAPACITY, "cluster workspace too small");
    hipStream_t s = (hipStream_t)stream;
    int32_t *maxs = (int32_t *)ws_d;
    int64_t *tmp = (int64_t *)((char *)ws_d + 256);
    HCSP_HIP(launch_fill_u32((uint32_t *)maxs, 1, 0u, s));
    HCSP_HIP(launch_fill_i64(cl_col_ptr_d + ncl, 1, 0, s));
    HCSP_HIP(launch_fill_i64(cl_val_ptr_d + ncl, 1, 0, s));
    HCSP_HIP(launch_cluster_count(*A, perm_d, cl_row_ptr_d, ncl, cl_col_ptr_d, cl_val_ptr_d, maxs, s));
    HCSP_HIP(launch_scan_exclusive(cl_col_ptr_d, ncl + 1, tmp, s));
    HCSP_HIP(launch_scan_exclusive(cl_val_ptr_d, ncl + 1, tmp, s));
    int32_t mx = 0;
    HCSP_HIP(hipMemcpyAsync(ncc_h, cl_col_ptr_d + ncl, 8, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipMemcpyAsync(nslots_h, cl_val_ptr_d + ncl, 8, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipMemcpyAsync(&mx, maxs, 4, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));
    if (mx > 16) return fail(HCSP_E_INVALID, "a cluster of the plan has 0 or more than 16 rows");
    if (max_cluster_h) *max_cluster_h = mx;
    return HCSP_OK;
}

int hcsp_cluster_fill(const hcsp_csr *A, const hcsp_csr_cluster *out, void *stream)
{
    clear_error();
    int rc = check_csr_shape(A, "A", true);
    if (rc) return rc;
    if (!out || out->nclusters < 0 || (out->nclusters > 0 && (!out->perm || !out->cl_row_ptr)) ||
        !out->cl_col_ptr || !out->cl_val_ptr || (out->ncc > 0 && (!out->cl_col || !out->cl_mask)) ||
        (out->nslots > 0 && !out->cl_val))
        return fail(HCSP_E_INVALID, "bad CSR_Cluster output");
    HCSP_HIP(launch_cluster_fill(*A, *out, (hipStream_t)stream));
    return HCSP_OK;
}

int hcsp_spgemm_workspace(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts, size_t *bytes)
{
    clear_error();
    OpView v;
    int rc = check_operands(A, B, &v);
    if (rc) return rc;
    if (!bytes) return fail(HCSP_E_INVALID, "null bytes");
    Tune tu;
    rc = make_tune(opts, B, false, &tu);
    if (rc) return rc;
    Workspace ws;
    *bytes = layout_workspace(v.nunits, v.nrows, B->ncols, B->nrows, tu.dense_slots, true, nullptr, &ws);
    return HCSP_OK;
}

}  // extern "C"

// Symbolic phase over the units with active[u] != 0 (all when null); the
// counts of the other rows must already be in C_row_ptr_d, since the final
// scan covers every row.
static int symbolic_impl(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts, int64_t *C_row_ptr_d,
                         hcsp_sym_info *info, void *ws_d, size_t ws_bytes, void *stream, const uint8_t *active)
{
    OpView v;
    int rc = check_operands(A, B, &v);
    if (rc) return rc;
    if (!C_row_ptr_d || !info) return fail(HCSP_E_INVALID, "null output");
    Tune tu;
    rc = make_tune(opts, B, true, &tu);
    if (rc) return rc;
    Workspace ws;
    const size_t need = layout_workspace(v.nunits, v.nrows, B->ncols, B->nrows, tu.dense_slots, true, (char *)ws_d, &ws);
    if (!ws_d || ws_bytes < need) return fail(HCSP_E_CAPACITY, "SpGEMM workspace too small");
    hipStream_t s = (hipStream_t)stream;
    std::memset(info, 0, sizeof *info);

    // one launch: the bin counters, the error word and C's last row offset
    // cleared, and B's 2-byte row lengths for the work estimate
    HCSP_HIP(launch_sym_start(B->row_ptr, B->nrows, ws.b_len, ws.sym_count, ws.num_count, HCSP_MAX_BINS, ws.err,
                              C_row_ptr_d + v.nrows, s));

    BinArgs ba = bin_args(A, B, ws, tu, v.nunits, C_row_ptr_d);
    ba.active = active;
    ba.b_len = ws.b_len;
    HCSP_HIP(launch_work(v.cluster, ba, s));
    HCSP_HIP(launch_scatter(ws.bin, v.nunits, ws.bin_hist, kSymBins, ws.sym_count, ws.order_sym, s));
    int64_t cnt[HCSP_MAX_BINS];
    HCSP_HIP(hipMemcpyAsync(cnt, ws.sym_count, 8 * kSymBins, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));

    SpArgs a = base_args(A, B, ws, tu);
    a.order = ws.order_sym;
    a.c_rp = C_row_ptr_d;
    std::vector<int64_t> begin(kSymBins), work(kSymBins, 0);
    int64_t start = 0;
    for (int b = 0; b < kSymBins; ++b) {
        info->sym_bin_count[b] = cnt[b];
        begin[b] = start;
        start += cnt[b];
        if (cnt[b] > 0 && b != kBinEmpty)
            work[b] = b == kSymGlobal ? INT64_MAX / 2 : cnt[b] << ((b - 1) % kSymT + kSymLog2Min);
    }
    rc = run_bins(s, work, tu.one_stream, [&](int b, hipStream_t t) -> int {
        const int64_t c = cnt[b];
        a.bin_begin = begin[b];
        a.count = c;
        if (b == kSymGlobal) {
            HCSP_HIP(launch_win_prep(true, v.cluster, a, t));
            HCSP_HIP(launch_scan_exclusive(ws.win_base, c + 1, ws.scan_tmp, t));
            const int e = ensure_lds((size_t)sym_bm_bytes(), tu.lds_budget);
            if (e) return e;
            const int64_t per_cu = std::max<int64_t>(1, (160 * 1024) / sym_bm_bytes());
            HCSP_HIP(launch_sym_bm(v.cluster, a, (int)(per_cu * cu_count()), t));
            return HCSP_OK;
        }
        const int sc = (b - 1) / kSymT;
        const int l2 = (b - 1) % kSymT + kSymLog2Min;
        a.T = 1 << l2;
        a.log2T = l2;
        const int64_t gb = sym_wave_bytes(v.cluster ? mask_bytes_of_class(sc) : 0, a.T);
        a.group_bytes = (int)gb;
        int blocks, threads;
        size_t lds;
        geometry(gb, c, &blocks, &threads, &lds);
        const int e = ensure_lds(lds, tu.lds_budget);
        if (e) return e;
        HCSP_HIP(launch_sym(sc, v.cluster, false, a, blocks, threads, lds, t));
        return HCSP_OK;
    });
    if (rc) return rc;
    HCSP_HIP(launch_scan_exclusive(C_row_ptr_d, v.nrows + 1, ws.scan_tmp, s));
    HCSP_HIP(launch_numbin(v.cluster, ba, s));
    HCSP_HIP(launch_scatter(ws.bin, v.nunits, ws.bin_hist, kNumBins, ws.num_count, ws.order_num, s));
    // the numeric bin counts, nnz(C) and the error word in one read-back
    static_assert(kNumBins + 2 <= HCSP_MAX_BINS, "room for nnz and the error word after the bin counts");
    int64_t ncnt[HCSP_MAX_BINS];
    HCSP_HIP(launch_gather_words(ws.num_count + kNumBins, GatherWords{{C_row_ptr_d + v.nrows, ws.err}, {8, 4}, 2}, s));
    HCSP_HIP(hipMemcpyAsync(ncnt, ws.num_count, 8 * (kNumBins + 2), hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));
    const int64_t nnz = ncnt[kNumBins];
    const uint32_t e = (uint32_t)ncnt[kNumBins + 1];
    if (e & kErrWindows)
        return fail(HCSP_E_CAPACITY, "more (row, chunk) pairs of long rows than the workspace holds (raise "
                                     "opts.win_chunk_log2 for fewer chunks)");
    info->nnz = nnz;
    info->units = v.nunits;
    for (int b = 0; b < kNumBins; ++b) info->num_bin_count[b] = ncnt[b];
    info->lanes = tu.G;
    info->load_pct = tu.load_pct;
    info->win_chunk_log2 = tu.win_log2;
    info->valid = 1;
    return HCSP_OK;
}

extern "C" {

int hcsp_spgemm_symbolic(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts, int64_t *C_row_ptr_d,
                         hcsp_sym_info *info, void *ws_d, size_t ws_bytes, void *stream)
{
    clear_error();
    return symbolic_impl(A, B, opts, C_row_ptr_d, info, ws_d, ws_bytes, stream, nullptr);
}

int hcsp_spgemm_numeric(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts, const hcsp_sym_info *info,
                        const int64_t *C_row_ptr_d, int32_t *C_col_d, double *C_val_d, int64_t capacity, void *ws_d,
                        size_t ws_bytes, void *stream)
{
    clear_error();
    OpView v;
    int rc = check_operands(A, B, &v);
    if (rc) return rc;
    if (!info || !info->valid || info->units != v.nunits) return fail(HCSP_E_INVALID, "info is not from a matching symbolic call");
    if (!C_row_ptr_d || capacity < 0 || (capacity > 0 && (!C_col_d || !C_val_d)))
        return fail(HCSP_E_INVALID, "bad output arrays");
    Tune tu;
    rc = make_tune(opts, B, true, &tu);
    if (rc) return rc;
    if (tu.G != info->lanes || tu.load_pct != info->load_pct || tu.win_log2 != info->win_chunk_log2)
        return fail(HCSP_E_INVALID, "opts differ from the symbolic call");
    Workspace ws;
    const size_t need = layout_workspace(v.nunits, v.nrows, B->ncols, B->nrows, tu.dense_slots, true, (char *)ws_d, &ws);
    if (!ws_d || ws_bytes < need) return fail(HCSP_E_CAPACITY, "SpGEMM workspace too small");
    hipStream_t s = (hipStream_t)stream;
    hcsp_opts z;
    std::memset(&z, 0, sizeof z);
    const hcsp_opts *o = opts ? opts : &z;

    HCSP_HIP(launch_fill_u32(ws.err, 1, 0u, s));
    SpArgs a = base_args(A, B, ws, tu);
    a.order = ws.order_num;
    a.c_rp = const_cast<int64_t *>(C_row_ptr_d);
    a.c_col = C_col_d;
    a.c_val = C_val_d;
    a.cap = capacity;
    a.out_base = o->out_base;
    a.unit_lo = o->unit_lo;
    a.unit_hi = o->unit_hi > 0 ? o->unit_hi : INT64_MAX;
    rc = numeric_bins(a, info, v.cluster, tu, ws, s);
    if (rc) return rc;
    if (o->flags & HCSP_F_SYNC_CHECK) {
        uint32_t e = 0;
        HCSP_HIP(hipMemcpyAsync(&e, ws.err, 4, hipMemcpyDeviceToHost, s));
        HCSP_HIP(hipStreamSynchronize(s));
        if (e & kErrCapacity) return fail(HCSP_E_CAPACITY, "output capacity too small for the requested units");
        if (e & kErrCount) return fail(HCSP_E_INVALID, "row counts differ from the symbolic phase (inputs changed?)");
        if (e & kErrWindows) return fail(HCSP_E_INVALID, "chunk counts of long rows missing (no matching symbolic call)");
    }
    return HCSP_OK;
}

}  // extern "C"

// The numeric launches of every bin the symbolic phase filled (a: the
// product's arguments and outputs).
static int numeric_bins(SpArgs &a, const hcsp_sym_info *info, bool cluster, const Tune &tu, const Workspace &ws,
                        hipStream_t s)
{
    std::vector<int64_t> begin(kNumBins), work(kNumBins, 0);
    int64_t start = 0;
    for (int b = 0; b < kNumBins; ++b) {
        const int64_t c = info->num_bin_count[b];
        begin[b] = start;
        start += c;
        if (c > 0 && b != kBinEmpty) work[b] = b == kNumGlobal ? INT64_MAX / 2 : c * num_table((b - 1) % kNumT);
    }
    return run_bins(s, work, tu.one_stream, [&](int b, hipStream_t st) -> int {
        const int64_t c = info->num_bin_count[b];
        a.bin_begin = begin[b];
        a.count = c;
        if (b == kNumGlobal) {
            HCSP_HIP(launch_win_prep(false, cluster, a, st));
            HCSP_HIP(launch_scan_exclusive(ws.win_base, c + 1, ws.scan_tmp, st));
            const int e = ensure_lds((size_t)num_bm_bytes(), tu.lds_budget);
            if (e) return e;
            // workgroups: as many as fit on the device, each wavefront with a
            // slot of carried positions in the workspace
            const int64_t blocks = std::min<int64_t>(num_bm_blocks(), ws.win_cur_slots / kNumBmWaves);
            if (blocks < 1) return fail(HCSP_E_CAPACITY, "workspace has no room for the long rows' positions");
            HCSP_HIP(launch_num_bm(cluster, a, (int)blocks, st));
            return HCSP_OK;
        }
        const int sc = (b - 1) / kNumT;
        const int t = (b - 1) % kNumT;
        a.T = num_table(t);
        a.vcap = num_vcap(a.T, tu.load_pct);
        const int64_t gb = num_wave_bytes(cluster, sc, a.T, tu.load_pct);
        a.group_bytes = (int)gb;
        int blocks, threads;
        size_t lds;
        geometry(gb, c, &blocks, &threads, &lds, true);
        const int e = ensure_lds(lds, tu.lds_budget);
        if (e) return e;
        HCSP_HIP(launch_num(sc, cluster, false, a, blocks, threads, lds, st));
        return HCSP_OK;
    });
}

// Checks shared by the numeric entry points: operands, info, options and
// workspace; fills v, tu and ws.
static int numeric_setup(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts, const hcsp_sym_info *info,
                         void *ws_d, size_t ws_bytes, OpView *v, Tune *tu, Workspace *ws)
{
    int rc = check_operands(A, B, v);
    if (rc) return rc;
    if (!info || !info->valid || info->units != v->nunits)
        return fail(HCSP_E_INVALID, "info is not from a matching symbolic call");
    rc = make_tune(opts, B, true, tu);
    if (rc) return rc;
    if (tu->G != info->lanes || tu->load_pct != info->load_pct || tu->win_log2 != info->win_chunk_log2)
        return fail(HCSP_E_INVALID, "opts differ from the symbolic call");
    const size_t need = layout_workspace(v->nunits, v->nrows, B->ncols, B->nrows, tu->dense_slots, true, (char *)ws_d, ws);
    if (!ws_d || ws_bytes < need) return fail(HCSP_E_CAPACITY, "SpGEMM workspace too small");
    return HCSP_OK;
}

extern "C" {

int hcsp_topk_candidates(const hcsp_csr *O, const int64_t *a_rp_d, const int32_t *pos_d, hcsp_ratio jacc_th,
                         int32_t topk, int32_t *cnt_d, int32_t *nbr_d, int64_t *ov_d, void *stream)
{
    clear_error();
    if (!O || O->nrows < 0 || O->nrows != O->ncols || (O->nrows > 0 && !O->row_ptr) ||
        (O->nnz > 0 && (!O->col || !O->val)))
        return fail(HCSP_E_INVALID, "topk: bad overlap matrix");
    if (jacc_th.den <= 0 || jacc_th.num < 0 || topk < 1 || topk > 15)
        return fail(HCSP_E_INVALID, "topk: bad threshold or topk (1..15)");
    if (O->nrows > 0 && (!a_rp_d || !cnt_d || !nbr_d || !ov_d)) return fail(HCSP_E_INVALID, "topk: null array");
    HCSP_HIP(launch_topk(O->row_ptr, O->col, O->val, a_rp_d, pos_d, O->nrows, jacc_th.num, jacc_th.den, topk, cnt_d,
                         nbr_d, ov_d, (hipStream_t)stream));
    return HCSP_OK;
}

int hcsp_spgemm_status(const void *ws_d, size_t ws_bytes, void *stream)
{
    clear_error();
    if (!ws_d || ws_bytes < 256) return fail(HCSP_E_INVALID, "status: not a SpGEMM workspace");
    hipStream_t s = (hipStream_t)stream;
    uint32_t e = 0;
    HCSP_HIP(hipMemcpyAsync(&e, ws_d, 4, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));
    if (e & kErrCapacity) return fail(HCSP_E_CAPACITY, "output capacity too small for the requested units");
    if (e & kErrCount) return fail(HCSP_E_INVALID, "row counts differ from the symbolic phase (inputs changed?)");
    if (e & kErrWindows) return fail(HCSP_E_INVALID, "chunk counts of long rows missing (no matching symbolic call)");
    return HCSP_OK;
}

int hcsp_csr_transpose_workspace(int64_t nrows, int64_t ncols, size_t *bytes)
{
    clear_error();
    if (!bytes || nrows < 0 || ncols < 0) return fail(HCSP_E_INVALID, "transpose: bad arguments");
    TrWs w;
    *bytes = layout_transpose(nrows, ncols, nullptr, &w);
    return HCSP_OK;
}

int hcsp_csr_transpose(const hcsp_csr *A, hcsp_csr *At, void *ws_d, size_t ws_bytes, void *stream)
{
    clear_error();
    const bool vals = At && At->val;
    int rc = check_csr_shape(A, "A", vals);
    if (rc) return rc;
    if (!At || At->nrows != A->ncols || At->ncols != A->nrows || At->nnz != A->nnz || !At->row_ptr ||
        (A->nnz > 0 && !At->col))
        return fail(HCSP_E_INVALID, "transpose: At must be ncols x nrows with nnz entries and its arrays set");
    TrWs w;
    const size_t need = layout_transpose(A->nrows, A->ncols, (char *)ws_d, &w);
    if (!ws_d || ws_bytes < need) return fail(HCSP_E_CAPACITY, "transpose workspace too small");
    HCSP_HIP(launch_transpose(*A, *At, w, (hipStream_t)stream));
    return HCSP_OK;
}

int hcsp_cluster_output_layout(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts,
                               const hcsp_sym_info *info, int64_t *cl_col_ptr_d, int64_t *cl_val_ptr_d,
                               int64_t *ncc_h, int64_t *nslots_h, void *ws_d, size_t ws_bytes, void *stream)
{
    clear_error();
    if (!A || A->kind != HCSP_OP_CLUSTER) return fail(HCSP_E_INVALID, "CSR_Cluster output needs a CSR_Cluster A");
    if (!cl_col_ptr_d || !cl_val_ptr_d || !ncc_h || !nslots_h) return fail(HCSP_E_INVALID, "null output");
    OpView v;
    Tune tu;
    Workspace ws;
    int rc = numeric_setup(A, B, opts, info, ws_d, ws_bytes, &v, &tu, &ws);
    if (rc) return rc;
    if (info->num_bin_count[kNumGlobal] > 0)
        return fail(HCSP_E_UNSUPPORTED, "clusters too large for shared-memory tables cannot be written as CSR_Cluster");
    hipStream_t s = (hipStream_t)stream;
    HCSP_HIP(launch_fill_u32(ws.err, 1, 0u, s));
    HCSP_HIP(launch_cl_out_counts(ws.ucount, A->cl.cl_row_ptr, v.nunits, cl_col_ptr_d, cl_val_ptr_d, ws.err, s));
    HCSP_HIP(launch_scan_exclusive(cl_col_ptr_d, v.nunits + 1, ws.scan_tmp, s));
    HCSP_HIP(launch_scan_exclusive(cl_val_ptr_d, v.nunits + 1, ws.scan_tmp, s));
    // both totals and the error word in one read-back, through spare bin-count slots
    static_assert(kNumBins + 3 <= HCSP_MAX_BINS, "room for three words after the bin counts");
    int64_t w[3];
    HCSP_HIP(launch_gather_words(ws.num_count + kNumBins,
                                 GatherWords{{cl_col_ptr_d + v.nunits, cl_val_ptr_d + v.nunits, ws.err}, {8, 8, 4}, 3}, s));
    HCSP_HIP(hipMemcpyAsync(w, ws.num_count + kNumBins, sizeof w, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));
    *ncc_h = w[0];
    *nslots_h = w[1];
    if ((uint32_t)w[2]) return fail(HCSP_E_UNSUPPORTED, "a cluster's union exceeds shared memory (no CSR_Cluster output)");
    return HCSP_OK;
}

int hcsp_spgemm_numeric_cluster(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts,
                                const hcsp_sym_info *info, const hcsp_csr_cluster *C, void *ws_d, size_t ws_bytes,
                                void *stream)
{
    clear_error();
    if (!A || A->kind != HCSP_OP_CLUSTER) return fail(HCSP_E_INVALID, "CSR_Cluster output needs a CSR_Cluster A");
    OpView v;
    Tune tu;
    Workspace ws;
    int rc = numeric_setup(A, B, opts, info, ws_d, ws_bytes, &v, &tu, &ws);
    if (rc) return rc;
    if (!C || C->nclusters != A->cl.nclusters || C->nrows != A->cl.nrows || C->ncols != B->ncols || C->ncc < 0 ||
        C->nslots < 0 || !C->cl_col_ptr || !C->cl_val_ptr || (C->ncc > 0 && (!C->cl_col || !C->cl_mask)) ||
        (C->nslots > 0 && !C->cl_val))
        return fail(HCSP_E_INVALID, "bad CSR_Cluster output");
    if (info->num_bin_count[kNumGlobal] > 0)
        return fail(HCSP_E_UNSUPPORTED, "clusters too large for shared-memory tables cannot be written as CSR_Cluster");
    hipStream_t s = (hipStream_t)stream;
    HCSP_HIP(launch_fill_u32(ws.err, 1, 0u, s));
    SpArgs a = base_args(A, B, ws, tu);
    a.order = ws.order_num;
    a.oc_col_ptr = C->cl_col_ptr;
    a.oc_val_ptr = C->cl_val_ptr;
    a.oc_col = C->cl_col;
    a.oc_mask = C->cl_mask;
    a.oc_val = C->cl_val;
    a.oc_ncc = C->ncc;
    a.oc_nslots = C->nslots;
    rc = numeric_bins(a, info, true, tu, ws, s);
    if (rc) return rc;
    uint32_t e = 0;
    HCSP_HIP(hipMemcpyAsync(&e, ws.err, 4, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));
    if (e & kErrCapacity) return fail(HCSP_E_CAPACITY, "CSR_Cluster output arrays too small");
    if (e & kErrCount) return fail(HCSP_E_INVALID, "cluster counts differ from the symbolic phase (inputs changed?)");
    return HCSP_OK;
}

// ================================================================ predicted sizes

int hcsp_spgemm_products(const hcsp_csr *A, const hcsp_csr *B, int64_t *products_h, void *ws_d, size_t ws_bytes,
                         void *stream)
{
    clear_error();
    hcsp_operand op;
    std::memset(&op, 0, sizeof op);
    if (A) op.csr = *A;
    OpView v;
    int rc = check_operands(A ? &op : nullptr, B, &v);
    if (rc) return rc;
    if (!products_h || !ws_d || ws_bytes < 8) return fail(HCSP_E_INVALID, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    int64_t *acc = (int64_t *)ws_d;
    HCSP_HIP(launch_fill_i64(acc, 1, 0, s));
    HCSP_HIP(launch_products(*A, *B, acc, s));
    HCSP_HIP(hipMemcpyAsync(products_h, acc, 8, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));
    return HCSP_OK;
}

// padded scratch entries for a predicted product
static int64_t pred_entries(float ratio, int64_t products, int64_t nrows)
{
    const double e = std::ceil((double)ratio * (double)products) + (double)nrows;
    return std::max<int64_t>(1, std::min<int64_t>(products, (int64_t)e));
}

struct PredWs {
    int64_t *pad_off, *novf;
    int2 *span;  // first and last column of each row of B
    uint8_t *active;
    int32_t *scol;
    double *sval;
    int64_t entries;
};

static size_t layout_pred(size_t base_bytes, int64_t nrows, int64_t brows, int64_t entries, char *base, PredWs *p)
{
    size_t off = base_bytes;
    auto take = [&](size_t bytes) -> void * {
        off = align_up(off, 256);
        void *q = base ? (void *)(base + off) : nullptr;
        off += bytes;
        return q;
    };
    p->pad_off = (int64_t *)take(8 * ((size_t)nrows + 1));
    p->novf = (int64_t *)take(8);
    p->span = (int2 *)take(8 * (size_t)std::max<int64_t>(brows, 1));
    p->active = (uint8_t *)take((size_t)std::max<int64_t>(nrows, 1));
    p->scol = (int32_t *)take(4 * (size_t)entries);
    p->sval = (double *)take(8 * (size_t)entries);
    p->entries = entries;
    return align_up(off, 256);
}

// workspace bytes of a predicted product whose padded scratch holds `entries`
static int pred_workspace(const hcsp_csr *A, const hcsp_csr *B, const hcsp_opts *opts, int64_t entries,
                          size_t *bytes)
{
    hcsp_operand op;
    std::memset(&op, 0, sizeof op);
    if (A) op.csr = *A;
    OpView v;
    int rc = check_operands(A ? &op : nullptr, B, &v);
    if (rc) return rc;
    Tune tu;
    rc = make_tune(opts, B, false, &tu);
    if (rc) return rc;
    Workspace ws;
    const size_t base = layout_workspace(v.nunits, v.nrows, B->ncols, B->nrows, tu.dense_slots, true, nullptr, &ws);
    PredWs p;
    *bytes = layout_pred(base, v.nrows, B->nrows, entries, nullptr, &p);
    return HCSP_OK;
}

int hcsp_predicted_workspace(const hcsp_csr *A, const hcsp_csr *B, const hcsp_opts *opts, float ratio,
                             int64_t products, size_t *bytes)
{
    clear_error();
    if (!bytes || !(ratio > 0.0f && ratio <= 1.0f) || products < 0)
        return fail(HCSP_E_INVALID, "bad arguments (ratio must be in (0, 1])");
    return pred_workspace(A, B, opts, pred_entries(ratio, products, A ? A->nrows : 0), bytes);
}

// padded scratch entries for per-row capacities whose positive values sum to cap_sum (rows with a
// capacity below 1 get 1)
static int64_t pred_rows_entries(int64_t cap_sum, int64_t nrows) { return std::max<int64_t>(1, cap_sum + nrows); }

int hcsp_predicted_rows_workspace(const hcsp_csr *A, const hcsp_csr *B, const hcsp_opts *opts, int64_t cap_sum,
                                  size_t *bytes)
{
    clear_error();
    if (!bytes || cap_sum < 0) return fail(HCSP_E_INVALID, "bad arguments");
    return pred_workspace(A, B, opts, pred_rows_entries(cap_sum, A ? A->nrows : 0), bytes);
}

// The predicted-size product with row capacities from one ratio (cap_row_d null) or given per row; the
// padded scratch holds `entries`.
static int predicted_impl(const hcsp_csr *A, const hcsp_csr *B, const hcsp_opts *opts, float ratio,
                          const int32_t *cap_row_d, int64_t entries, int64_t *C_row_ptr_d, int32_t *C_col_d,
                          double *C_val_d, int64_t capacity, int64_t *nnz_h, int64_t *n_overflow_h, void *ws_d,
                          size_t ws_bytes, void *stream)
{
    hcsp_operand op;
    std::memset(&op, 0, sizeof op);
    if (A) op.csr = *A;
    OpView v;
    int rc = check_operands(A ? &op : nullptr, B, &v);
    if (rc) return rc;
    if (!C_row_ptr_d || capacity < 0 || (capacity > 0 && (!C_col_d || !C_val_d)))
        return fail(HCSP_E_INVALID, "bad arguments");
    Tune tu;
    rc = make_tune(opts, B, true, &tu);
    if (rc) return rc;
    Workspace ws;
    const size_t base = layout_workspace(v.nunits, v.nrows, B->ncols, B->nrows, tu.dense_slots, true, (char *)ws_d, &ws);
    PredWs pw;
    const size_t need = layout_pred(base, v.nrows, B->nrows, entries, (char *)ws_d, &pw);
    if (!ws_d || ws_bytes < need) return fail(HCSP_E_CAPACITY, "predicted-size workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = v.nrows;

    HCSP_HIP(launch_fill_i64(ws.num_count, HCSP_MAX_BINS, 0, s));
    HCSP_HIP(launch_fill_u32(ws.err, 1, 0u, s));
    HCSP_HIP(launch_fill_i64(C_row_ptr_d + n, 1, 0, s));
    HCSP_HIP(launch_fill_i64(pw.pad_off + n, 1, 0, s));
    HCSP_HIP(launch_fill_i64(pw.novf, 1, 0, s));
    // 1. capacities and bins from the prediction, padded row starts
    BinArgs ba = bin_args(&op, B, ws, tu, n, C_row_ptr_d);
    ba.ratio = ratio;
    ba.cap_row = cap_row_d;
    ba.pad = pw.pad_off;
    ba.b_span = pw.span;
    HCSP_HIP(launch_row_span(B->row_ptr, B->col, B->nrows, pw.span, s));
    HCSP_HIP(launch_work_pred(ba, s));
    HCSP_HIP(launch_scatter(ws.bin, n, ws.bin_hist, kNumBins, ws.num_count, ws.order_num, s));
    HCSP_HIP(launch_scan_exclusive(pw.pad_off, n + 1, ws.scan_tmp, s));
    // the bin counts and the padded total in one read-back
    int64_t cnt[HCSP_MAX_BINS];
    HCSP_HIP(launch_gather_words(ws.num_count + kNumBins, GatherWords{{pw.pad_off + n}, {8}, 1}, s));
    HCSP_HIP(hipMemcpyAsync(cnt, ws.num_count, 8 * (kNumBins + 1), hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));
    const int64_t padded = cnt[kNumBins];
    if (padded > pw.entries)  // per-row capacities summing past what the caller declared
        return fail(HCSP_E_INVALID, "row capacities need " + std::to_string(padded) + " scratch entries, " +
                                        std::to_string(pw.entries) + " declared");
    // 2. numeric with the predicted tables, into the padded scratch
    SpArgs a = base_args(&op, B, ws, tu);
    a.order = ws.order_num;
    a.c_rp = C_row_ptr_d;
    a.c_col = pw.scol;
    a.c_val = pw.sval;
    a.cap = pw.entries;
    a.pad_off = pw.pad_off;
    // the bins' launches, the largest on s and the others on side streams
    std::vector<int64_t> pbegin(kNumBins), pwork(kNumBins, 0);
    int64_t start = 0;
    for (int b = 0; b < kNumBins; ++b) {
        pbegin[b] = start;
        start += cnt[b];
        if (cnt[b] > 0 && b != kBinEmpty && b != kNumGlobal) pwork[b] = cnt[b] * num_table((b - 1) % kNumT);
    }
    rc = run_bins(s, pwork, tu.one_stream, [&](int b, hipStream_t st) -> int {
        SpArgs ab = a;
        ab.bin_begin = pbegin[b];
        ab.count = cnt[b];
        ab.T = num_table((b - 1) % kNumT);
        ab.vcap = num_vcap(ab.T, tu.load_pct);
        const int64_t gb = num_wave_bytes(false, 0, ab.T, tu.load_pct);
        ab.group_bytes = (int)gb;
        int blocks, threads;
        size_t lds;
        geometry(gb, cnt[b], &blocks, &threads, &lds, true);
        const int e = ensure_lds(lds, tu.lds_budget);
        if (e) return e;
        HCSP_HIP(launch_num_pred(ab, blocks, threads, lds, st));
        return HCSP_OK;
    });
    if (rc) return rc;
    // 3. rows the prediction did not hold: exact symbolic (it also scans every
    //    row's count into offsets), else just the scan
    int64_t novf = 0, nnz = 0;
    HCSP_HIP(launch_mark_overflow(C_row_ptr_d, n, pw.active, pw.novf, s));
    HCSP_HIP(hipMemcpyAsync(&novf, pw.novf, 8, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));
    hcsp_sym_info info;
    if (novf > 0) {
        rc = symbolic_impl(&op, B, opts, C_row_ptr_d, &info, ws_d, base, stream, pw.active);
        if (rc) return rc;
        nnz = info.nnz;
    } else {
        HCSP_HIP(launch_scan_exclusive(C_row_ptr_d, n + 1, ws.scan_tmp, s));
        HCSP_HIP(hipMemcpyAsync(&nnz, C_row_ptr_d + n, 8, hipMemcpyDeviceToHost, s));
        HCSP_HIP(hipStreamSynchronize(s));
    }
    if (nnz_h) *nnz_h = nnz;
    if (n_overflow_h) *n_overflow_h = novf;
    if (nnz > capacity) return fail(HCSP_E_CAPACITY, "C capacity smaller than nnz(C) = " + std::to_string(nnz));
    // 4. the other rows computed exactly; predicted rows to their exact place
    if (novf > 0) {
        hcsp_opts o2;
        std::memset(&o2, 0, sizeof o2);
        if (opts) o2 = *opts;
        o2.flags &= ~HCSP_F_SYNC_CHECK;
        o2.unit_lo = 0;
        o2.unit_hi = 0;
        o2.out_base = 0;
        rc = hcsp_spgemm_numeric(&op, B, &o2, &info, C_row_ptr_d, C_col_d, C_val_d, capacity, ws_d, base, stream);
        if (rc) return rc;
    } else {
        HCSP_HIP(launch_fill_u32(ws.err, 1, 0u, s));
    }
    HCSP_HIP(launch_copy_rows(pw.pad_off, pw.scol, pw.sval, C_row_ptr_d, pw.active, n, C_col_d, C_val_d, capacity,
                              ws.err, s));
    uint32_t e = 0;
    HCSP_HIP(hipMemcpyAsync(&e, ws.err, 4, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));
    if (e & kErrCapacity) return fail(HCSP_E_CAPACITY, "output capacity too small");
    if (e & kErrCount) return fail(HCSP_E_INVALID, "row counts differ between the phases (inputs changed?)");
    return HCSP_OK;
}

int hcsp_spgemm_predicted(const hcsp_csr *A, const hcsp_csr *B, const hcsp_opts *opts, float ratio,
                          int64_t products, int64_t *C_row_ptr_d, int32_t *C_col_d, double *C_val_d,
                          int64_t capacity, int64_t *nnz_h, int64_t *n_overflow_h, void *ws_d, size_t ws_bytes,
                          void *stream)
{
    clear_error();
    if (!(ratio > 0.0f && ratio <= 1.0f) || products < 0)
        return fail(HCSP_E_INVALID, "bad arguments (ratio must be in (0, 1])");
    return predicted_impl(A, B, opts, ratio, nullptr, pred_entries(ratio, products, A ? A->nrows : 0), C_row_ptr_d,
                          C_col_d, C_val_d, capacity, nnz_h, n_overflow_h, ws_d, ws_bytes, stream);
}

int hcsp_spgemm_predicted_rows(const hcsp_csr *A, const hcsp_csr *B, const hcsp_opts *opts,
                               const int32_t *cap_row_d, int64_t cap_sum, int64_t *C_row_ptr_d, int32_t *C_col_d,
                               double *C_val_d, int64_t capacity, int64_t *nnz_h, int64_t *n_overflow_h, void *ws_d,
                               size_t ws_bytes, void *stream)
{
    clear_error();
    if (!cap_row_d || cap_sum < 0) return fail(HCSP_E_INVALID, "bad arguments");
    return predicted_impl(A, B, opts, 1.0f, cap_row_d, pred_rows_entries(cap_sum, A ? A->nrows : 0), C_row_ptr_d,
                          C_col_d, C_val_d, capacity, nnz_h, n_overflow_h, ws_d, ws_bytes, stream);
}

// ================================================================ batches

int hcsp_batch_plan_init(int32_t count, const hcsp_batch_item *items, const hcsp_opts *opts, hcsp_batch_plan *plan)
{
    clear_error();
    if (!plan || count < 0 || (count > 0 && !items)) return fail(HCSP_E_INVALID, "bad arguments");
    std::memset(plan, 0, sizeof *plan);
    if (opts) plan->opts = *opts;
    plan->count = count;
    plan->kind = count > 0 ? items[0].A.kind : HCSP_OP_CSR;
    int maxs = 1;
    for (int32_t p = 0; p < count; ++p) {
        OpView v;
        int rc = check_operands(&items[p].A, &items[p].B, &v);
        if (rc) return fail(rc, "batch item " + std::to_string(p) + ": " + g_err);
        if (items[p].A.kind != plan->kind) return fail(HCSP_E_INVALID, "all items of a batch must have the same kind");
        if (v.cluster) maxs = std::max(maxs, (int)std::max<int64_t>(1, items[p].A.cl.max_cluster));
        plan->units += v.nunits;
        plan->rows += v.nrows;
        plan->max_ncols = std::max(plan->max_ncols, items[p].B.ncols);
    }
    if (plan->units >= INT32_MAX) return fail(HCSP_E_OVERFLOW, "a batch holds fewer than 2^31 units");
    plan->row_ptr_len = plan->rows + count;
    plan->max_class = sclass_of(maxs);
    Tune tu;
    hcsp_csr widest;
    std::memset(&widest, 0, sizeof widest);
    widest.ncols = plan->max_ncols;
    int rc = make_tune(&plan->opts, &widest, false, &tu);
    if (rc) return rc;
    BatchWs ws;
    plan->ws_bytes = layout_batch(count, plan->units, plan->row_ptr_len, plan->max_ncols, tu.dense_slots, nullptr, &ws);
    return HCSP_OK;
}

int hcsp_batch_prepare(hcsp_batch_plan *plan, const hcsp_batch_item *items, void *ws_d, size_t ws_bytes,
                       int64_t *out_offset_h, int64_t *seg_offset_h, void *stream)
{
    clear_error();
    if (!plan || (plan->count > 0 && !items)) return fail(HCSP_E_INVALID, "bad arguments");
    hcsp_batch_plan chk;
    int rc = hcsp_batch_plan_init(plan->count, items, &plan->opts, &chk);
    if (rc) return rc;
    if (chk.units != plan->units || chk.rows != plan->rows || chk.ws_bytes != plan->ws_bytes)
        return fail(HCSP_E_INVALID, "items differ from the ones the plan was made for");
    if (!ws_d || ws_bytes < plan->ws_bytes) return fail(HCSP_E_CAPACITY, "batch workspace too small");
    Tune tu;
    hcsp_csr widest;
    std::memset(&widest, 0, sizeof widest);
    widest.ncols = plan->max_ncols;
    rc = make_tune(&plan->opts, &widest, true, &tu);
    if (rc) return rc;
    BatchWs ws;
    layout_batch(plan->count, plan->units, plan->row_ptr_len, plan->max_ncols, tu.dense_slots, (char *)ws_d, &ws);
    hipStream_t s = (hipStream_t)stream;
    const int32_t n = plan->count;
    const bool cl = plan->kind == HCSP_OP_CLUSTER;

    // descriptors with unit / segment bases; capacities follow from the bounds
    std::vector<BatchProb> bp((size_t)std::max(n, 1));
    std::vector<int64_t> ubase((size_t)n + 1), segs((size_t)n + 1);
    int64_t u0 = 0, s0 = 0;
    for (int32_t p = 0; p < n; ++p) {
        BatchProb &d = bp[(size_t)p];
        std::memset(&d, 0, sizeof d);
        const hcsp_operand &A = items[p].A;
        const hcsp_csr &B = items[p].B;
        if (cl) {
            d.cl_row_ptr = A.cl.cl_row_ptr;
            d.perm = A.cl.perm;
            d.cl_col_ptr = A.cl.cl_col_ptr;
            d.cl_col = A.cl.cl_col;
            d.cl_mask = A.cl.cl_mask;
            d.cl_val_ptr = A.cl.cl_val_ptr;
            d.cl_val = A.cl.cl_val;
            d.nunits = A.cl.nclusters;
            d.nrows = A.cl.nrows;
        } else {
            d.a_rp = A.csr.row_ptr;
            d.a_col = A.csr.col;
            d.a_val = A.csr.val;
            d.nunits = A.csr.nrows;
            d.nrows = A.csr.nrows;
        }
        d.b_rp = B.row_ptr;
        d.b_col = B.col;
        d.b_val = B.val;
        d.ncols = B.ncols;
        d.unit_base = u0;
        d.seg_base = s0;
        ubase[(size_t)p] = u0;
        segs[(size_t)p] = s0;
        u0 += d.nunits;
        s0 += d.nrows + 1;
    }
    ubase[(size_t)n] = u0;
    segs[(size_t)n] = s0;
    HCSP_HIP(hipMemcpyAsync(ws.units, ubase.data(), 8 * ((size_t)n + 1), hipMemcpyHostToDevice, s));
    HCSP_HIP(hipMemcpyAsync(ws.segs, segs.data(), 8 * ((size_t)n + 1), hipMemcpyHostToDevice, s));
    HCSP_HIP(hipMemcpyAsync(ws.probs, bp.data(), sizeof(BatchProb) * (size_t)n, hipMemcpyHostToDevice, s));
    HCSP_HIP(launch_fill_i64(ws.ub, n, 0, s));
    HCSP_HIP(launch_batch_bound(ws.probs, n, cl, ws.ub, s));
    // the largest unit bounds which bins a batched call can reach
    BinArgs ba = batch_bin_args(*plan, ws, tu, nullptr);
    HCSP_HIP(launch_fill_i64(ws.maxp, 1, 0, s));
    HCSP_HIP(launch_work(cl, ba, s));
    HCSP_HIP(launch_max_i64(ws.w.probes, plan->units, ws.maxp, s));
    std::vector<int64_t> ub((size_t)std::max(n, 1));
    int64_t maxp = 0;
    HCSP_HIP(hipMemcpyAsync(ub.data(), ws.ub, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipMemcpyAsync(&maxp, ws.maxp, 8, hipMemcpyDeviceToHost, s));
    HCSP_HIP(hipStreamSynchronize(s));
    int64_t off = 0;
    for (int32_t p = 0; p < n; ++p) {
        bp[(size_t)p].out_base = off;
        bp[(size_t)p].cap = ub[(size_t)p];
        if (out_offset_h) out_offset_h[p] = off;
        off += ub[(size_t)p];
    }
    if (out_offset_h) out_offset_h[n] = off;
    if (seg_offset_h)
        for (int32_t p = 0; p <= n; ++p) seg_offset_h[p] = segs[(size_t)p];
    HCSP_HIP(hipMemcpyAsync(ws.probs, bp.data(), sizeof(BatchProb) * (size_t)n, hipMemcpyHostToDevice, s));
    HCSP_HIP(hipStreamSynchronize(s));
    plan->max_probes = maxp;
    plan->out_capacity = off;
    plan->prepared = 1;
    return HCSP_OK;
}

int hcsp_spgemm_batched(const hcsp_batch_plan *plan, int64_t *C_row_ptr_d, int32_t *C_col_d, double *C_val_d,
                        void *ws_d, size_t ws_bytes, void *stream)
{
    clear_error();
    if (!plan || !plan->prepared) return fail(HCSP_E_INVALID, "the plan was not prepared");
    if (!ws_d || ws_bytes < plan->ws_bytes) return fail(HCSP_E_CAPACITY, "batch workspace too small");
    if (plan->count == 0) return HCSP_OK;
    if (!C_row_ptr_d || (plan->out_capacity > 0 && (!C_col_d || !C_val_d)))
        return fail(HCSP_E_INVALID, "null output array");
    Tune tu;
    hcsp_csr widest;
    std::memset(&widest, 0, sizeof widest);
    widest.ncols = plan->max_ncols;
    int rc = make_tune(&plan->opts, &widest, true, &tu);
    if (rc) return rc;
    BatchWs ws;
    layout_batch(plan->count, plan->units, plan->row_ptr_len, plan->max_ncols, tu.dense_slots, (char *)ws_d, &ws);
    hipStream_t s = (hipStream_t)stream;
    const int32_t n = plan->count;
    const bool cl = plan->kind == HCSP_OP_CLUSTER;
    const int ncu = cu_count();

    HCSP_HIP(launch_fill_i64(ws.w.sym_count, HCSP_MAX_BINS, 0, s));
    HCSP_HIP(launch_fill_i64(ws.w.num_count, HCSP_MAX_BINS, 0, s));
    HCSP_HIP(launch_fill_u32(ws.errs, n, 0u, s));

    SpArgs a;
    std::memset(&a, 0, sizeof a);
    a.keylo = ws.w.keylo;
    a.keyhi = ws.w.keyhi;
    a.ucount = ws.w.ucount;
    a.c_rp = C_row_ptr_d;
    a.G = tu.G;
    a.dense_bits = ws.w.dense_bits;
    a.dense_vals = ws.w.dense_vals;
    a.dense_words = ws.w.dense_words;
    a.ncols = plan->max_ncols;
    a.unit_lo = 0;
    a.unit_hi = INT64_MAX;
    a.batch = ws.probs;
    a.batch_units = ws.units;
    a.nprob = n;
    a.errs = ws.errs;
    a.err = ws.errs;

    // persistent launch of one bin: enough wavefronts to fill every compute
    // unit the bin's shared memory allows, never more than the batch's units
    auto persistent = [&](int64_t wave_bytes, int *blocks, int *threads, size_t *lds) {
        int b0;
        geometry(wave_bytes, 1, &b0, threads, lds);
        const int wpb = *threads / 64;
        const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(32 / wpb, (160 * 1024) / (int64_t)*lds));
        *blocks = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)ncu * per_cu, (plan->units + wpb - 1) / wpb));
    };

    // ---- symbolic
    BinArgs ba = batch_bin_args(*plan, ws, tu, C_row_ptr_d);
    HCSP_HIP(launch_work(cl, ba, s));
    HCSP_HIP(launch_scatter(ws.w.bin, plan->units, ws.w.bin_hist, kSymBins, ws.w.sym_count, ws.w.order_sym, s));
    HCSP_HIP(launch_bin_begin(ws.w.sym_count, kSymBins, ws.sym_begin, s));
    a.order = ws.w.order_sym;
    a.dcount = ws.w.sym_count;
    a.dbegin = ws.sym_begin;
    const int64_t sym_need = (plan->max_probes * 100 + tu.sym_load_pct - 1) / tu.sym_load_pct;
    int sym_l2 = kSymLog2Min;
    while (sym_l2 < tu.sym_tmax_log2 && ((int64_t)1 << sym_l2) < sym_need) ++sym_l2;
    for (int sc = 0; sc <= (cl ? plan->max_class : 0); ++sc) {
        for (int l2 = kSymLog2Min; l2 <= sym_l2; ++l2) {
            a.bin = 1 + sc * kSymT + (l2 - kSymLog2Min);
            a.T = 1 << l2;
            a.log2T = l2;
            const int64_t gb = sym_wave_bytes(cl ? mask_bytes_of_class(sc) : 0, a.T);
            a.group_bytes = (int)gb;
            int blocks, threads;
            size_t lds;
            persistent(gb, &blocks, &threads, &lds);
            rc = ensure_lds(lds, tu.lds_budget);
            if (rc) return rc;
            HCSP_HIP(launch_sym(sc, cl, true, a, blocks, threads, lds, s));
        }
    }
    const bool dense = sym_need > ((int64_t)1 << tu.sym_tmax_log2);
    if (dense) {
        a.bin = kSymGlobal;
        HCSP_HIP(launch_fill_u32(ws.w.dense_bits, (int64_t)tu.dense_slots * ws.w.dense_words, 0u, s));
        HCSP_HIP(launch_sym_dense(cl, true, a, tu.dense_slots / 4, s));
    }
    // ---- per-product row offsets
    HCSP_HIP(launch_batch_seg_tail(ws.probs, n, C_row_ptr_d, s));
    HCSP_HIP(launch_scan_exclusive(C_row_ptr_d, plan->row_ptr_len, ws.w.scan_tmp, s));
    HCSP_HIP(launch_batch_seg_rebase(ws.probs, ws.segs, n, C_row_ptr_d, plan->row_ptr_len, ws.seg_base, ws.nnz, s));
    // ---- numeric
    HCSP_HIP(launch_numbin(cl, ba, s));
    HCSP_HIP(launch_scatter(ws.w.bin, plan->units, ws.w.bin_hist, kNumBins, ws.w.num_count, ws.w.order_num, s));
    HCSP_HIP(launch_bin_begin(ws.w.num_count, kNumBins, ws.num_begin, s));
    a.order = ws.w.order_num;
    a.dcount = ws.w.num_count;
    a.dbegin = ws.num_begin;
    a.c_col = C_col_d;
    a.c_val = C_val_d;
    int tmax[kSClasses];
    num_tmax_classes(tu, cl, tmax);
    const int64_t need = (plan->max_probes * 100 + tu.load_pct - 1) / tu.load_pct;
    bool num_dense = dense;
    for (int sc = 0; sc <= (cl ? plan->max_class : 0); ++sc) {
        for (int t = 0; t < kNumT; ++t) {
            const int T = num_table(t);
            if (T > tmax[sc]) {
                num_dense = true;
                break;
            }
            a.bin = 1 + sc * kNumT + t;
            a.T = T;
            a.vcap = num_vcap(T, tu.load_pct);
            const int64_t gb = num_wave_bytes(cl, sc, T, tu.load_pct);
            a.group_bytes = (int)gb;
            int blocks, threads;
            size_t lds;
            persistent(gb, &blocks, &threads, &lds);
            rc = ensure_lds(lds, tu.lds_budget);
            if (rc) return rc;
            HCSP_HIP(launch_num(sc, cl, true, a, blocks, threads, lds, s));
            if (T >= need) break;
        }
    }
    if (num_dense) {
        a.bin = kNumGlobal;
        HCSP_HIP(launch_fill_u32(ws.w.dense_bits, (int64_t)tu.dense_slots * ws.w.dense_words, 0u, s));
        HCSP_HIP(launch_num_dense(cl, true, a, tu.dense_slots / 4, s));
    }
    return HCSP_OK;
}

int hcsp_batch_status(const hcsp_batch_plan *plan, void *ws_d, size_t ws_bytes, int64_t *nnz_h, void *stream)
{
    clear_error();
    if (!plan || !plan->prepared) return fail(HCSP_E_INVALID, "the plan was not prepared");
    if (!ws_d || ws_bytes < plan->ws_bytes) return fail(HCSP_E_CAPACITY, "batch workspace too small");
    Tune tu;
    hcsp_csr widest;
    std::memset(&widest, 0, sizeof widest);
    widest.ncols = plan->max_ncols;
    int rc = make_tune(&plan->opts, &widest, false, &tu);
    if (rc) return rc;
    BatchWs ws;
    layout_batch(plan->count, plan->units, plan->row_ptr_len, plan->max_ncols, tu.dense_slots, (char *)ws_d, &ws);
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)plan->count;
    std::vector<uint32_t> e(std::max<size_t>(n, 1));
    std::vector<int64_t> z(std::max<size_t>(n, 1));
    if (n) {
        HCSP_HIP(hipMemcpyAsync(e.data(), ws.errs, 4 * n, hipMemcpyDeviceToHost, s));
        HCSP_HIP(hipMemcpyAsync(z.data(), ws.nnz, 8 * n, hipMemcpyDeviceToHost, s));
    }
    HCSP_HIP(hipStreamSynchronize(s));
    if (nnz_h)
        for (size_t p = 0; p < n; ++p) nnz_h[p] = z[p];
    for (size_t p = 0; p < n; ++p) {
        if (e[p] & kErrCapacity) return fail(HCSP_E_CAPACITY, "product " + std::to_string(p) + ": output bound exceeded");
        if (e[p] & kErrCount)
            return fail(HCSP_E_INVALID, "product " + std::to_string(p) + ": row counts differ between the phases");
    }
    return HCSP_OK;
}

}  // extern "C"
