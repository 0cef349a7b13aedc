// Support kernels: fills, per-unit work estimate and binning, counting-sort
// scatter of units into bins, a device-wide exclusive scan (int64), and CSR
// validation.
#include <algorithm>
#include <climits>

#include "device.h"
#include "internal.h"
#include "unit.h"

namespace hcsp {

// ------------------------------------------------------------------ fills
template <class T>
__global__ void k_fill(T *p, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
static hipError_t fill(T *p, int64_t n, T v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s) { return fill(p, n, v, s); }
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) { return fill(p, n, v, s); }
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) { return fill(p, n, v, s); }

__global__ void k_gather_words(int64_t *dst, GatherWords g)
{
    const int i = (int)threadIdx.x;
    if (i < g.n)
        dst[i] = g.bytes[i] == 8 ? *(const int64_t *)g.src[i] : (int64_t) * (const uint32_t *)g.src[i];
}

hipError_t launch_gather_words(int64_t *dst, const GatherWords &g, hipStream_t s)
{
    if (g.n < 1 || g.n > 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather_words, dim3(1), dim3(64), 0, s, dst, g);
    return hipGetLastError();
}

__global__ void k_sym_start(const int64_t *rp, int64_t n, uint16_t *out, int64_t *z0, int64_t *z1, int nz,
                            uint32_t *err, int64_t *z2)
{
    if (blockIdx.x == 0) {
        for (int i = (int)threadIdx.x; i < nz; i += blockDim.x) {
            z0[i] = 0;
            z1[i] = 0;
        }
        if (threadIdx.x == 0) {
            *err = 0u;
            *z2 = 0;
        }
    }
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = (uint16_t)min<int64_t>(rp[k + 1] - rp[k], 65535);
}

hipError_t launch_sym_start(const int64_t *rp, int64_t n, uint16_t *out, int64_t *z0, int64_t *z1, int nz,
                            uint32_t *err, int64_t *z2, hipStream_t s)
{
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
    hipLaunchKernelGGL(k_sym_start, dim3((unsigned)blocks), dim3(256), 0, s, rp, std::max<int64_t>(n, 0), out, z0,
                       z1, nz, err, z2);
    return hipGetLastError();
}

// ------------------------------------------------------------------ binning
__device__ __forceinline__ int ceil_log2(int64_t x)
{
    int l = 0;
    while (((int64_t)1 << l) < x) ++l;
    return l;
}

// Table size: the smallest power of two with at least probes*100/load_pct
// slots (the product count bounds the number of distinct columns).
__device__ __forceinline__ int sym_bin(int sc, int64_t probes, int tmax_log2, int load_pct)
{
    int l = ceil_log2((probes * 100 + load_pct - 1) / load_pct);
    if (l < kSymLog2Min) l = kSymLog2Min;
    if (l > tmax_log2) return kSymGlobal;
    return 1 + sc * kSymT + (l - kSymLog2Min);
}

// Units are split into kBinBlocks contiguous chunks, one per block.  Each
// block counts its units per bin in shared memory and stores the counts as
// one row of a [blocks x bins] matrix (no global atomics); k_binscan turns
// the matrix into per-block starting offsets, and k_scatter places units so
// that a bin lists the units of block 0 first, then block 1, and so on.
__device__ __forceinline__ void chunk_of(int64_t n, int64_t *b, int64_t *e)
{
    const int64_t ch = (n + gridDim.x - 1) / gridDim.x;
    *b = min(n, (int64_t)blockIdx.x * ch);
    *e = min(n, *b + ch);
}

// A unit's arrays for the work estimate: the unit's own product, or in a
// batch the product holding batch-wide unit g.
struct WorkView {
    const int64_t *b_rp;
    const uint16_t *b_len;  // B's row lengths saturated at 65535 (nullable)
    const int32_t *col;     // A's columns, or the cluster's union columns
    const int32_t *perm;
    int64_t *c_rp;
    int64_t it0, it1, pos0, u;
    int s;
};

template <bool CL, bool BATCH>
__device__ __forceinline__ WorkView work_view(const BinArgs &a, int64_t g)
{
    WorkView w;
    const int64_t *a_rp = a.a_rp, *cl_row_ptr = a.cl_row_ptr, *cl_col_ptr = a.cl_col_ptr;
    w.b_rp = a.b_rp;
    w.b_len = BATCH ? nullptr : a.b_len;
    w.col = CL ? a.cl_col : a.a_col;
    w.perm = a.perm;
    w.c_rp = a.c_rp;
    w.u = g;
    if (BATCH) {
        const int p = batch_find(a.batch_units, a.nprob, g);
        const BatchProb &bp = a.batch[p];
        a_rp = global_ptr(bp.a_rp);
        cl_row_ptr = global_ptr(bp.cl_row_ptr);
        cl_col_ptr = global_ptr(bp.cl_col_ptr);
        w.b_rp = global_ptr(bp.b_rp);
        w.col = global_ptr(CL ? bp.cl_col : bp.a_col);
        w.perm = global_ptr(bp.perm);
        w.c_rp = a.c_rp + bp.seg_base;
        w.u = g - bp.unit_base;
    }
    if (CL) {
        w.it0 = cl_col_ptr[w.u];
        w.it1 = cl_col_ptr[w.u + 1];
        w.pos0 = cl_row_ptr[w.u];
        w.s = (int)(cl_row_ptr[w.u + 1] - w.pos0);
    } else {
        w.it0 = a_rp[w.u];
        w.it1 = a_rp[w.u + 1];
        w.pos0 = w.u;
        w.s = 1;
    }
    return w;
}

// One group of 8 lanes per unit: probes = sum of |B_k| over the unit's
// columns k (an upper bound on its distinct output columns) and its
// symbolic bin.  Units with no products get their zero row counts here.
template <bool CL, bool BATCH>
__global__ void __launch_bounds__(256) k_work(BinArgs a)
{
    __shared__ int hist[kSymBins];
    for (int i = threadIdx.x; i < kSymBins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    constexpr int G = 8;
    const Group g = make_group(G);
    int64_t cb, ce;
    chunk_of(a.nunits, &cb, &ce);
    for (int64_t u = cb + (threadIdx.x / G); u < ce; u += blockDim.x / G) {
        const WorkView w = work_view<CL, BATCH>(a, u);
        int64_t probes = 0;
        // a row of B's length, from the 2-byte lengths where they are given and
        // below the saturation value
        auto blen = [&](int k) -> int64_t {
            if (w.b_len) {
                const int l = w.b_len[k];
                if (l < 65535) return l;
            }
            return w.b_rp[k + 1] - w.b_rp[k];
        };
        // two items per lane and step, so that both items' loads are in flight together
        int64_t q = w.it0 + g.gl;
        for (; q + G < w.it1; q += 2 * G) {
            const int k0 = w.col[q], k1 = w.col[q + G];
            probes += blen(k0) + blen(k1);
        }
        if (q < w.it1) probes += blen(w.col[q]);
        probes = gsum64(g, probes);
        const bool on = !a.active || a.active[u];
        if (!on) probes = 0;
        const int bin = probes == 0 ? kBinEmpty : sym_bin(sclass_of(w.s), probes, a.sym_tmax_log2, a.sym_load_pct);
        if (g.gl == 0) {
            a.ws.probes[u] = probes;
            a.ws.bin[u] = (uint8_t)bin;
            atomicAdd(&hist[bin], 1);
            if (bin == kBinEmpty) {
                a.ws.ucount[u] = 0;
                if (a.c_rp && on)  // null: estimate only; inactive units keep their count
                    for (int l = 0; l < w.s; ++l) w.c_rp[CL ? (int64_t)w.perm[w.pos0 + l] : w.u] = 0;
            } else if (!BATCH && bin == kSymGlobal && a.c_rp) {
                // the column-window chunks add their counts to the rows
                for (int l = 0; l < w.s; ++l) w.c_rp[CL ? (int64_t)w.perm[w.pos0 + l] : w.u] = 0;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSymBins; i += blockDim.x) a.ws.bin_hist[(int64_t)blockIdx.x * HCSP_MAX_BINS + i] = hist[i];
}

int bin_blocks(int64_t nunits)
{
    const int64_t b = (nunits + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(kBinBlocks, b));
}

hipError_t launch_work(bool cluster, const BinArgs &a, hipStream_t s)
{
    if (a.nunits <= 0) return hipSuccess;
    const int blocks = bin_blocks(a.nunits);
    const bool batch = a.batch != nullptr;
    if (cluster && batch) hipLaunchKernelGGL((k_work<true, true>), dim3(blocks), dim3(256), 0, s, a);
    else if (cluster) hipLaunchKernelGGL((k_work<true, false>), dim3(blocks), dim3(256), 0, s, a);
    else if (batch) hipLaunchKernelGGL((k_work<false, true>), dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_work<false, false>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Numeric bin from the exact number of distinct output columns found by the
// symbolic phase: the smallest table that keeps the fill below load_pct.
template <bool CL, bool BATCH>
__global__ void __launch_bounds__(256) k_numbin(BinArgs a)
{
    __shared__ int hist[kNumBins];
    for (int i = threadIdx.x; i < kNumBins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    int64_t cb, ce;
    chunk_of(a.nunits, &cb, &ce);
    for (int64_t u = cb + threadIdx.x; u < ce; u += blockDim.x) {
        int s = 1;
        if (CL) {
            const WorkView w = work_view<CL, BATCH>(a, u);
            s = w.s;
        }
        const int sc = sclass_of(s);
        const int32_t U = a.ws.ucount[u];
        int bin;
        if (a.ws.probes[u] == 0 || U == 0) {
            bin = kBinEmpty;
        } else if (U == INT32_MAX) {
            bin = kNumGlobal;
        } else {
            const int64_t need = ((int64_t)U * 100 + a.load_pct - 1) / a.load_pct;
            bin = kNumGlobal;
            for (int t = 0; t < kNumT; ++t) {
                const int T = num_table(t);
                if (T > a.num_tmax_by_class[sc]) break;
                if (T >= need) {
                    bin = 1 + sc * kNumT + t;
                    break;
                }
            }
        }
        a.ws.bin[u] = (uint8_t)bin;
        atomicAdd(&hist[bin], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNumBins; i += blockDim.x) a.ws.bin_hist[(int64_t)blockIdx.x * HCSP_MAX_BINS + i] = hist[i];
}

hipError_t launch_numbin(bool cluster, const BinArgs &a, hipStream_t s)
{
    if (a.nunits <= 0) return hipSuccess;
    const int blocks = bin_blocks(a.nunits);
    const bool batch = a.batch != nullptr;
    if (cluster && batch) hipLaunchKernelGGL((k_numbin<true, true>), dim3(blocks), dim3(256), 0, s, a);
    else if (cluster) hipLaunchKernelGGL((k_numbin<true, false>), dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_numbin<false, false>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ predicted sizes
// Sum over A's entries (i, k) of |B_k|: the number of products of A x B.
__global__ void __launch_bounds__(256) k_products(const int64_t *a_rp, const int32_t *a_col, int64_t nnz,
                                                  const int64_t *b_rp, int64_t *out)
{
    int64_t s = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
        const int k = a_col[q];
        s += b_rp[k + 1] - b_rp[k];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd((unsigned long long *)out, (unsigned long long)s);
}

hipError_t launch_products(const hcsp_csr &A, const hcsp_csr &B, int64_t *out, hipStream_t s)
{
    if (A.nnz <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((A.nnz + 255) / 256, 4096);
    hipLaunchKernelGGL(k_products, dim3((unsigned)blocks), dim3(256), 0, s, A.row_ptr, A.col, A.nnz, B.row_ptr, out);
    return hipGetLastError();
}

// Per CSR row: products, a column range that holds every output column (the
// smallest first and largest last column over the rows of B it reaches), and
// the predicted capacity min(products, ceil(products * ratio)) -- or the
// caller's per-row capacity clamped to [1, products] -- which picks the
// numeric bin directly (no symbolic phase).  Empty rows get count 0.
__global__ void __launch_bounds__(256) k_work_pred(BinArgs a)
{
    __shared__ int hist[kNumBins];
    for (int i = threadIdx.x; i < kNumBins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const Group g = make_group(16);
    int64_t cb, ce;
    chunk_of(a.nunits, &cb, &ce);
    for (int64_t u = cb + (threadIdx.x >> 4); u < ce; u += blockDim.x >> 4) {
        int64_t probes = 0;
        int lo = INT_MAX, hi = -1;
        for (int64_t q = a.a_rp[u] + g.gl; q < a.a_rp[u + 1]; q += 16) {
            const int k = a.a_col[q];
            const int64_t b0 = a.b_rp[k], b1 = a.b_rp[k + 1];
            if (b1 > b0) {
                probes += b1 - b0;
                const int2 sp = a.b_span ? a.b_span[k] : make_int2(a.b_col[b0], a.b_col[b1 - 1]);
                lo = min(lo, sp.x);
                hi = max(hi, sp.y);
            }
        }
        probes = gsum64(g, probes);
        lo = gmin32(g, lo);
        hi = gmax32(g, hi);
        int bin = kBinEmpty;
        int64_t cap = 0;
        if (probes > 0) {
            cap = a.cap_row ? (int64_t)a.cap_row[u] : (int64_t)ceilf((float)probes * a.ratio);
            cap = max(min(cap, probes), (int64_t)1);
            const int64_t need = (cap * 100 + a.load_pct - 1) / a.load_pct;
            bin = kNumGlobal;
            for (int t = 0; t < kNumT; ++t) {
                const int T = num_table(t);
                if (T > a.num_tmax_by_class[0]) break;
                if (T >= need) {
                    bin = 1 + t;
                    break;
                }
            }
        }
        if (g.gl == 0) {
            a.ws.probes[u] = probes;
            a.ws.keylo[u] = lo;
            a.ws.keyhi[u] = hi;
            a.ws.ucount[u] = (int32_t)cap;
            a.ws.bin[u] = (uint8_t)bin;
            a.pad[u] = bin == kNumGlobal ? 0 : cap;
            if (bin == kBinEmpty || bin == kNumGlobal) a.c_rp[u] = bin == kBinEmpty ? 0 : -1;
            atomicAdd(&hist[bin], 1);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNumBins; i += blockDim.x) a.ws.bin_hist[(int64_t)blockIdx.x * HCSP_MAX_BINS + i] = hist[i];
}

__global__ void __launch_bounds__(256) k_row_span(const int64_t *rp, const int32_t *col, int64_t n, int2 *span)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b0 = rp[k], b1 = rp[k + 1];
        span[k] = b1 > b0 ? make_int2(col[b0], col[b1 - 1]) : make_int2(INT_MAX, -1);
    }
}

hipError_t launch_row_span(const int64_t *rp, const int32_t *col, int64_t n, int2 *span, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_row_span, dim3((unsigned)blocks), dim3(256), 0, s, rp, col, n, span);
    return hipGetLastError();
}

hipError_t launch_work_pred(const BinArgs &a, hipStream_t s)
{
    if (a.nunits <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_work_pred, dim3(bin_blocks(a.nunits)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// active[u] = the predicted pass gave up on row u (count -1); *count += rows.
__global__ void __launch_bounds__(256) k_mark_overflow(const int64_t *c_rp, int64_t n, uint8_t *active, int64_t *count)
{
    int64_t c = 0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const bool o = c_rp[u] < 0;
        active[u] = o;
        c += o;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd((unsigned long long *)count, (unsigned long long)c);
}

hipError_t launch_mark_overflow(const int64_t *c_rp, int64_t n, uint8_t *active, int64_t *count, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_mark_overflow, dim3((unsigned)blocks), dim3(256), 0, s, c_rp, n, active, count);
    return hipGetLastError();
}

// Rows finished by the predicted pass move from their padded slot to their
// exact place in C (one 64-lane group per row).
__global__ void __launch_bounds__(256) k_copy_rows(const int64_t *pad_off, const int32_t *scol, const double *sval,
                                                   const int64_t *c_rp, const uint8_t *active, int64_t n,
                                                   int32_t *C_col, double *C_val, int64_t cap, uint32_t *err)
{
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t u = w0; u < n; u += nw) {
        if (active[u]) continue;
        const int64_t d0 = c_rp[u], len = c_rp[u + 1] - d0, s0 = pad_off[u];
        if (d0 < 0 || d0 + len > cap) {
            if (lane == 0) atomicOr(err, kErrCapacity);
            continue;
        }
        for (int64_t e = lane; e < len; e += 64) {
            C_col[d0 + e] = scol[s0 + e];
            C_val[d0 + e] = sval[s0 + e];
        }
    }
}

hipError_t launch_copy_rows(const int64_t *pad_off, const int32_t *scol, const double *sval, const int64_t *c_rp,
                            const uint8_t *active, int64_t n, int32_t *C_col, double *C_val, int64_t cap,
                            uint32_t *err, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 3) / 4, 16384);
    hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)blocks), dim3(256), 0, s, pad_off, scol, sval, c_rp, active, n,
                       C_col, C_val, cap, err);
    return hipGetLastError();
}

// ------------------------------------------------------------------ batches
// Largest value of x[0..n) into *out (which must hold a value <= it).
__global__ void __launch_bounds__(256) k_max_i64(const int64_t *x, int64_t n, int64_t *out)
{
    int64_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, x[i]);
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) atomicMax((unsigned long long *)out, (unsigned long long)m);
}

hipError_t launch_max_i64(const int64_t *x, int64_t n, int64_t *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_max_i64, dim3((unsigned)blocks), dim3(256), 0, s, x, n, out);
    return hipGetLastError();
}

// Start of every bin in the unit order (exclusive prefix of the bin sizes),
// kept on the device so batch launches need no host read-back.
__global__ void k_bin_begin(const int64_t *counts, int nbins, int64_t *begin)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t acc = 0;
        for (int b = 0; b < nbins; ++b) {
            begin[b] = acc;
            acc += counts[b];
        }
    }
}

hipError_t launch_bin_begin(const int64_t *counts, int nbins, int64_t *begin, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_begin, dim3(1), dim3(64), 0, s, counts, nbins, begin);
    return hipGetLastError();
}

// Upper bound on nnz(C_p) for every product p of a batch: the number of
// products sum_i sum_{k in A_i} |B_k| (a cluster counts every member row that
// has column k).  ub[] must be zero on entry; blockIdx.y splits a product.
template <bool CL>
__global__ void __launch_bounds__(256) k_batch_bound(const BatchProb *batch, int64_t *ub)
{
    const BatchProb &bp = batch[blockIdx.x];
    const int64_t *b_rp = global_ptr(bp.b_rp);
    const int32_t *col = global_ptr(CL ? bp.cl_col : bp.a_col);
    const uint16_t *mask = global_ptr(bp.cl_mask);
    const int64_t n = CL ? (bp.nunits > 0 ? global_ptr(bp.cl_col_ptr)[bp.nunits] : 0)
                         : (bp.nrows > 0 ? global_ptr(bp.a_rp)[bp.nrows] : 0);
    int64_t s = 0;
    for (int64_t q = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.y * blockDim.x) {
        const int k = col[q];
        const int64_t len = b_rp[k + 1] - b_rp[k];
        s += CL ? len * __popc((uint32_t)mask[q]) : len;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd((unsigned long long *)&ub[blockIdx.x], (unsigned long long)s);
}

hipError_t launch_batch_bound(const BatchProb *batch, int nprob, bool cluster, int64_t *ub, hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    const dim3 grid((unsigned)nprob, 16);
    if (cluster) hipLaunchKernelGGL((k_batch_bound<true>), grid, dim3(256), 0, s, batch, ub);
    else hipLaunchKernelGGL((k_batch_bound<false>), grid, dim3(256), 0, s, batch, ub);
    return hipGetLastError();
}

// Row counts of product p sit in flat[seg_base .. seg_base + nrows), with a
// zero after them; one exclusive scan of the whole flat array is then made
// local to every product by subtracting the value at its segment start.
__global__ void k_seg_tail(const BatchProb *batch, int nprob, int64_t *flat)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) flat[batch[p].seg_base + batch[p].nrows] = 0;
}

__global__ void k_seg_base(const BatchProb *batch, int nprob, const int64_t *flat, int64_t *base, int64_t *nnz)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) {
        const int64_t b = flat[batch[p].seg_base];
        base[p] = b;
        nnz[p] = flat[batch[p].seg_base + batch[p].nrows] - b;
    }
}

__global__ void __launch_bounds__(256) k_seg_sub(const int64_t *segs, int nprob, int64_t *flat, int64_t nflat,
                                                 const int64_t *base)
{
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < nflat; x += (int64_t)gridDim.x * blockDim.x)
        flat[x] -= base[batch_find(segs, nprob, x)];
}

hipError_t launch_batch_seg_tail(const BatchProb *batch, int nprob, int64_t *flat, hipStream_t s)
{
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_tail, dim3((nprob + 255) / 256), dim3(256), 0, s, batch, nprob, flat);
    return hipGetLastError();
}

hipError_t launch_batch_seg_rebase(const BatchProb *batch, const int64_t *segs, int nprob, int64_t *flat,
                                   int64_t nflat, int64_t *base, int64_t *nnz, hipStream_t s)
{
    if (nprob <= 0 || nflat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_base, dim3((nprob + 255) / 256), dim3(256), 0, s, batch, nprob, flat, base, nnz);
    const int64_t blocks = std::min<int64_t>((nflat + 255) / 256, 8192);
    hipLaunchKernelGGL(k_seg_sub, dim3((unsigned)blocks), dim3(256), 0, s, segs, nprob, flat, nflat, base);
    return hipGetLastError();
}

// Column b of the [blocks x bins] count matrix becomes its exclusive prefix
// (the offset of each block inside bin b), and counts[b] its total.
__global__ void __launch_bounds__(1024) k_bincol(int32_t *hist, int nblocks, int64_t *counts)
{
    __shared__ int wsum[16];
    const int b = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int carry = 0;
    for (int c0 = 0; c0 < nblocks; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const int v = i < nblocks ? hist[(int64_t)i * HCSP_MAX_BINS + b] : 0;
        int inc = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        int wb = 0, tot = 0;
        for (int x = 0; x < 16; ++x) {
            if (x < w) wb += wsum[x];
            tot += wsum[x];
        }
        if (i < nblocks) hist[(int64_t)i * HCSP_MAX_BINS + b] = carry + wb + inc - v;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[b] = carry;
}

// Scatter: each block hands out positions from its own per-bin offsets
// (bin start + the block's offset inside the bin).
__global__ void __launch_bounds__(256) k_scatter(const uint8_t *bin, int64_t n, const int32_t *hist, int nbins,
                                                 const int64_t *counts, int32_t *order)
{
    __shared__ int cursor[HCSP_MAX_BINS];
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int x = 0; x < nbins; ++x) {
            cursor[x] = (int)acc;
            acc += counts[x];
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < nbins; x += blockDim.x) cursor[x] += hist[(int64_t)blockIdx.x * HCSP_MAX_BINS + x];
    __syncthreads();
    int64_t cb, ce;
    chunk_of(n, &cb, &ce);
    for (int64_t u = cb + threadIdx.x; u < ce; u += blockDim.x) {
        const int b = bin[u];
        const int pos = atomicAdd(&cursor[b], 1);
        if (pos >= 0 && pos < n) order[pos] = (int32_t)u;
    }
}

hipError_t launch_scatter(const uint8_t *bin, int64_t n, int32_t *hist, int nbins, int64_t *counts, int32_t *order,
                          hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int blocks = bin_blocks(n);
    hipLaunchKernelGGL(k_bincol, dim3(nbins), dim3(1024), 0, s, hist, blocks, counts);
    hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(256), 0, s, bin, n, hist, nbins, counts, order);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int64_t kScanChunk = (int64_t)kScanThreads * kScanItems;

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + kScanChunk - 1) / kScanChunk) + 1; }

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ int64_t block_exclusive(int64_t v, int64_t *out)
{
    __shared__ int64_t wsum[kScanThreads / kWave];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int64_t wbase = 0, tot = 0;
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        if (i < w) wbase += wsum[i];
        tot += wsum[i];
    }
    *out = wbase + inc - v;
    __syncthreads();
    return tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const int64_t *d, int64_t n, int64_t *tmp)
{
    const int64_t b0 = (int64_t)blockIdx.x * kScanChunk;
    int64_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t x = b0 + (int64_t)i * kScanThreads + threadIdx.x;
        if (x < n) s += d[x];
    }
    int64_t ex;
    const int64_t tot = block_exclusive(s, &ex);
    if (threadIdx.x == 0) tmp[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_top(int64_t *tmp, int64_t nb)
{
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
        const int64_t x = c0 + threadIdx.x;
        const int64_t v = x < nb ? tmp[x] : 0;
        int64_t ex;
        const int64_t tot = block_exclusive(v, &ex);
        if (x < nb) tmp[x] = carry + ex;
        carry += tot;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_down(int64_t *d, int64_t n, const int64_t *tmp)
{
    const int64_t b0 = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t x = b0 + i;
        v[i] = x < n ? d[x] : 0;
        s += v[i];
    }
    int64_t ex;
    block_exclusive(s, &ex);
    int64_t run = tmp[blockIdx.x] + ex;
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t x = b0 + i;
        if (x < n) d[x] = run;
        run += v[i];
    }
}

hipError_t launch_scan_exclusive(int64_t *data, int64_t n, int64_t *tmp, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    // k_scan_reduce sums strided chunks; k_scan_down scans contiguous ones: both
    // cover block b's elements [b*chunk, (b+1)*chunk), so the block totals agree.
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, tmp);
    return hipGetLastError();
}

// ------------------------------------------------------------------ validation
__global__ void __launch_bounds__(256) k_csr_check(const int64_t *rp, const int32_t *col, int64_t nrows,
                                                   int64_t ncols, int64_t nnz, uint32_t *flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rp[0] != 0 || rp[nrows] != nnz)) atomicOr(flags, kErrPtr);
    if (i >= nrows) return;
    const int64_t b = rp[i], e = rp[i + 1];
    if (b > e || b < 0 || e > nnz) {
        atomicOr(flags, kErrPtr);
        return;
    }
    int prev = -1;
    uint32_t f = 0;
    for (int64_t p = b; p < e; ++p) {
        const int c = col[p];
        if (c < 0 || (int64_t)c >= ncols) f |= kErrRange;
        if (c <= prev) f |= kErrUnsorted;
        prev = c;
    }
    if (f) atomicOr(flags, f);
}

hipError_t launch_csr_check(const hcsp_csr &A, uint32_t *flags, hipStream_t s)
{
    const int64_t blocks = (A.nrows + 256) / 256;
    hipLaunchKernelGGL(k_csr_check, dim3((unsigned)blocks), dim3(256), 0, s, A.row_ptr, A.col, A.nrows, A.ncols,
                       A.nnz, flags);
    return hipGetLastError();
}

// ------------------------------------------------------- CSR_Cluster output
__global__ void __launch_bounds__(256) k_cl_out_counts(const int32_t *ucount, const int64_t *cl_row_ptr, int64_t n,
                                                       int64_t *colp, int64_t *valp, uint32_t *err)
{
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n; u += (int64_t)gridDim.x * blockDim.x) {
        if (u == n) {
            colp[n] = 0;
            valp[n] = 0;
            continue;
        }
        const int32_t U = ucount[u];
        if (U == INT32_MAX) atomicOr(err, 1u);
        const int64_t c = U == INT32_MAX ? 0 : U;
        colp[u] = c;
        valp[u] = c * (cl_row_ptr[u + 1] - cl_row_ptr[u]);
    }
}

hipError_t launch_cl_out_counts(const int32_t *ucount, const int64_t *cl_row_ptr, int64_t nunits, int64_t *colp,
                                int64_t *valp, uint32_t *err, hipStream_t s)
{
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(4096, (nunits + 256) / 256));
    hipLaunchKernelGGL(k_cl_out_counts, dim3((unsigned)blocks), dim3(256), 0, s, ucount, cl_row_ptr, nunits, colp,
                       valp, err);
    return hipGetLastError();
}

// ------------------------------------------------------- SpGEMM_TopK (Alg. 3)
// One wavefront per row i of the overlap matrix O = A A^T (values: the
// number of columns rows i and j share): among the j != i with
// J = ov / (|S_i| + |S_j| - ov) strictly above num/den it picks the topk best
// by (J descending, position of j ascending), one per round: every lane
// takes the best of its strided share that comes after the previous pick,
// then the wavefront keeps the best of the lanes.  Comparisons are exact
// (cross-multiplied 64-bit integers).  Results go to row i's position.
struct TkCand {
    int64_t ov, un;
    int32_t p;  // -1: none
};

__device__ __forceinline__ bool tk_better(const TkCand &a, const TkCand &b)  // a before b
{
    if (a.p < 0) return false;
    if (b.p < 0) return true;
    const int64_t l = a.ov * b.un, r = b.ov * a.un;
    return l > r || (l == r && a.p < b.p);
}

__global__ void __launch_bounds__(256) k_topk(const int64_t *o_rp, const int32_t *o_col, const double *o_val,
                                              const int64_t *a_rp, const int32_t *pos, int64_t n, int64_t num,
                                              int64_t den, int topk, int32_t *cnt, int32_t *nbr, int64_t *nov)
{
    const int lane = (int)__lane_id();
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= n) return;
    const int64_t b0 = o_rp[i], b1 = o_rp[i + 1];
    const int64_t li = a_rp[i + 1] - a_rp[i];
    const int64_t pi = pos ? pos[i] : i;
    TkCand last{0, 1, -1};
    int k = 0;
    for (; k < topk; ++k) {
        TkCand best{0, 1, -1};
        for (int64_t e = b0 + lane; e < b1; e += 64) {
            const int32_t j = o_col[e];
            if (j == i) continue;
            const int64_t ov = (int64_t)o_val[e];
            const TkCand c{ov, li + (a_rp[j + 1] - a_rp[j]) - ov, pos ? pos[j] : j};
            if (ov * den <= c.un * num) continue;  // J not above the threshold
            if (last.p >= 0 && !tk_better(last, c)) continue;
            if (tk_better(c, best)) best = c;
        }
        for (int o = 32; o > 0; o >>= 1) {
            TkCand x;
            x.ov = __shfl_xor(best.ov, o);
            x.un = __shfl_xor(best.un, o);
            x.p = __shfl_xor(best.p, o);
            if (tk_better(x, best)) best = x;
        }
        if (best.p < 0) break;
        if (lane == 0) {
            nbr[pi * topk + k] = best.p;
            nov[pi * topk + k] = best.ov;
        }
        last = best;
    }
    if (lane == 0) cnt[pi] = k;
}

hipError_t launch_topk(const int64_t *o_rp, const int32_t *o_col, const double *o_val, const int64_t *a_rp,
                       const int32_t *pos, int64_t n, int64_t num, int64_t den, int topk, int32_t *cnt, int32_t *nbr,
                       int64_t *nov, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 3) / 4;
    hipLaunchKernelGGL(k_topk, dim3((unsigned)blocks), dim3(256), 0, s, o_rp, o_col, o_val, a_rp, pos, n, num, den,
                       topk, cnt, nbr, nov);
    return hipGetLastError();
}

}  // namespace hcsp

