// CSR transpose on the device, for the overlap matrix A A^T of the
// hierarchical plan's candidate search (Alg. 3 forms the transpose of A
// before SpGEMM_TopK).  A counting sort of A's entries by column: column
// counts, an exclusive scan into A^T's row offsets, a scatter through atomic
// cursors (which leaves each row of A^T with the right entries in no
// particular order), then every row of A^T is sorted by one of three
// kernels chosen by its length, and finally the values are gathered (entry
// (j, i) of A^T takes a_ij, found by binary search in row i of A).  Nothing
// synchronizes with the host: the lists of rows for the two larger sorts
// are built on the device and walked by persistent grids.
#include <algorithm>
#include <climits>

#include "device.h"
#include "internal.h"

namespace hcsp {

constexpr int kTrShort = 256;     // rows up to this length: one wavefront, rank sort in shared memory
constexpr int kTrMid = 8192;      // up to this: one 1024-thread block, bitonic sort in shared memory
constexpr int kTrLongBlocks = 64; // longer rows: a bitmap over A's rows per block, this many blocks
constexpr int kTrMidBlocks = 1024;


static size_t tr_align(size_t x) { return (x + 255) / 256 * 256; }

size_t layout_transpose(int64_t nrows, int64_t ncols, char *base, TrWs *w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        off = tr_align(off);
        void *p = base ? (void *)(base + off) : nullptr;
        off += bytes;
        return p;
    };
    const size_t nc = (size_t)std::max<int64_t>(ncols, 1);
    w->cursor = (int64_t *)take(8 * nc);
    w->mid = (int32_t *)take(4 * nc);
    w->lng = (int32_t *)take(4 * nc);
    w->counts = (uint32_t *)take(256);
    w->words = (std::max<int64_t>(nrows, 1) + 31) / 32;
    w->bits = (uint32_t *)take(4 * (size_t)w->words * kTrLongBlocks);
    w->scan_tmp = (int64_t *)take(8 * scan_tmp_elems(ncols + 1));
    return tr_align(off);
}

// column counts into rp[c] (rp zeroed; rp[ncols] stays 0 for the exclusive scan)
__global__ void __launch_bounds__(256) k_tr_count(const int32_t *col, int64_t nnz, int64_t *rp)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd((unsigned long long *)&rp[col[p]], 1ull);
}

__global__ void __launch_bounds__(256) k_tr_copy(const int64_t *src, int64_t n, int64_t *dst)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// one wavefront per row i of A: its entries go to the next free slots of their columns' rows of A^T
__global__ void __launch_bounds__(256) k_tr_scatter(const int64_t *rp, const int32_t *col, int64_t nrows,
                                                    int64_t *cursor, int32_t *tcol)
{
    const int lane = (int)__lane_id();
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= nrows) return;
    for (int64_t p = rp[i] + lane; p < rp[i + 1]; p += kWave) {
        const int64_t slot = (int64_t)atomicAdd((unsigned long long *)&cursor[col[p]], 1ull);
        tcol[slot] = (int32_t)i;
    }
}

// One wavefront per row j of A^T.  Rows of at most kTrShort entries are
// sorted here: the entries (distinct row ids of A) go to shared memory and
// each is written at its rank, the number of smaller entries.  Longer rows
// are listed for the other two sorts.
__global__ void __launch_bounds__(256) k_tr_sort_short(const int64_t *trp, int64_t nrows_t, int32_t *tcol,
                                                       int32_t *mid, int32_t *lng, uint32_t *counts)
{
    __shared__ int32_t buf[4][kTrShort];
    const int lane = (int)__lane_id(), w = threadIdx.x >> 6;
    const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (j >= nrows_t) return;
    const int64_t b = trp[j];
    const int64_t L = trp[j + 1] - b;
    if (L <= 1) return;
    if (L > kTrShort) {
        if (lane == 0) {
            if (L <= kTrMid) mid[atomicAdd(&counts[0], 1u)] = (int32_t)j;
            else lng[atomicAdd(&counts[1], 1u)] = (int32_t)j;
        }
        return;
    }
    const int n = (int)L;
    int32_t mine[kTrShort / kWave];
#pragma unroll
    for (int t = 0; t < kTrShort / kWave; ++t) {
        const int e = lane + t * kWave;
        mine[t] = e < n ? tcol[b + e] : INT_MAX;
        if (e < n) buf[w][e] = mine[t];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    int rank[kTrShort / kWave] = {0, 0, 0, 0};
    for (int e = 0; e < n; ++e) {
        const int32_t y = buf[w][e];
#pragma unroll
        for (int t = 0; t < kTrShort / kWave; ++t) rank[t] += y < mine[t];
    }
#pragma unroll
    for (int t = 0; t < kTrShort / kWave; ++t)
        if (lane + t * kWave < n) tcol[b + rank[t]] = mine[t];
}

// One 1024-thread block per listed row of kTrShort < L <= kTrMid entries:
// bitonic sort of the row padded to a power of two in shared memory.
__global__ void __launch_bounds__(1024) k_tr_sort_mid(const int64_t *trp, int32_t *tcol, const int32_t *mid,
                                                      const uint32_t *counts)
{
    __shared__ int32_t buf[kTrMid];
    const uint32_t nmid = counts[0];
    for (uint32_t r = blockIdx.x; r < nmid; r += gridDim.x) {
        const int64_t j = mid[r];
        const int64_t b = trp[j];
        const int n = (int)(trp[j + 1] - b);
        int P = 1;
        while (P < n) P <<= 1;
        for (int e = threadIdx.x; e < P; e += blockDim.x) buf[e] = e < n ? tcol[b + e] : INT_MAX;
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int d = k >> 1; d > 0; d >>= 1) {
                for (int e = threadIdx.x; e < P; e += blockDim.x) {
                    const int f = e ^ d;
                    if (f > e) {
                        const int32_t x = buf[e], y = buf[f];
                        const bool up = (e & k) == 0;
                        if ((x > y) == up) {
                            buf[e] = y;
                            buf[f] = x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int e = threadIdx.x; e < n; e += blockDim.x) tcol[b + e] = buf[e];
        __syncthreads();
    }
}

// Rows longer than kTrMid: the block marks the row's entries in its own
// bitmap over A's rows (cleared before the launch), then writes the set bits
// in ascending order (a block-wide prefix count over the bitmap words),
// clearing the words as it goes so the bitmap is empty for the next row.
// The bitmap is read and cleared with agent-scope atomics, and a device
// fence before each barrier makes the other waves' ORs and clears visible.
__global__ void __launch_bounds__(1024) k_tr_sort_long(const int64_t *trp, int32_t *tcol, const int32_t *lng,
                                                       const uint32_t *counts, uint32_t *bits_all, int64_t words)
{
    __shared__ int32_t wsum[1024 / kWave];
    __shared__ int64_t carry_s;
    uint32_t *bits = bits_all + (int64_t)blockIdx.x * words;
    const uint32_t nlong = counts[1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (uint32_t r = blockIdx.x; r < nlong; r += gridDim.x) {
        const int64_t j = lng[r];
        const int64_t b = trp[j], e1 = trp[j + 1];
        for (int64_t e = b + threadIdx.x; e < e1; e += blockDim.x) {
            const int32_t v = tcol[e];
            atomicOr(&bits[v >> 5], 1u << (v & 31));
        }
        if (threadIdx.x == 0) carry_s = b;
        __threadfence();  // every OR has reached memory before any wave reads the bitmap
        __syncthreads();
        for (int64_t w0 = 0; w0 < words; w0 += blockDim.x) {
            const int64_t wi = w0 + threadIdx.x;
            uint32_t x = 0;
            if (wi < words) {
                x = __hip_atomic_load(&bits[wi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (x) __hip_atomic_store(&bits[wi], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            const int c = __popc(x);
            int inc = c;
            for (int o = 1; o < kWave; o <<= 1) {
                const int y = __shfl_up(inc, o);
                if (lane >= o) inc += y;
            }
            if (lane == kWave - 1) wsum[wv] = inc;
            __syncthreads();
            int wb = 0, tot = 0;
            for (int q = 0; q < nw; ++q) {
                if (q < wv) wb += wsum[q];
                tot += wsum[q];
            }
            int64_t pos = carry_s + wb + inc - c;
            while (x) {
                const int t = __ffs(x) - 1;
                x &= x - 1;
                tcol[pos++] = (int32_t)(wi * 32 + t);
            }
            __threadfence();  // the words cleared here are zero before the next row's ORs
            __syncthreads();
            if (threadIdx.x == 0) carry_s += tot;
            __syncthreads();
        }
    }
}

// one wavefront per row j of A^T: entry (j, i) takes a_ij, found by binary search in row i of A
__global__ void __launch_bounds__(256) k_tr_values(const int64_t *rp, const int32_t *col, const double *val,
                                                   const int64_t *trp, const int32_t *tcol, int64_t nrows_t,
                                                   double *tval)
{
    const int lane = (int)__lane_id();
    const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (j >= nrows_t) return;
    for (int64_t e = trp[j] + lane; e < trp[j + 1]; e += kWave) {
        const int32_t i = tcol[e];
        int64_t lo = rp[i], hi = rp[i + 1];
        while (hi - lo > 1) {
            const int64_t m = (lo + hi) >> 1;
            if (col[m] <= j) lo = m;
            else hi = m;
        }
        tval[e] = val[lo];
    }
}

// blocks of 256 threads for `threads` threads (one wavefront per row: 64 per row)
static unsigned grid_for(int64_t threads)
{
    return (unsigned)std::max<int64_t>(1, (threads + 255) / 256);
}

hipError_t launch_transpose(const hcsp_csr &A, const hcsp_csr &At, const TrWs &w, hipStream_t s)
{
    hipError_t e;
    if ((e = launch_fill_i64(At.row_ptr, A.ncols + 1, 0, s)) != hipSuccess) return e;
    if ((e = launch_fill_u32(w.counts, 2, 0u, s)) != hipSuccess) return e;
    if ((e = launch_fill_u32(w.bits, w.words * kTrLongBlocks, 0u, s)) != hipSuccess) return e;
    if (A.nnz > 0) {
        const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(16384, (A.nnz + 255) / 256));
        hipLaunchKernelGGL(k_tr_count, dim3(g), dim3(256), 0, s, A.col, A.nnz, At.row_ptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = launch_scan_exclusive(At.row_ptr, A.ncols + 1, w.scan_tmp, s)) != hipSuccess) return e;
    if (A.nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tr_copy, dim3(grid_for(A.ncols)), dim3(256), 0, s, At.row_ptr, A.ncols, w.cursor);
    hipLaunchKernelGGL(k_tr_scatter, dim3(grid_for(A.nrows * 64)), dim3(256), 0, s, A.row_ptr, A.col, A.nrows,
                       w.cursor, At.col);
    hipLaunchKernelGGL(k_tr_sort_short, dim3(grid_for(A.ncols * 64)), dim3(256), 0, s, At.row_ptr, A.ncols, At.col,
                       w.mid, w.lng, w.counts);
    hipLaunchKernelGGL(k_tr_sort_mid, dim3(kTrMidBlocks), dim3(1024), 0, s, At.row_ptr, At.col, w.mid, w.counts);
    hipLaunchKernelGGL(k_tr_sort_long, dim3(kTrLongBlocks), dim3(1024), 0, s, At.row_ptr, At.col, w.lng, w.counts,
                       w.bits, w.words);
    if (At.val) {
        hipLaunchKernelGGL(k_tr_values, dim3(grid_for(A.ncols * 64)), dim3(256), 0, s, A.row_ptr, A.col, A.val,
                           At.row_ptr, At.col, A.ncols, At.val);
    }
    return hipGetLastError();
}

}  // namespace hcsp
