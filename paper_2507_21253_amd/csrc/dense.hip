// Dense global-memory path for units whose tables do not fit in shared
// memory.  One wavefront per unit, each with a private bitmap (and, for the
// numeric phase, a value array) covering every column of B in global memory.
// Member rows are handled one after another, each like a single CSR row.
#include "unit.h"

namespace hcsp {

// The dense bin's units as (count, first) for this launch; in a batch they
// are read from device memory and each unit is resolved to its product.
template <bool BATCH>
__device__ __forceinline__ void dense_range(const SpArgs &a, int64_t *count, int64_t *begin)
{
    *count = BATCH ? a.dcount[a.bin] : a.count;
    *begin = BATCH ? a.dbegin[a.bin] : a.bin_begin;
}

template <bool BATCH>
__device__ __forceinline__ int dense_unit(SpArgs &a, const SpArgs &a0, int64_t i)
{
    a = a0;
    return BATCH ? batch_resolve(a, a0.order[i]) : a0.order[i];
}

// ============================================================== dense path
// Units whose tables do not fit in shared memory.  One wavefront per unit,
// each with a private bitmap (and, for the numeric phase, a value array)
// covering every column of B in global memory.  Member rows are handled one
// after another, each exactly like a single CSR row.

// Symbolic: lanes take different columns k of the row (no order needed to
// count distinct columns), set bits with atomic OR and count the bits they
// were first to set; a second walk clears the bits it set.
template <bool CL, bool BATCH>
__global__ void __launch_bounds__(256) k_sym_dense(SpArgs a0)
{
    const int lane = threadIdx.x & 63;
    const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t *bm = a0.dense_bits + wv * a0.dense_words;
    int64_t count, begin;
    dense_range<BATCH>(a0, &count, &begin);
    for (int64_t ti = wv; ti < count; ti += nw) {
        SpArgs a;
        const int u = dense_unit<BATCH>(a, a0, begin + ti);
        const UnitView v = unit_view<CL>(a, u);
        for (int l = 0; l < v.s; ++l) {
            int64_t cnt = 0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int64_t q = v.it0 + lane; q < v.it1; q += 64) {
                    if (CL && !((a.cl_mask[q] >> l) & 1u)) continue;
                    const int k = CL ? a.cl_col[q] : a.a_col[q];
                    const int64_t e = a.b_rp[k + 1];
                    for (int64_t p = a.b_rp[k]; p < e; ++p) {
                        const int j = a.b_col[p];
                        if (pass == 0) {
                            const uint32_t bit = 1u << (j & 31);
                            const uint32_t old = atomicOr(&bm[j >> 5], bit);
                            cnt += (old & bit) ? 0 : 1;
                        } else {
                            bm[j >> 5] = 0u;
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            }
            for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
            if (lane == 0) a.c_rp[member_row<CL>(a, v, l)] = cnt;
        }
        if (lane == 0) a.ucount[u] = INT32_MAX;
    }
}

// Numeric: the row's columns k are taken in ascending order and the lanes
// split row k of B, so each c_j still sees its products in ascending k; the
// accumulator lives in global memory, so every step waits for its stores
// before the next step reads.  Output: scan the bitmap in column order.
template <bool CL, bool BATCH>
__global__ void __launch_bounds__(256) k_num_dense(SpArgs a0)
{
    const int lane = threadIdx.x & 63;
    const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t *bm = a0.dense_bits + wv * a0.dense_words;
    double *acc = a0.dense_vals + wv * a0.ncols;  // stride: the widest B of the launch
    int64_t count, begin;
    dense_range<BATCH>(a0, &count, &begin);
    for (int64_t ti = wv; ti < count; ti += nw) {
        SpArgs a;
        const int u = dense_unit<BATCH>(a, a0, begin + ti);
        if (u < a.unit_lo || u >= a.unit_hi) continue;
        const UnitView v = unit_view<CL>(a, u);
        for (int l = 0; l < v.s; ++l) {
            for (int64_t q = v.it0; q < v.it1; ++q) {
                if (CL && !((a.cl_mask[q] >> l) & 1u)) continue;
                const int k = CL ? a.cl_col[q] : a.a_col[q];
                const double av = CL ? a.cl_val[v.vbase + (q - v.it0) * v.s + l] : a.a_val[q];
                const int64_t e = a.b_rp[k + 1];
                for (int64_t p = a.b_rp[k] + lane; p < e; p += 64) {
                    const int j = a.b_col[p];
                    const uint32_t bit = 1u << (j & 31);
                    const uint32_t old = atomicOr(&bm[j >> 5], bit);
                    const double prev = (old & bit) ? __hip_atomic_load(&acc[j], __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_WORKGROUP)
                                                    : 0.0;
                    __hip_atomic_store(&acc[j], __fma_rn(av, a.b_val[p], prev), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            }
            const int64_t row = member_row<CL>(a, v, l);
            const int64_t o0 = a.c_rp[row] - a.out_base;
            const int64_t want = a.c_rp[row + 1] - a.c_rp[row];
            int64_t w = 0;
            for (int64_t w0 = 0; w0 < a.dense_words; w0 += 64) {
                const int64_t wi = w0 + lane;
                uint32_t word = wi < a.dense_words ? bm[wi] : 0u;
                int c = __popc(word);
                int pre = c;
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(pre, o);
                    if (lane >= o) pre += y;
                }
                const int tot = __shfl(pre, 63);
                int64_t dst = o0 + w + pre - c;
                while (word) {
                    const int b = __ffs(word) - 1;
                    word &= word - 1u;
                    const int j = (int)(wi * 32 + b);
                    if (dst >= 0 && dst < a.cap && dst - o0 < want) {
                        a.c_col[dst] = j;
                        a.c_val[dst] = acc[j];
                    } else {
                        atomicOr(a.err, kErrCapacity);
                    }
                    ++dst;
                }
                if (wi < a.dense_words) bm[wi] = 0u;
                w += tot;
            }
            if (lane == 0 && w != want) atomicOr(a.err, kErrCount);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        }
    }
}

hipError_t launch_sym_dense(bool cluster, bool batch, const SpArgs &a, int blocks, hipStream_t s)
{
    if (cluster && batch) hipLaunchKernelGGL((k_sym_dense<true, true>), dim3(blocks), dim3(256), 0, s, a);
    else if (cluster) hipLaunchKernelGGL((k_sym_dense<true, false>), dim3(blocks), dim3(256), 0, s, a);
    else if (batch) hipLaunchKernelGGL((k_sym_dense<false, true>), dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_sym_dense<false, false>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_num_dense(bool cluster, bool batch, const SpArgs &a, int blocks, hipStream_t s)
{
    if (cluster && batch) hipLaunchKernelGGL((k_num_dense<true, true>), dim3(blocks), dim3(256), 0, s, a);
    else if (cluster) hipLaunchKernelGGL((k_num_dense<true, false>), dim3(blocks), dim3(256), 0, s, a);
    else if (batch) hipLaunchKernelGGL((k_num_dense<false, true>), dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_num_dense<false, false>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace hcsp
