// Symbolic and numeric SpGEMM kernels for gfx950.
//
// Work unit: one row of a CSR A, or one cluster of a CSR_Cluster A (paper,
// Alg. 1: for a cluster, every union column k is visited once, row k of B is
// read once, and each of its entries b_kj updates every member row l whose
// mask bit is set: c_lj += a_lk * b_kj).  A CSR row is a cluster of one row.
//
// A group of G lanes (G <= 64, inside one wavefront) owns one unit and a
// private slice of shared memory (LDS).  The unit's columns k are taken in
// ascending order; for each k the group's lanes take the entries of row k of
// B (distinct columns j), so within a step no two lanes touch the same
// accumulator slot and across steps the wavefront's LDS operations stay in
// program order.  Every output c_lj therefore receives its products in
// ascending k, each by one fused multiply-add starting from +0.0 — the same
// sequence the row-by-row Gustavson reference performs.
//
// Loads of B rows are batched R steps ahead of their use so each lane keeps
// several independent global loads in flight.
#include "device.h"
#include "internal.h"

namespace hcsp {

constexpr int kSymR = 8;   // B-entry loads in flight per lane, symbolic
constexpr int kNumR = 4;   // ... numeric (each carries a double)

struct UnitView {
    int64_t it0, it1;   // item (union column) range
    int64_t pos0;       // cluster: first position in perm; CSR: the row
    int64_t vbase;      // cluster: first value slot
    int s;              // member rows
};

template <bool CL>
__device__ __forceinline__ UnitView unit_view(const SpArgs &a, int u)
{
    UnitView v;
    if (CL) {
        v.it0 = a.cl_col_ptr[u];
        v.it1 = a.cl_col_ptr[u + 1];
        v.pos0 = a.cl_row_ptr[u];
        v.s = (int)(a.cl_row_ptr[u + 1] - v.pos0);
        v.vbase = a.cl_val_ptr[u];
    } else {
        v.it0 = a.a_rp[u];
        v.it1 = a.a_rp[u + 1];
        v.pos0 = u;
        v.s = 1;
        v.vbase = 0;
    }
    return v;
}

template <bool CL>
__device__ __forceinline__ int64_t member_row(const SpArgs &a, const UnitView &v, int l)
{
    return CL ? (int64_t)a.perm[v.pos0 + l] : v.pos0;
}

// ============================================================== symbolic
// Counts, per member row, the distinct output columns, and per unit the
// distinct columns of the union (used to size the numeric tables).  Keys go
// into a power-of-two open-addressing table with a multiplicative hash; the
// table has at least as many slots as the unit has products, so it never
// fills.  For clusters each key carries the OR of the masks of the k that
// reached it: row l's count is the number of keys with bit l set.
template <int S, bool CL>
__global__ void __launch_bounds__(256) k_sym(SpArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Group g = make_group(a.G);
    const int gidx = threadIdx.x / a.G;
    const int gpb = blockDim.x / a.G;
    const int64_t ui = xcd_block() * gpb + gidx;
    if (gidx >= gpb || ui >= a.count) return;
    const int u = a.order[a.bin_begin + ui];
    unsigned char *base = smem + (size_t)gidx * a.group_bytes;
    int *keys = (int *)base;
    uint32_t *masks = (uint32_t *)(keys + a.T);
    for (int i = g.gl; i < a.T; i += a.G) {
        keys[i] = kEmpty;
        if (CL) masks[i] = 0;
    }
    const UnitView v = unit_view<CL>(a, u);
    const uint32_t hmask = (uint32_t)a.T - 1u;
    const int hshift = 32 - a.log2T;
    int inserted = 0;

    for (int64_t r0 = v.it0; r0 < v.it1; r0 += a.G) {
        const int64_t q = r0 + g.gl;
        int64_t bs = 0;
        int bl = 0;
        uint32_t m = 1;
        if (q < v.it1) {
            const int k = CL ? a.cl_col[q] : a.a_col[q];
            if (CL) m = a.cl_mask[q];
            bs = a.b_rp[k];
            bl = (int)(a.b_rp[k + 1] - bs);
        }
        const int nit = (int)min((int64_t)a.G, v.it1 - r0);
        int t = 0, off = 0;
        while (t < nit) {
            int cj[kSymR];
            uint32_t cm[kSymR];
#pragma unroll
            for (int rr = 0; rr < kSymR; ++rr) {
                cj[rr] = -1;
                cm[rr] = 0;
                if (t < nit) {
                    const int len = gbcast(g, bl, t);
                    const int64_t st = gbcast(g, bs, t);
                    const uint32_t mm = gbcast(g, m, t);
                    const int idx = off + g.gl;
                    if (idx < len) {
                        cj[rr] = a.b_col[st + idx];
                        cm[rr] = mm;
                    }
                    off += a.G;
                    if (off >= len) {
                        ++t;
                        off = 0;
                    }
                }
            }
#pragma unroll
            for (int rr = 0; rr < kSymR; ++rr) {
                const int j = cj[rr];
                if (j < 0) continue;
                uint32_t h = ((uint32_t)j * 2654435761u) >> hshift;
                for (;;) {
                    const int cur = lds_load_relaxed(&keys[h]);
                    if (cur == j) break;
                    if (cur == kEmpty) {
                        const int old = atomicCAS(&keys[h], kEmpty, j);
                        if (old == kEmpty) {
                            ++inserted;
                            break;
                        }
                        if (old == j) break;
                    }
                    h = (h + 1u) & hmask;
                }
                if (CL) atomicOr(&masks[h], cm[rr]);
            }
        }
    }

    if (!CL) {
        const int64_t cnt = gsum64(g, inserted);
        if (g.gl == 0) {
            a.c_rp[u] = cnt;
            a.ucount[u] = (int32_t)cnt;
        }
    } else {
        int cnt[S];
#pragma unroll
        for (int l = 0; l < S; ++l) cnt[l] = 0;
        for (int i = g.gl; i < a.T; i += a.G) {
            if (keys[i] != kEmpty) {
                const uint32_t mm = masks[i];
#pragma unroll
                for (int l = 0; l < S; ++l) cnt[l] += (int)((mm >> l) & 1u);
            }
        }
        const int U = gsum32(g, inserted);
#pragma unroll
        for (int l = 0; l < S; ++l) cnt[l] = gsum32(g, cnt[l]);
        if (g.gl == 0) {
            a.ucount[u] = U;
#pragma unroll
            for (int l = 0; l < S; ++l)
                if (l < v.s) a.c_rp[member_row<CL>(a, v, l)] = cnt[l];
        }
    }
}

// ============================================================== numeric
// Keys go into a table of T slots plus a short tail, placed by an
// order-preserving hash h(j) = floor((j - lo) * T / (hi - lo + 1)) (lo/hi:
// the unit's smallest and largest possible output column) with linear
// probing.  Because h never decreases with j and probing only moves
// forward, the occupied slots form runs whose keys are all smaller than the
// keys of any later run; sorting the row only needs each key's rank inside
// its run.  If a probe ever wraps past the tail the order is lost and ranks
// are computed by full comparison instead.
template <int S, bool CL>
__global__ void __launch_bounds__(256) k_num(SpArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Group g = make_group(a.G);
    const int gidx = threadIdx.x / a.G;
    const int gpb = blockDim.x / a.G;
    const int64_t ui = xcd_block() * gpb + gidx;
    if (gidx >= gpb || ui >= a.count) return;
    const int u = a.order[a.bin_begin + ui];
    if (u < a.unit_lo || u >= a.unit_hi) return;

    const int T = a.T, TX = a.T + kTail;
    unsigned char *base = smem + (size_t)gidx * a.group_bytes;
    int *keys = (int *)base;
    uint32_t *masks = (uint32_t *)(keys + TX);
    size_t off_vals = (size_t)TX * 4 * (CL ? 2 : 1);
    off_vals = (off_vals + 7) & ~(size_t)7;
    double *vals = (double *)(base + off_vals);
    double *aval = vals + (size_t)TX * S;
    uint16_t *order = (uint16_t *)(aval + (size_t)a.G * S);

    const UnitView v = unit_view<CL>(a, u);
    for (int i = g.gl; i < TX; i += a.G) {
        keys[i] = kEmpty;
        if (CL) masks[i] = 0;
#pragma unroll
        for (int l = 0; l < S; ++l)
            if (l < v.s) vals[(size_t)l * TX + i] = 0.0;
    }
    const int lo = a.keylo[u], hi = a.keyhi[u];
    const float scale = (float)T / (float)((int64_t)hi - lo + 1);
    int wrapped = 0;

    for (int64_t r0 = v.it0; r0 < v.it1; r0 += a.G) {
        const int64_t q = r0 + g.gl;
        int64_t bs = 0;
        int bl = 0;
        uint32_t m = 1;
        if (q < v.it1) {
            const int k = CL ? a.cl_col[q] : a.a_col[q];
            if (CL) {
                m = a.cl_mask[q];
                const double *src = a.cl_val + v.vbase + (q - v.it0) * v.s;
#pragma unroll
                for (int l = 0; l < S; ++l)
                    if (l < v.s) aval[g.gl * S + l] = src[l];
            } else {
                aval[g.gl] = a.a_val[q];
            }
            bs = a.b_rp[k];
            bl = (int)(a.b_rp[k + 1] - bs);
        }
        const int nit = (int)min((int64_t)a.G, v.it1 - r0);
        int t = 0, off = 0;
        while (t < nit) {
            int cj[kNumR], ct[kNumR];
            double cb[kNumR];
#pragma unroll
            for (int rr = 0; rr < kNumR; ++rr) {
                cj[rr] = -1;
                ct[rr] = -1;
                cb[rr] = 0.0;
                if (t < nit) {
                    const int len = gbcast(g, bl, t);
                    const int64_t st = gbcast(g, bs, t);
                    const int idx = off + g.gl;
                    ct[rr] = t;
                    if (idx < len) {
                        cj[rr] = a.b_col[st + idx];
                        cb[rr] = a.b_val[st + idx];
                    }
                    off += a.G;
                    if (off >= len) {
                        ++t;
                        off = 0;
                    }
                }
            }
#pragma unroll
            for (int rr = 0; rr < kNumR; ++rr) {
                const int tt = ct[rr];
                if (tt < 0) continue;                         // uniform in the group
                const uint32_t mt = CL ? (uint32_t)gbcast(g, (int)m, tt) : 1u;
                const int j = cj[rr];
                if (j < 0) continue;
                int h = (int)((float)(j - lo) * scale);
                h = h < T ? h : T - 1;
                for (;;) {
                    const int cur = lds_load_relaxed(&keys[h]);
                    if (cur == j) break;
                    if (cur == kEmpty) {
                        const int old = atomicCAS(&keys[h], kEmpty, j);
                        if (old == kEmpty || old == j) break;
                    }
                    if (++h == TX) {
                        h = 0;
                        wrapped = 1;
                    }
                }
                if (CL) atomicOr(&masks[h], mt);
                const double b = cb[rr];
#pragma unroll
                for (int l = 0; l < S; ++l) {
                    if ((mt >> l) & 1u) {
                        double *p = &vals[(size_t)l * TX + h];
                        *p = __fma_rn(aval[tt * S + l], b, *p);
                    }
                }
            }
        }
    }

    // ---- rank every key: runs of occupied slots are ordered among themselves
    wrapped = gor32(g, wrapped);
    int U = 0;
    for (int c0 = 0; c0 < TX; c0 += a.G) {
        const int sidx = c0 + g.gl;
        const int key = sidx < TX ? keys[sidx] : kEmpty;
        const bool occ = key != kEmpty;
        const uint64_t bal = gballot(g, occ);
        if (occ) {
            int rank;
            if (!wrapped) {
                int rs = sidx;
                while (rs > 0 && keys[rs - 1] != kEmpty) --rs;
                int re = sidx + 1;
                while (re < TX && keys[re] != kEmpty) ++re;
                int rk = 0;
                for (int x = rs; x < re; ++x) rk += keys[x] < key;
                rank = U + gprefix(g, bal) - (sidx - rs) + rk;
            } else {
                rank = 0;
                for (int x = 0; x < TX; ++x) {
                    const int kx = keys[x];
                    rank += (kx != kEmpty) & (kx < key);
                }
            }
            order[rank] = (uint16_t)sidx;
        }
        U += __popcll(bal);
    }

    // ---- write each member row's entries in column order
    for (int l = 0; l < S && l < v.s; ++l) {
        const int64_t row = member_row<CL>(a, v, l);
        const int64_t o0 = a.c_rp[row] - a.out_base;
        const int64_t want = a.c_rp[row + 1] - a.c_rp[row];
        int64_t w = 0;
        for (int c0 = 0; c0 < U; c0 += a.G) {
            const int i = c0 + g.gl;
            const int sl = i < U ? (int)order[i] : -1;
            const bool pr = sl >= 0 && (!CL || ((masks[sl] >> l) & 1u));
            const uint64_t bal = gballot(g, pr);
            if (pr) {
                const int64_t dst = o0 + w + gprefix(g, bal);
                if (dst >= 0 && dst < a.cap && w + gprefix(g, bal) < want) {
                    a.c_col[dst] = keys[sl];
                    a.c_val[dst] = vals[(size_t)l * TX + sl];
                } else {
                    atomicOr(a.err, kErrCapacity);
                }
            }
            w += __popcll(bal);
        }
        if (g.gl == 0 && w != want) atomicOr(a.err, kErrCount);
    }
}

// ============================================================== dense path
// Units whose tables do not fit in shared memory.  One wavefront per unit,
// each with a private bitmap (and, for the numeric phase, a value array)
// covering every column of B in global memory.  Member rows are handled one
// after another, each exactly like a single CSR row.

// Symbolic: lanes take different columns k of the row (no order needed to
// count distinct columns), set bits with atomic OR and count the bits they
// were first to set; a second walk clears the bits it set.
template <bool CL>
__global__ void __launch_bounds__(256) k_sym_dense(SpArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t *bm = a.dense_bits + wv * a.dense_words;
    for (int64_t ti = wv; ti < a.count; ti += nw) {
        const int u = a.order[a.bin_begin + ti];
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
template <bool CL>
__global__ void __launch_bounds__(256) k_num_dense(SpArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t *bm = a.dense_bits + wv * a.dense_words;
    double *acc = a.dense_vals + wv * a.ncols;
    for (int64_t ti = wv; ti < a.count; ti += nw) {
        const int u = a.order[a.bin_begin + ti];
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

// ============================================================== launchers
template <int S, bool CL>
static hipError_t go_sym(const SpArgs &a, int blocks, int threads, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_sym<S, CL>), dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <int S, bool CL>
static hipError_t go_num(const SpArgs &a, int blocks, int threads, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_num<S, CL>), dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_sym(int sclass, bool cluster, const SpArgs &a, int blocks, int threads, size_t lds,
                      hipStream_t s)
{
    if (!cluster) return go_sym<1, false>(a, blocks, threads, lds, s);
    switch (sclass) {
    case 0: return go_sym<1, true>(a, blocks, threads, lds, s);
    case 1: return go_sym<2, true>(a, blocks, threads, lds, s);
    case 2: return go_sym<4, true>(a, blocks, threads, lds, s);
    case 3: return go_sym<8, true>(a, blocks, threads, lds, s);
    default: return go_sym<16, true>(a, blocks, threads, lds, s);
    }
}

hipError_t launch_num(int sclass, bool cluster, const SpArgs &a, int blocks, int threads, size_t lds,
                      hipStream_t s)
{
    if (!cluster) return go_num<1, false>(a, blocks, threads, lds, s);
    switch (sclass) {
    case 0: return go_num<1, true>(a, blocks, threads, lds, s);
    case 1: return go_num<2, true>(a, blocks, threads, lds, s);
    case 2: return go_num<4, true>(a, blocks, threads, lds, s);
    case 3: return go_num<8, true>(a, blocks, threads, lds, s);
    default: return go_num<16, true>(a, blocks, threads, lds, s);
    }
}

hipError_t launch_sym_dense(bool cluster, const SpArgs &a, int blocks, hipStream_t s)
{
    if (cluster) hipLaunchKernelGGL((k_sym_dense<true>), dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_sym_dense<false>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_num_dense(bool cluster, const SpArgs &a, int blocks, hipStream_t s)
{
    if (cluster) hipLaunchKernelGGL((k_num_dense<true>), dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_num_dense<false>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace hcsp
