// Views of a work unit (a CSR row, or a CSR_Cluster cluster) shared by the
// shared-memory and the dense global-memory kernels.
#pragma once
#include "device.h"
#include "internal.h"

namespace hcsp {

struct UnitView {
    int64_t it0, it1;   // item range: the row's columns, or the cluster's union columns
    int64_t pos0;       // cluster: first position in perm; CSR: the row itself
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

// Product of a batch holding batch-wide unit g: the largest p with
// bases[p] <= g (products without units share their successor's base).
__device__ __forceinline__ int batch_find(const int64_t *bases, int nprob, int64_t g)
{
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bases[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Points the arguments at the product holding batch-wide unit g and returns
// the unit's index inside that product.
__device__ __forceinline__ int batch_resolve(SpArgs &a, int64_t g)
{
    const int p = batch_find(a.batch_units, a.nprob, g);
    const BatchProb &bp = a.batch[p];
    a.a_rp = bp.a_rp;
    a.a_col = bp.a_col;
    a.a_val = bp.a_val;
    a.cl_row_ptr = bp.cl_row_ptr;
    a.perm = bp.perm;
    a.cl_col_ptr = bp.cl_col_ptr;
    a.cl_col = bp.cl_col;
    a.cl_mask = bp.cl_mask;
    a.cl_val_ptr = bp.cl_val_ptr;
    a.cl_val = bp.cl_val;
    a.b_rp = bp.b_rp;
    a.b_col = bp.b_col;
    a.b_val = bp.b_val;
    a.keylo += bp.unit_base;
    a.keyhi += bp.unit_base;
    a.ucount += bp.unit_base;
    a.c_rp += bp.seg_base;
    if (a.c_col) a.c_col += bp.out_base;
    if (a.c_val) a.c_val += bp.out_base;
    a.cap = bp.cap;
    a.err = a.errs + p;
    a.ncols = bp.ncols;
    return (int)(g - bp.unit_base);
}

template <bool CL>
__device__ __forceinline__ int64_t member_row(const SpArgs &a, const UnitView &v, int l)
{
    return CL ? (int64_t)a.perm[v.pos0 + l] : v.pos0;
}

}  // namespace hcsp
