// Views of a work unit (a CSR row, or a CSR_Cluster cluster) shared by the
// shared-memory, column-window and dense global-memory kernels.
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

// Read by a whole wavefront for its (wave-uniform) unit u: every field is
// moved to scalar registers.
template <bool CL>
__device__ __forceinline__ UnitView unit_view(const SpArgs &a, int u)
{
    UnitView v;
    if (CL) {
        v.it0 = (int64_t)uniform64((uint64_t)a.cl_col_ptr[u]);
        v.it1 = (int64_t)uniform64((uint64_t)a.cl_col_ptr[u + 1]);
        v.pos0 = (int64_t)uniform64((uint64_t)a.cl_row_ptr[u]);
        v.s = uniform((int)(a.cl_row_ptr[u + 1] - v.pos0));
        v.vbase = (int64_t)uniform64((uint64_t)a.cl_val_ptr[u]);
    } else {
        v.it0 = (int64_t)uniform64((uint64_t)a.a_rp[u]);
        v.it1 = (int64_t)uniform64((uint64_t)a.a_rp[u + 1]);
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
// the unit's index inside that product.  Called by a whole wavefront with a
// wave-uniform g; the product's fields are moved to scalar registers.
__device__ __forceinline__ int batch_resolve(SpArgs &a, int64_t g)
{
    g = (int64_t)uniform64((uint64_t)g);
    const int p = uniform(batch_find(a.batch_units, a.nprob, g));
    const BatchProb &bp = a.batch[p];
    a.a_rp = uniform_ptr(bp.a_rp);
    a.a_col = uniform_ptr(bp.a_col);
    a.a_val = uniform_ptr(bp.a_val);
    a.cl_row_ptr = uniform_ptr(bp.cl_row_ptr);
    a.perm = uniform_ptr(bp.perm);
    a.cl_col_ptr = uniform_ptr(bp.cl_col_ptr);
    a.cl_col = uniform_ptr(bp.cl_col);
    a.cl_mask = uniform_ptr(bp.cl_mask);
    a.cl_val_ptr = uniform_ptr(bp.cl_val_ptr);
    a.cl_val = uniform_ptr(bp.cl_val);
    a.b_rp = uniform_ptr(bp.b_rp);
    a.b_col = uniform_ptr(bp.b_col);
    a.b_val = uniform_ptr(bp.b_val);
    const int64_t ub = (int64_t)uniform64((uint64_t)bp.unit_base);
    const int64_t sb = (int64_t)uniform64((uint64_t)bp.seg_base);
    const int64_t ob = (int64_t)uniform64((uint64_t)bp.out_base);
    a.keylo += ub;
    a.keyhi += ub;
    a.ucount += ub;
    a.c_rp += sb;
    if (a.c_col) a.c_col += ob;
    if (a.c_val) a.c_val += ob;
    a.cap = (int64_t)uniform64((uint64_t)bp.cap);
    a.err = a.errs + p;
    a.ncols = (int64_t)uniform64((uint64_t)bp.ncols);
    return (int)(g - ub);
}

template <bool CL>
__device__ __forceinline__ int64_t member_row(const SpArgs &a, const UnitView &v, int l)
{
    return CL ? (int64_t)a.perm[v.pos0 + l] : v.pos0;
}

}  // namespace hcsp
