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

template <bool CL>
__device__ __forceinline__ int64_t member_row(const SpArgs &a, const UnitView &v, int l)
{
    return CL ? (int64_t)a.perm[v.pos0 + l] : v.pos0;
}

}  // namespace hcsp
