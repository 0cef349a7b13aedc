// Device construction of CSR_Cluster from CSR and a cluster plan (paper,
// "Access Pattern and Matrix Format": a cluster's non-zeros are stored
// together column by column, with placeholders where a member row has no
// entry).  One group of 16 lanes per cluster: lane l follows member row l
// with a cursor, and each step takes the smallest pending column across the
// members (a 16-way merge), which yields the sorted union; the ballot of the
// lanes holding that column is the column's row mask.
#include <climits>

#include "device.h"
#include "internal.h"

namespace hcsp {

__global__ void __launch_bounds__(256) k_cl_count(const int64_t *rp, const int32_t *col, const int32_t *perm,
                                                  const int64_t *cl_row_ptr, int64_t ncl, int64_t *col_cnt,
                                                  int64_t *val_cnt, int32_t *maxsize)
{
    const Group g = make_group(16);
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    if (c >= ncl) return;
    const int64_t b = cl_row_ptr[c];
    const int s = (int)(cl_row_ptr[c + 1] - b);
    if (s < 1 || s > 16) {
        if (g.gl == 0) {
            col_cnt[c] = 0;
            val_cnt[c] = 0;
            atomicMax(maxsize, 1 << 20);   // reported by the host as an invalid plan
        }
        return;
    }
    int64_t cur = 0, end = 0;
    if (g.gl < s) {
        const int r = perm[b + g.gl];
        cur = rp[r];
        end = rp[r + 1];
    }
    int64_t cnt = 0;
    for (;;) {
        const int head = cur < end ? col[cur] : INT_MAX;
        const int mn = gmin32(g, head);
        if (mn == INT_MAX) break;
        if (head == mn) ++cur;
        ++cnt;
    }
    if (g.gl == 0) {
        col_cnt[c] = cnt;
        val_cnt[c] = cnt * s;
        atomicMax(maxsize, s);
    }
}

__global__ void __launch_bounds__(256) k_cl_fill(const int64_t *rp, const int32_t *col, const double *val,
                                                 const int32_t *perm, const int64_t *cl_row_ptr, int64_t ncl,
                                                 const int64_t *cl_col_ptr, const int64_t *cl_val_ptr,
                                                 int32_t *cl_col, uint16_t *cl_mask, double *cl_val)
{
    const Group g = make_group(16);
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    if (c >= ncl) return;
    const int64_t b = cl_row_ptr[c];
    const int s = (int)(cl_row_ptr[c + 1] - b);
    if (s < 1 || s > 16) return;
    int64_t cur = 0, end = 0;
    if (g.gl < s) {
        const int r = perm[b + g.gl];
        cur = rp[r];
        end = rp[r + 1];
    }
    const int64_t o = cl_col_ptr[c], oe = cl_col_ptr[c + 1];
    const int64_t vo = cl_val_ptr[c];
    int64_t t = 0;
    for (;;) {
        const int head = cur < end ? col[cur] : INT_MAX;
        const int mn = gmin32(g, head);
        if (mn == INT_MAX || o + t >= oe) break;
        const bool has = head == mn;
        const uint64_t bal = gballot(g, has);
        if (g.gl == 0) {
            cl_col[o + t] = mn;
            cl_mask[o + t] = (uint16_t)bal;
        }
        if (g.gl < s) cl_val[vo + t * s + g.gl] = has ? val[cur] : 0.0;
        if (has) ++cur;
        ++t;
    }
}

hipError_t launch_cluster_count(const hcsp_csr &A, const int32_t *perm, const int64_t *cl_row_ptr, int64_t ncl,
                                int64_t *col_cnt, int64_t *val_cnt, int32_t *maxsize, hipStream_t s)
{
    if (ncl <= 0) return hipSuccess;
    const int64_t blocks = (ncl * 16 + 255) / 256;
    hipLaunchKernelGGL(k_cl_count, dim3((unsigned)blocks), dim3(256), 0, s, A.row_ptr, A.col, perm, cl_row_ptr,
                       ncl, col_cnt, val_cnt, maxsize);
    return hipGetLastError();
}

hipError_t launch_cluster_fill(const hcsp_csr &A, const hcsp_csr_cluster &out, hipStream_t s)
{
    if (out.nclusters <= 0) return hipSuccess;
    const int64_t blocks = (out.nclusters * 16 + 255) / 256;
    hipLaunchKernelGGL(k_cl_fill, dim3((unsigned)blocks), dim3(256), 0, s, A.row_ptr, A.col, A.val, out.perm,
                       out.cl_row_ptr, out.nclusters, out.cl_col_ptr, out.cl_val_ptr, out.cl_col, out.cl_mask,
                       out.cl_val);
    return hipGetLastError();
}

}  // namespace hcsp
