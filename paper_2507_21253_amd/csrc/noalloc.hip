// A whole product (symbolic phase, nnz read-back, numeric phase) that
// allocates nothing: its workspace is a file-scope device array of fixed
// size, for callers that cannot allocate device memory.  Each device the
// library runs on holds its own copy of the array until the process ends;
// every call on one device shares it (calls that overlap on one device race).
//
// In host code the array's name is only a host-side stand-in.  Its device
// address is looked up once per device (with that device current) and kept;
// kernels and copies get that address, never the name.
#include <cstring>
#include <mutex>
#include <string>

#include "internal.h"

namespace hcsp {

static_assert(HCSP_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size is a multiple of 256");

static __device__ __align__(256) unsigned char scratch[HCSP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// The device address of this device's copy of the scratch array (looked up
// on the first call on the device).
static int scratch_ptr(void **out)
{
    static std::mutex mu;
    static void *ptr[kMaxDevices] = {nullptr};
    int dev = -1;
    HCSP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(HCSP_E_UNSUPPORTED, "noalloc: device id out of range");
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        HCSP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(HCSP_E_HIP, "noalloc: no device address for the scratch array");
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return HCSP_OK;
}

}  // namespace hcsp

using namespace hcsp;

extern "C" int hcsp_spgemm_noalloc(const hcsp_operand *A, const hcsp_csr *B, const hcsp_opts *opts,
                                   int64_t *C_row_ptr_d, int32_t *C_col_d, double *C_val_d, int64_t capacity,
                                   int64_t *nnz_h, void *stream)
{
    clear_error();
    if (nnz_h) *nnz_h = -1;
    if (!C_row_ptr_d || capacity < 0 || (capacity > 0 && (!C_col_d || !C_val_d)))
        return fail(HCSP_E_INVALID, "noalloc: bad output arrays");
    hcsp_opts o;
    if (opts) o = *opts;
    else std::memset(&o, 0, sizeof o);
    // whole matrix, every launch on the caller's stream (no side streams to create)
    o.unit_lo = 0;
    o.unit_hi = 0;
    o.out_base = 0;
    o.flags = (o.flags | HCSP_F_ONE_STREAM) & ~HCSP_F_SYNC_CHECK;
    size_t need = 0;
    int rc = hcsp_spgemm_workspace(A, B, &o, &need);
    if (rc) return rc;
    if (need > (size_t)HCSP_NOALLOC_SCRATCH_BYTES)
        return fail(HCSP_E_CAPACITY, "noalloc: the product needs " + std::to_string(need) +
                                         " bytes of workspace, the static scratch holds " +
                                         std::to_string((size_t)HCSP_NOALLOC_SCRATCH_BYTES));
    void *ws = nullptr;
    rc = scratch_ptr(&ws);
    if (rc) return rc;
    hcsp_sym_info info;
    rc = hcsp_spgemm_symbolic(A, B, &o, C_row_ptr_d, &info, ws, HCSP_NOALLOC_SCRATCH_BYTES, stream);
    if (rc) return rc;
    if (nnz_h) *nnz_h = info.nnz;
    if (info.nnz > capacity)
        return fail(HCSP_E_CAPACITY, "noalloc: nnz(C) = " + std::to_string(info.nnz) + " exceeds the capacity " +
                                         std::to_string(capacity));
    o.flags |= HCSP_F_SYNC_CHECK;
    return hcsp_spgemm_numeric(A, B, &o, &info, C_row_ptr_d, C_col_d, C_val_d, capacity, ws,
                               HCSP_NOALLOC_SCRATCH_BYTES, stream);
}
