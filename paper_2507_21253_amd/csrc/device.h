// Device-side helpers shared by the gfx950 kernels: lane groups inside a
// 64-wide wavefront, group-scoped ballot/prefix/broadcast/reductions, and the
// XCD-aware block renumbering.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hcsp {

constexpr int kWave = 64;
constexpr int kEmpty = -1;

// Values the whole wavefront agrees on, moved to scalar registers (the
// first active lane's copy).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Pointers to global memory (device buffers the caller passed in) that were
// read from memory: marked as global-address-space pointers, so loads through
// them are global loads instead of generic ones.
template <class T>
__device__ __forceinline__ T *global_ptr(T *p)
{
    typedef __attribute__((address_space(1))) T GT;
    return (T *)(GT *)(uintptr_t)p;
}

// The same for a wave-uniform pointer, moved to scalar registers.
template <class T>
__device__ __forceinline__ T *uniform_ptr(T *p)
{
    typedef __attribute__((address_space(1))) T GT;
    return (T *)(GT *)(uintptr_t)uniform64((uint64_t)(uintptr_t)p);
}

// A group of G consecutive lanes (G a power of two, 1 <= G <= 64) of one
// wavefront that works on one row or cluster.  Groups never span waves, so
// every group-level exchange is wave-local and needs no barrier.
struct Group {
    int G;          // lanes in the group
    int gl;         // this lane's index inside the group
    int base;       // wave lane of the group's first lane
    uint64_t mask;  // the group's lanes as a wave lane mask
};

__device__ __forceinline__ Group make_group(int G)
{
    Group g;
    const int lane = (int)__lane_id();
    g.G = G;
    g.gl = lane & (G - 1);
    g.base = lane - g.gl;
    g.mask = (G == kWave) ? ~0ull : (((1ull << G) - 1ull) << g.base);
    return g;
}

// Ballot of the group's lanes, bit t = group lane t.
__device__ __forceinline__ uint64_t gballot(const Group &g, bool p)
{
    return (__ballot(p) & g.mask) >> g.base;
}

// Number of set bits of a group ballot below this lane.
__device__ __forceinline__ int gprefix(const Group &g, uint64_t b)
{
    return __popcll(b & ((1ull << g.gl) - 1ull));
}

template <class T>
__device__ __forceinline__ T gbcast(const Group &g, T v, int t)
{
    return __shfl(v, g.base + t);
}

__device__ __forceinline__ int64_t gsum64(const Group &g, int64_t v)
{
    for (int o = g.G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int gsum32(const Group &g, int v)
{
    for (int o = g.G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int gmin32(const Group &g, int v)
{
    for (int o = g.G >> 1; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int gmax32(const Group &g, int v)
{
    for (int o = g.G >> 1; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int gor32(const Group &g, int v)
{
    for (int o = g.G >> 1; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on
// XCD b % 8), and each XCD has its own L2.  Renumber blocks so that every
// XCD receives one contiguous range of logical blocks: neighbouring rows or
// clusters, which share rows of B, then share an L2.
__device__ __forceinline__ int64_t xcd_block()
{
    const int64_t nb = gridDim.x, b = blockIdx.x;
    if (nb < 16) return b;
    const int64_t q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

template <class T>
__device__ __forceinline__ T lds_load_relaxed(T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

}  // namespace hcsp
