// Symbolic and numeric SpGEMM kernels for gfx950, shared-memory path.
//
// Work unit: one row of a CSR A, or one cluster of a CSR_Cluster A (paper,
// Alg. 1: for a cluster, every union column k is visited once, row k of B is
// read once, and each entry b_kj updates every member row l whose mask bit
// is set: c_lj += a_lk * b_kj).  A CSR row is a cluster of one row.
//
// One wavefront owns one unit and a private slice of shared memory (LDS).
// The unit's products are taken as one flattened list in ascending k (item
// = one column k of the unit, contributing the entries of row k of B), and
// the wavefront walks it 64 entries per pass, so short rows of B still fill
// every lane.  Within a pass all lanes probe the hash table at once; the
// fused multiply-adds are then applied item by item (a scalar loop over the
// few items a pass touches), so an output c_lj receives its products in
// ascending k, each by one fma starting from +0.0 — the same sequence the
// row-by-row Gustavson reference performs.  Entries of one row of B have
// distinct columns, so lanes of one sub-step never share a slot, and the
// wavefront's LDS operations stay in program order across sub-steps.  When
// every item of a round has at most 32 products and they average at least 24
// (stencil-like rows), the numeric phase walks the round two items per pass
// instead, one per half of the wavefront, and applies the two halves in two
// fixed sub-steps.
//
// The kernels are bound by instruction issue, so the pass loop is written
// to keep the common path branch-free: a probe is one LDS compare-and-swap
// (taking the slot if empty, confirming it if it already holds the key);
// lanes past the end of the list work on a reserved dummy slot instead of
// being masked off; B is addressed by 32-bit offsets from a scalar base; and
// the loads of several passes are issued before any of them is consumed.
#include <climits>
#include <type_traits>

#include "unit.h"

namespace hcsp {

// passes whose B loads are in flight together (fewer for clusters, whose
// per-member updates need more registers)
template <int S>
struct Depth {
    static constexpr int R = S >= 8 ? 2 : (S >= 4 ? 4 : (S == 2 ? 5 : 6));
};
constexpr int kRoundW = 4096;               // products per round
constexpr int kRoundPasses = kRoundW / 64;  // == 64: one start-bit word per lane
constexpr int kDummyKey = INT_MAX;          // key of the reserved slot used by idle lanes

// Narrow clusters keep each item's member values of A in the registers of the
// lane that loaded the item (read back by lane broadcast); wider ones stage
// them in shared memory.
__host__ __device__ constexpr bool a_in_regs(int S) { return S <= 4; }

// 16-byte item record: one column k of the unit inside the current round.
struct __align__(16) ItemRec {
    uint32_t bs;  // offset in B of the item's first product in this round
    int32_t P;    // first position of the item in the round's flattened list
    uint32_t x;   // CSR: low word of a_ik.  Cluster: member-row mask of the column
    uint32_t y;   // CSR: high word of a_ik. Cluster: lane holding the item's A values
};
static_assert(sizeof(ItemRec) == 16, "ItemRec layout");

__device__ __forceinline__ uint64_t lanemask_lt(int L) { return (1ull << L) - 1ull; }
__device__ __forceinline__ uint64_t lanemask_le(int L) { return L == 63 ? ~0ull : ((2ull << L) - 1ull); }

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = (int)__lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(v, o);
        if (lane >= o) v += y;
    }
    return v;
}

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l)
{
    const int lo = __builtin_amdgcn_readlane((int)v, l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    return ((int64_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// B entry at a 32-bit element offset from the array base (scalar base +
// vector offset addressing).
__device__ __forceinline__ int ld_col(const int32_t *base, uint32_t off)
{
    return *(const int32_t *)((const char *)base + (uint64_t)(off << 2));
}
__device__ __forceinline__ double ld_val(const double *base, uint32_t off)
{
    return *(const double *)((const char *)base + (uint64_t)(off << 3));
}

// ---------------------------------------------------------------- LDS layout
// Slot counts include one reserved dummy slot at the end.  A cluster's
// member-presence masks take one byte per slot (up to 8 rows) or two (16).
template <int S>
using MaskT = typename std::conditional<(S <= 8), uint8_t, uint16_t>::type;

// Atomic OR of m into the mask of slot h, through the aligned 32-bit word
// that holds it, returning nothing (nothing to wait for).  The word is found
// by pointer arithmetic from the (4-byte aligned) mask array, never through
// an integer, so the compiler keeps the access in shared memory.
template <int S>
__device__ __forceinline__ void mask_set(MaskT<S> *masks, uint32_t h, uint32_t m)
{
    const uint32_t byte = h * (uint32_t)sizeof(MaskT<S>);
    atomicOr(reinterpret_cast<uint32_t *>(masks) + (byte >> 2), m << (8 * (byte & 3u)));
}

// Fills n bytes (rounded up to 16; the region is padded to 16) at a
// 16-byte aligned shared-memory address with a 4-byte pattern, 16 bytes per
// lane and store.
__device__ __forceinline__ void lds_fill(void *p, int n, uint32_t w)
{
    uint4 *q = reinterpret_cast<uint4 *>(p);
    const uint4 v = make_uint4(w, w, w, w);
    for (int i = (int)__lane_id(); 16 * i < n; i += 64) q[i] = v;
}

// sizes of the cluster mask region (rounded to whole 32-bit words)
__host__ __device__ constexpr int mask_region(int mb, int slots) { return (mb * slots + 3) & ~3; }

// Regions start on 16-byte boundaries so that they are cleared with 16-byte
// stores.
__host__ __device__ constexpr int align16(int x) { return (x + 15) & ~15; }

struct SymLayout {
    int keys, masks, items, sbits, bytes;
    __host__ __device__ SymLayout(int mb, int T)  // mb: mask bytes per slot, 0 for one-row units
    {
        keys = 0;
        masks = align16(keys + 4 * (T + 1));
        items = align16(masks + mb * (T + 1));
        sbits = items + 16 * 64;
        bytes = (sbits + 8 * kRoundPasses + 15) & ~15;
    }
};

// The arrays of the final sweep (an occupancy bitmap of the slots with a
// prefix count per 64-slot word, the per-home key counts of the general
// ranking and, for a cluster, the rank-ordered slot list, 2 bytes per entry)
// reuse the item and start-bit area, which is free once the passes are done,
// when they fit there.
// A cluster of several rows keeps its member values (and masks) compactly:
// one entry per distinct key, numbered in insertion order (at most vcap keys,
// plus a dummy entry), found through a 16-bit index per slot.  A CSR row
// keeps its value in the key's slot.
// Large numeric tables (at least kHashedMinT slots) place keys by a
// multiplicative hash instead of the order-preserving one: the output
// columns of long rows can crowd into a small part of their range (rows of
// power-law graphs meet the low-numbered hubs), which would make the
// order-preserving placement's probe runs hundreds of slots long.  Their keys
// are ranked by a counting sort over T/2 buckets of equal column range, then
// by comparison within a bucket (a bucket never holds more keys than its
// width in columns); the sort needs bucket ends and a key array.
constexpr int kHashedMinT = 1024;
__host__ __device__ constexpr bool hashed_table(int T) { return T >= kHashedMinT; }

struct NumLayout {
    int keys, vidx, masks, vals, aval, order, items, sbits, hcnt, obits, opre, bend, arr, bytes;
    __host__ __device__ NumLayout(bool cl, int S, int T, int vcap)
    {
        const int TX = T + num_tail(T);
        cl = cl && S > 1;
        const int mb = cl ? (S <= 8 ? 1 : 2) : 0;
        const int nv = cl ? vcap + 1 : TX + 1;  // value entries incl. the dummy
        keys = 0;
        vidx = align16(keys + 4 * (TX + 1));
        masks = align16(vidx + (cl ? 2 * (TX + 1) : 0));
        vals = align16(masks + mb * nv);
        aval = vals + 8 * S * nv;
        const int end = aval + (cl && !a_in_regs(S) ? 8 * S * 64 : 0);
        items = (end + 15) & ~15;
        sbits = items + 16 * 64;
        const int top = sbits + 8 * kRoundPasses;
        const int nw = (TX + 63) >> 6;
        const int ord_b = cl ? (2 * TX + 3) & ~3 : 0;
        if (hashed_table(T)) {
            const int need = 4 * (T / 2 + 1) + 4 * TX + ord_b;
            const int at = need <= top - items ? items : top;
            bend = at;
            arr = bend + 4 * (T / 2 + 1);
            order = arr + 4 * TX;
            obits = opre = hcnt = at;  // unused
            bytes = (at == items ? top : at + need + 15) & ~15;
            return;
        }
        const int hc_b = 2 * (T + 1);  // 16-bit counts, read through aligned 32-bit words
        const int need = 12 * nw + ord_b + hc_b;
        const int at = need <= top - items ? items : top;
        obits = at;
        opre = at + 8 * nw;
        order = opre + 4 * nw;
        hcnt = order + ord_b;
        bend = arr = at;  // unused
        bytes = (at == items ? top : at + need + 15) & ~15;
    }
};

int64_t sym_wave_bytes(int mask_bytes, int T) { return SymLayout(mask_bytes, T).bytes; }
int64_t num_wave_bytes(bool cl, int sclass, int T, int load_pct)
{
    return NumLayout(cl, 1 << sclass, T, num_vcap(T, load_pct)).bytes;
}

// ---------------------------------------------------------------- rounds
// Lays out one round from the items the lanes hold (lane i: column q0+i of
// the unit, its first product bs in B, its product count bl and its record
// words rx, ry): the non-empty ones are compacted, their products laid out
// back to back (positions P), and a start bit set at each P.  An item longer
// than what fits is cut and resumed in the next round (q0, off0 advance;
// off0 products of the item at q0 were taken by earlier rounds).  Returns the
// number of products in the round.
__device__ __forceinline__ int flatten_round(int64_t it1, int64_t &q0, int &off0, ItemRec *items, uint64_t *sbits,
                                             int64_t bs, int bl, uint32_t rx, uint32_t ry, int *nitems = nullptr,
                                             bool *fin = nullptr)
{
    const int lane = (int)__lane_id();
    if (lane == 0) {
        bs += off0;
        bl -= off0;
    }
    const int blc = min(bl, kRoundW);
    const int incl = wave_incl_scan(blc);
    const int P = incl - blc;
    const int E = uniform(min(__shfl(incl, 63), kRoundW));
    const bool in = blc > 0 && P < kRoundW;
    const uint64_t inb = __ballot(in);
    if (nitems) *nitems = __popcll(inb);
    if (in) {
        ItemRec r;
        r.bs = (uint32_t)bs;
        r.P = P;
        r.x = rx;
        r.y = ry;
        items[__popcll(inb & lanemask_lt(lane))] = r;
        atomicOr((unsigned long long *)&sbits[P >> 6], 1ull << (P & 63));
    }
    // fin: this lane's item needs nothing from later rounds
    if (fin) *fin = blc == 0 || (in && (int64_t)P + bl <= kRoundW);
    const uint64_t cutb = __ballot(in && (int64_t)P + bl > kRoundW);
    if (cutb) {
        const int cl = __ffsll((unsigned long long)cutb) - 1;
        const int used = kRoundW - __shfl(P, cl);
        off0 = (cl == 0 ? off0 : 0) + used;
        q0 += cl;
    } else {
        const uint64_t rest = __ballot(!in && blc > 0);
        if (rest) {
            q0 += __ffsll((unsigned long long)rest) - 1;
        } else {
            q0 = min(q0 + 64, it1);
        }
        off0 = 0;
    }
    return E;
}

// Loads the next round of a unit's items into LDS: lane i takes column q0+i
// of the unit (every product of row k of B).  For a cluster's numeric phase
// lane i also keeps the column's member values (areg, or aval[i*S ..]).
template <bool CL, int S, bool NUM>
__device__ __forceinline__ int load_round(const SpArgs &a, const UnitView &v, int64_t &q0, int &off0,
                                          ItemRec *items, uint64_t *sbits, double *aval, double *areg,
                                          int *nitems = nullptr)
{
    const int lane = (int)__lane_id();
    sbits[lane] = 0ull;
    const int64_t q = q0 + lane;
    int64_t bs = 0;
    int bl = 0;
    uint32_t m = 1u;
    double a1 = 0.0;
    if (q < v.it1) {
        const int k = CL ? a.cl_col[q] : a.a_col[q];
        if (CL && S > 1) m = a.cl_mask[q];
        bs = a.b_rp[k];
        bl = (int)(a.b_rp[k + 1] - bs);
        if (NUM) {
            if (CL && S > 1) {
                const double *src = a.cl_val + v.vbase + (q - v.it0) * v.s;
#pragma unroll
                for (int l = 0; l < S; ++l) {
                    if (a_in_regs(S))
                        areg[l] = l < v.s ? src[l] : 0.0;
                    else if (l < v.s)
                        aval[lane * S + l] = src[l];
                }
            } else {
                // a CSR row, or a one-row cluster (its values are contiguous)
                a1 = CL ? a.cl_val[v.vbase + (q - v.it0)] : a.a_val[q];
            }
        }
    }
    // record words: a cluster's member mask and the lane holding its values,
    // else the two halves of a_ik
    const uint64_t ab = (uint64_t)__double_as_longlong(a1);
    const uint32_t rx = CL && S > 1 ? m : (uint32_t)ab;
    const uint32_t ry = CL && S > 1 ? (uint32_t)lane : (uint32_t)(ab >> 32);
    return flatten_round(v.it1, q0, off0, items, sbits, bs, bl, rx, ry, nitems);
}

// One lane's share of one pass: its entry of the flattened product list.
// Lanes past the end get the dummy key and read B at offset 0; FULL passes
// (every lane inside the round) skip those checks.
template <bool MS, bool NUM>
struct Pass {
    int j;
    int t;        // item index (lanes past the end: the last item)
    uint32_t m;   // cluster: the item's row mask (symbolic)
    double b;     // numeric: b_kj (a_ik is read per item when the products are applied)
};

template <bool MS, bool NUM, bool FULL = false>
__device__ __forceinline__ Pass<MS, NUM> fetch_pass(const SpArgs &a, const ItemRec *items, uint64_t w, int cum,
                                                    int e, int E, uint64_t le)
{
    Pass<MS, NUM> d;
    // start bits at or below this lane: bit 0 plus the bits of w >> 1 below it
    const uint64_t w1 = w >> 1;
    d.t = cum + (int)(w & 1ull) - 1 +
          (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(w1 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)w1, 0u));
    (void)le;
    const ItemRec it = items[d.t];
    const bool ok = FULL || e < E;
    const uint32_t off = ok ? it.bs + (uint32_t)(e - it.P) : 0u;
    const int j = ld_col(a.b_col, off);
    d.j = ok ? j : kDummyKey;
    d.m = MS ? it.x : 1u;
    if (NUM) {
        const double b = ld_val(a.b_val, off);
        d.b = ok ? b : 0.0;
    }
    return d;
}

// ================================================================ symbolic
// Counts, per member row, its distinct output columns, and per unit the
// distinct columns of the union (used to size the numeric tables) and their
// smallest and largest value (used by the numeric phase's hash).  Keys go
// into a power-of-two open-addressing table with a multiplicative hash; the
// table has at least as many slots as the unit has products (by default
// 100/70 times as many, so it stays at most 70% full even when nearly every
// product hits a new column), so it never fills.  For clusters each key
// carries the OR of the masks of the columns k that reached it (atomic ORs
// that return nothing); once every product is in, one sweep over the table
// counts the keys and, per member row l, the keys whose bit l is set.
// Rounds of short items (at most 32 products each, 24 on average) are walked
// two items per pass, one per half of the wavefront, which needs no per-lane
// item search.
template <int S, bool CL>
__device__ __forceinline__ void sym_unit(const SpArgs &a, const int u, unsigned char *base)
{
    constexpr bool MS = CL && S > 1;  // several member rows (masks needed)
    const int lane = (int)__lane_id();
    const int T = a.T;
    const SymLayout L(MS ? (S <= 8 ? 1 : 2) : 0, T);
    int *keys = (int *)(base + L.keys);
    MaskT<S> *masks = (MaskT<S> *)(base + L.masks);
    ItemRec *items = (ItemRec *)(base + L.items);
    uint64_t *sbits = (uint64_t *)(base + L.sbits);
    lds_fill(keys, 4 * T, (uint32_t)kEmpty);
    if (MS) lds_fill(masks, (S <= 8 ? 1 : 2) * (T + 1), 0u);
    const UnitView v = unit_view<CL>(a, u);
    const uint32_t hmask = (uint32_t)T - 1u;
    const int hshift = 32 - a.log2T;
    const uint64_t le = lanemask_le(lane);
    int inserted = 0;  // one-row units: keys this lane inserted
    int kmin = INT_MAX, kmax = -1;
    int64_t q0 = v.it0;
    int off0 = 0;

    // key j into the table (one compare-and-swap takes an empty slot or
    // confirms the key already there; only collisions walk on), its mask
    // ORed into the slot's.  The table has more slots than the unit has
    // products, so the walk always ends.
    auto insert = [&](int j, uint32_t m) {
        kmin = min(kmin, j);
        kmax = max(kmax, j);
        uint32_t h = ((uint32_t)j * 2654435761u) >> hshift;
        int old = atomicCAS(&keys[h], kEmpty, j);
        while (old != kEmpty && old != j) {
            h = (h + 1u) & hmask;
            old = atomicCAS(&keys[h], kEmpty, j);
        }
        if (MS) mask_set<S>(masks, h, m);
        else inserted += old == kEmpty;
    };

    // two items per pass: half h of the wavefront takes item t0 + 2 rr + h
    auto paired_round = [&](int nit, int E) {
        {
            // each item's product count replaces its position in the record
            const int t = lane;
            const int Pt = t < nit ? items[t].P : 0;
            const int Pn = t + 1 < nit ? items[t + 1].P : E;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if (t < nit) items[t].P = Pn - Pt;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        const int half = lane >> 5, e = lane & 31;
        constexpr int kP = 8;
        for (int t0 = 0; t0 < nit; t0 += 2 * kP) {
            int j[kP];
            uint32_t m[kP];
            bool ok[kP];
#pragma unroll
            for (int rr = 0; rr < kP; ++rr) {
                const int ti = t0 + 2 * rr + half;
                const ItemRec it = items[min(ti, nit - 1)];
                ok[rr] = ti < nit && e < it.P;
                // (the select keeps the load ahead of its use rather than inside the branch)
                const int jj = ld_col(a.b_col, ok[rr] ? it.bs + (uint32_t)e : 0u);
                j[rr] = ok[rr] ? jj : kDummyKey;
                m[rr] = it.x;
            }
#pragma unroll
            for (int rr = 0; rr < kP; ++rr) {
                if (t0 + 2 * rr >= nit) break;
                if (j[rr] != kDummyKey) insert(j[rr], m[rr]);  // (tests the loaded key: idle lanes hold the dummy)
            }
        }
    };

    constexpr int kR = 8;
    while (q0 < v.it1) {
        int nit = 0;
        const int E = load_round<CL, S, false>(a, v, q0, off0, items, sbits, nullptr, nullptr, &nit);
        {
            const int t = lane;
            const int Pt = t < nit ? items[t].P : 0;
            const int Pn = t + 1 < nit ? items[t + 1].P : E;
            if (uniform(nit) > 0 && E >= 24 * uniform(nit) && __ballot(t < nit && Pn - Pt > 32) == 0ull) {
                paired_round(uniform(nit), E);
                continue;
            }
        }
        const int npass = (E + 63) >> 6;
        int cum = 0, p = 0;
        auto batch = [&](auto full_t) {
            constexpr bool FULL = decltype(full_t)::value;
            Pass<MS, false> d[kR];
#pragma unroll
            for (int rr = 0; rr < kR; ++rr) {
                const uint64_t w = uniform64(sbits[p + rr]);
                d[rr] = fetch_pass<MS, false, FULL>(a, items, w, cum, ((p + rr) << 6) + lane, E, le);
                cum += __popcll(w);
            }
#pragma unroll
            for (int rr = 0; rr < kR; ++rr)
                if (FULL || d[rr].j != kDummyKey) insert(d[rr].j, d[rr].m);
        };
        for (; p + kR <= npass; p += kR) {
            if (((p + kR) << 6) <= E) batch(std::true_type{});
            else batch(std::false_type{});
        }
        for (; p < npass; ++p) {
            const uint64_t w = uniform64(sbits[p]);
            const Pass<MS, false> d = fetch_pass<MS, false>(a, items, w, cum, (p << 6) + lane, E, le);
            cum += __popcll(w);
            if (d.j != kDummyKey) insert(d.j, d.m);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, __shfl_xor(kmin, o));
        kmax = max(kmax, __shfl_xor(kmax, o));
    }
    if (lane == 0) {
        a.keylo[u] = kmin;
        a.keyhi[u] = kmax;
    }
    if (!MS) {
        int U = inserted;
        for (int o = 32; o > 0; o >>= 1) U += __shfl_xor(U, o);
        if (lane == 0) {
            a.c_rp[member_row<CL>(a, v, 0)] = U;
            a.ucount[u] = U;
        }
        return;
    }
    // the keys, and per member the keys whose bit is set (T is a multiple of 64)
    int U = 0;
    int mcnt[S];  // wave-uniform per-member counts
#pragma unroll
    for (int l = 0; l < S; ++l) mcnt[l] = 0;
    for (int c0 = 0; c0 < T; c0 += 64) {
        const int sidx = c0 + lane;
        U += __popcll(__ballot(keys[sidx] != kEmpty));
        const uint32_t mk = (uint32_t)masks[sidx];
#pragma unroll
        for (int l = 0; l < S; ++l)
            if (l < v.s) mcnt[l] += __popcll(__ballot((mk >> l) & 1u));
    }
    int mine = 0;
#pragma unroll
    for (int l = 0; l < S; ++l)
        if (l == lane) mine = mcnt[l];
    if (lane < v.s) a.c_rp[member_row<CL>(a, v, lane)] = mine;
    if (lane == 0) a.ucount[u] = U;
}

// ================================================================ numeric
// Keys go into a table of T slots plus a short tail, placed by an
// order-preserving hash h(j) = floor((j - lo) * T / (hi - lo + 1)) (lo/hi:
// the unit's smallest and largest output column) with linear probing.
// Because h never decreases with j, a key's rank among the unit's keys is
// the number of keys whose home slot is lower (a prefix sum of per-home
// counts, taken once all keys are in) plus the smaller keys with the same home,
// which all lie on the probe path from that home; no sort is needed, and a
// CSR row's entries are written straight to their final positions.
// PRED (CSR rows only): no symbolic phase ran; the table was sized from a
// predicted capacity (ucount) and the key range is a bound from the rows of
// B.  Probing gives up when the table is full, and a row whose keys did not
// fit or exceed the capacity records -1 as its count and writes nothing;
// otherwise its entries go to its padded slot (pad_off) and its count to
// c_rp[row].
// PAIRS: rounds of short items may be walked two items per pass (off in the
// batch kernels, whose register budget is tighter).
template <int S, bool CL, bool PRED = false, bool PAIRS = true, bool HASHED = false>
__device__ __forceinline__ void num_unit(const SpArgs &a, const int u, unsigned char *base)
{
    static_assert(!PRED || (S == 1 && !CL), "predicted sizes are for CSR rows");
    constexpr bool MS = CL && S > 1;  // several member rows (masks needed)
    const int lane = (int)__lane_id();
    if (u < a.unit_lo || u >= a.unit_hi) return;

    const int T = a.T, TX = a.T + num_tail(a.T);
    const NumLayout L(MS, S, T, a.vcap);
    int *keys = (int *)(base + L.keys);
    uint16_t *vidx = (uint16_t *)(base + L.vidx);  // MS: slot -> value entry
    MaskT<S> *masks = (MaskT<S> *)(base + L.masks);
    double *vals = (double *)(base + L.vals);
    double *aval = (double *)(base + L.aval);
    uint16_t *order = (uint16_t *)(base + L.order);
    ItemRec *items = (ItemRec *)(base + L.items);
    uint64_t *sbits = (uint64_t *)(base + L.sbits);
    // per-home key counts, then their exclusive prefix (16 bits: a table holds
    // fewer than 2^16 keys); counted through the aligned 32-bit words once the
    // passes are done (the array may share the item area)
    uint16_t *hcnt = (uint16_t *)(base + L.hcnt);

    // value column stride: entries incl. the dummy (MS: one per key, else one per slot)
    const int VS = MS ? a.vcap + 1 : TX + 1;
    const UnitView v = unit_view<CL>(a, u);
    lds_fill(keys, 4 * TX, (uint32_t)kEmpty);
    if (MS) {
        lds_fill(vidx, 2 * (TX + 1), (uint32_t)a.vcap * 0x10001u);  // the dummy entry until a key takes the slot
        lds_fill(masks, (int)sizeof(MaskT<S>) * VS, 0u);
    }
    lds_fill(vals, 8 * S * VS, 0u);
    if (lane == 0) keys[TX] = kDummyKey;
    int nkeys = 0;  // MS: value entries handed out (wave-uniform)
    const int lo = a.keylo[u], hi = a.keyhi[u];
    const float scale = __fdividef((float)T, (float)(uint32_t)(hi - lo + 1));
    const uint64_t le = lanemask_le(lane);
    int64_t q0 = v.it0;
    int off0 = 0;
    double areg[S];  // this lane's item: member values of A (narrow clusters)
#pragma unroll
    for (int l = 0; l < S; ++l) areg[l] = 0.0;

    auto home = [&](int j) -> int {
        if (HASHED) return (int)__umulhi((uint32_t)j * 2654435761u, (uint32_t)T);
        const int h = (int)((float)(uint32_t)(j - lo) * scale);
        return h < T ? h : T - 1;
    };
    bool full = false;  // PRED: a key found no free slot
    bool fresh = false;  // MS: this lane's last probe inserted its key
    auto probe = [&](int j, auto full_t) -> int {
        fresh = false;
        if (!decltype(full_t)::value && j == kDummyKey) return TX;
        const int h0 = home(j);
        int h = h0;
        int old = atomicCAS(&keys[h], kEmpty, j);
        int steps = 0;
        while (old != kEmpty && old != j) {
            if (PRED && ++steps >= TX) {
                full = true;
                return TX;
            }
            if (++h == TX) h = 0;
            old = atomicCAS(&keys[h], kEmpty, j);
        }
        fresh = old == kEmpty;
        return h;
    };
    // MS: the value entry of slot h; keys inserted by this pass get the next
    // entries in lane order.  A lane that found its key may read the entry
    // another lane has just written: the fence keeps every write before every
    // read (the compiler would otherwise be free to run the reading lanes'
    // branch first).
    auto entry = [&](int h) -> int {
        if (!MS) return h;
        const uint64_t fb = __ballot(fresh);
        if (fresh) vidx[h] = (uint16_t)min(nkeys + (int)__popcll(fb & lanemask_lt(lane)), a.vcap);
        nkeys += (int)__popcll(fb);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        return vidx[h];
    };
    // products of one pass, applied item by item (ascending k)
    auto apply = [&](const Pass<MS, true> &d, int h, int tf, int tl) {
        for (int tt = tf; tt <= tl; ++tt) {
            if (d.t != tt) continue;
            if (MS) {
                const uint32_t mt = (uint32_t)uniform((int)items[tt].x);
                const int src = uniform((int)items[tt].y);
                mask_set<S>(masks, (uint32_t)h, mt);
#pragma unroll
                for (int l = 0; l < S; ++l) {
                    if ((mt >> l) & 1u) {
                        const double av = a_in_regs(S) ? readlane_f64(areg[l], src) : aval[src * S + l];
                        double *pv = &vals[l * VS + h];
                        *pv = __fma_rn(av, d.b, *pv);
                    }
                }
            } else {
                // the item's a_ik (same address in every lane)
                const double av = *(const double *)&items[tt].x;
                vals[h] = __fma_rn(av, d.b, vals[h]);
            }
        }
    };

    // a round whose items have at most 32 products each (24 on average) is
    // walked two items per pass, one per half of the wavefront: the products of the first half
    // are applied before those of the second, so each output entry still gets
    // its products in ascending k, in two fixed sub-steps per pass
    auto paired_round = [&](int nit, int E) {
        // each item's product count replaces its position in the record
        const int t = lane;
        const int Pt = t < nit ? items[t].P : 0;
        const int Pn = t + 1 < nit ? items[t + 1].P : E;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (t < nit) items[t].P = Pn - Pt;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int half = lane >> 5, e = lane & 31;
        constexpr int kP = Depth<S>::R;
        for (int t0 = 0; t0 < nit; t0 += 2 * kP) {
            int j[kP];
            double b[kP];
            ItemRec it[kP];
            bool ok[kP];
#pragma unroll
            for (int rr = 0; rr < kP; ++rr) {
                const int ti = t0 + 2 * rr + half;
                it[rr] = items[min(ti, nit - 1)];
                ok[rr] = ti < nit && e < it[rr].P;
                const uint32_t off = ok[rr] ? it[rr].bs + (uint32_t)e : 0u;
                const int jj = ld_col(a.b_col, off);
                const double bb = ld_val(a.b_val, off);
                j[rr] = ok[rr] ? jj : kDummyKey;
                b[rr] = ok[rr] ? bb : 0.0;
            }
#pragma unroll
            for (int rr = 0; rr < kP; ++rr) {
                if (t0 + 2 * rr >= nit) break;
                const int h = entry(probe(j[rr], std::false_type{}));
                for (int hf = 0; hf < 2; ++hf) {
                    if (half == hf && ok[rr]) {
                        if (MS) {
                            // the active lanes all hold item t0 + 2 rr + hf: its mask and
                            // the lane with its member values are uniform among them
                            const uint32_t mt = (uint32_t)uniform((int)it[rr].x);
                            const int src = uniform((int)it[rr].y);
                            mask_set<S>(masks, (uint32_t)h, mt);
#pragma unroll
                            for (int l = 0; l < S; ++l) {
                                if ((mt >> l) & 1u) {
                                    const double av = a_in_regs(S) ? readlane_f64(areg[l], src) : aval[src * S + l];
                                    double *pv = &vals[l * VS + h];
                                    *pv = __fma_rn(av, b[rr], *pv);
                                }
                            }
                        } else {
                            const double av = __longlong_as_double(((long long)it[rr].y << 32) | it[rr].x);
                            vals[h] = __fma_rn(av, b[rr], vals[h]);
                        }
                    }
                }
            }
        }
    };

    constexpr int kR = Depth<S>::R;
    while (q0 < v.it1) {
        int nit = 0;
        const int E = load_round<CL, S, true>(a, v, q0, off0, items, sbits, aval, areg, &nit);
        {
            const int t = lane;
            const int Pt = t < nit ? items[t].P : 0;
            const int Pn = t + 1 < nit ? items[t + 1].P : E;
            // two items per pass pay when they fill most of the lanes: at most
            // 32 products each, at least 24 on average
            if (PAIRS && uniform(nit) > 0 && E >= 24 * uniform(nit) && __ballot(t < nit && Pn - Pt > 32) == 0ull) {
                paired_round(uniform(nit), E);
                continue;
            }
        }
        const int npass = (E + 63) >> 6;
        int cum = 0, p = 0;
        auto batch = [&](auto full_t) {
            constexpr bool FULL = decltype(full_t)::value;
            Pass<MS, true> d[kR];
            int tf[kR], tl[kR];
#pragma unroll
            for (int rr = 0; rr < kR; ++rr) {
                const uint64_t w = uniform64(sbits[p + rr]);
                tf[rr] = cum + (int)(w & 1ull) - 1;
                tl[rr] = cum + (FULL ? __popcll(w) : __popcll(w & lanemask_le(min(63, E - 1 - ((p + rr) << 6))))) - 1;
                d[rr] = fetch_pass<MS, true, FULL>(a, items, w, cum, ((p + rr) << 6) + lane, E, le);
                cum += __popcll(w);
            }
#pragma unroll
            for (int rr = 0; rr < kR; ++rr) apply(d[rr], entry(probe(d[rr].j, full_t)), tf[rr], tl[rr]);
        };
        for (; p + kR <= npass; p += kR) {
            if (((p + kR) << 6) <= E) batch(std::true_type{});
            else batch(std::false_type{});
        }
        for (; p < npass; ++p) {
            const uint64_t w = uniform64(sbits[p]);
            const int last = min(63, E - 1 - (p << 6));
            const int tf = cum + (int)(w & 1ull) - 1;
            const int tl = cum + __popcll(w & lanemask_le(last)) - 1;
            const Pass<MS, true> d = fetch_pass<MS, true>(a, items, w, cum, (p << 6) + lane, E, le);
            cum += __popcll(w);
            apply(d, entry(probe(d.j, std::false_type{})), tf, tl);
        }
    }

    // ---- rank every key.  h never decreases with j, so a key x with home hx
    // is larger than every key homed below hx and smaller than every key homed
    // above it.  With linear probing every slot from a key's home to the key
    // is occupied, and a key stored below hx is homed below hx.  Hence, when
    // no probe run reaches the table's last slot (no run wrapped around):
    //   rank(x) = (occupied slots below hx) + (keys smaller than x from hx up
    //             to the end of the run),
    // the first term from an occupancy bitmap.  Otherwise the general form:
    // keys homed below hx (a prefix sum of per-home counts) plus the smaller
    // keys sharing hx, which lie on the probe path from hx.  (A predicted
    // table that filled up, or holds more keys than the row's capacity, is
    // given up before ranking.)  HASHED: the bucket sort described at
    // kHashedMinT.
    uint64_t *obits = (uint64_t *)(base + L.obits);
    int *opre = (int *)(base + L.opre);
    int *bend = (int *)(base + L.bend);
    int *arr = (int *)(base + L.arr);
    int U = 0;
    for (int c0 = 0; c0 < TX; c0 += 64) {
        const int sidx = c0 + lane;
        const uint64_t occ = __ballot(sidx < TX && keys[sidx] != kEmpty);
        if (!HASHED && lane == 0) {
            obits[c0 >> 6] = occ;
            opre[c0 >> 6] = U;
        }
        U += __popcll(occ);
    }
    const int64_t row0 = member_row<CL>(a, v, 0);
    if (PRED && (__ballot(full) != 0ull || U > a.ucount[u])) {
        if (lane == 0) a.c_rp[row0] = -1;
        return;
    }
    const int NB = T >> 1;
    const float bscale = __fdividef((float)NB, (float)(uint32_t)(hi - lo + 1));
    auto bucket = [&](int j) -> int {
        const int b = (int)((float)(uint32_t)(j - lo) * bscale);
        return b < NB ? b : NB - 1;
    };
    if (HASHED) {
        // counts per bucket, their inclusive prefix (bucket ends), then the
        // keys placed from each bucket's end down (the ends become starts)
        lds_fill(bend, 4 * NB, 0u);  // NB is a multiple of 4
        if (lane == 0) bend[NB] = U;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int c0 = 0; c0 < TX; c0 += 64) {
            const int sidx = c0 + lane;
            const int key = sidx < TX ? keys[sidx] : kEmpty;
            if (key != kEmpty) atomicAdd(&bend[bucket(key)], 1);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        int run = 0;
        for (int c0 = 0; c0 < NB; c0 += 64) {
            const int cnt = bend[c0 + lane];
            const int incl = wave_incl_scan(cnt);
            bend[c0 + lane] = run + incl;
            run += __shfl(incl, 63);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int c0 = 0; c0 < TX; c0 += 64) {
            const int sidx = c0 + lane;
            const int key = sidx < TX ? keys[sidx] : kEmpty;
            if (key != kEmpty) arr[atomicSub(&bend[bucket(key)], 1) - 1] = key;
        }
    }
    const bool runs_end = !HASHED && uniform(keys[TX - 1]) != kEmpty;
    if (runs_end) {
        for (int i = lane; 2 * i < T; i += 64) ((uint32_t *)hcnt)[i] = 0u;  // T is even
        for (int c0 = 0; c0 < TX; c0 += 64) {
            const int sidx = c0 + lane;
            const int key = sidx < TX ? keys[sidx] : kEmpty;
            if (key == kEmpty) continue;
            const int h0 = home(key);
            atomicAdd((uint32_t *)(hcnt + (h0 & ~1)), 1u << (16 * (h0 & 1)));
        }
        int V = 0;
        for (int c0 = 0; c0 < T; c0 += 64) {
            const int i = c0 + lane;
            const int cnt = i < T ? hcnt[i] : 0;
            const int incl = wave_incl_scan(cnt);
            if (i < T) hcnt[i] = (uint16_t)(V + incl - cnt);
            V += __shfl(incl, 63);
        }
        if (lane == 0) hcnt[T] = (uint16_t)V;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const bool cl_out = CL && !PRED && a.oc_col != nullptr;  // C in CSR_Cluster form
    int64_t o0 = 0, want = 0, vo = 0;
    int32_t *ccol = nullptr;
    double *cval = nullptr;
    if (PRED) {
        o0 = a.pad_off[row0];
        want = U;
    } else if (cl_out) {
        o0 = a.oc_col_ptr[u];
        want = a.oc_col_ptr[u + 1] - o0;
        vo = a.oc_val_ptr[u];
    } else if (!MS) {
        o0 = a.c_rp[row0] - a.out_base;
        want = a.c_rp[row0 + 1] - a.c_rp[row0];
    }
    // a CSR row's place in C (uniform): the whole row must fit, else every
    // entry is reported and none written
    const bool row_fits = cl_out ? o0 >= 0 && o0 + want <= a.oc_ncc && vo >= 0 &&
                                       vo + want * v.s <= a.oc_nslots && a.oc_val_ptr[u + 1] - vo == want * v.s
                                 : o0 >= 0 && o0 + want <= a.cap;
    if (!MS && row_fits) {
        ccol = (cl_out ? a.oc_col : a.c_col) + o0;
        cval = cl_out ? a.oc_val + vo : a.c_val + o0;
    }
    for (int c0 = 0; c0 < TX; c0 += 64) {
        const int sidx = c0 + lane;
        const int key = sidx < TX ? keys[sidx] : kEmpty;
        if (key == kEmpty) continue;
        const int hx = home(key);
        int rank;
        if (HASHED) {
            const int b = bucket(key);
            const int s0 = bend[b], s1 = bend[b + 1];
            rank = s0;
            for (int t = s0; t < s1; ++t) rank += arr[t] < key;
        } else if (!runs_end) {
            rank = opre[hx >> 6] + __popcll(obits[hx >> 6] & lanemask_lt(hx & 63));
            for (int x = hx;; ++x) {  // ends at an empty slot below TX - 1
                const int kx = keys[x];
                if (kx == kEmpty) break;
                rank += kx < key;
            }
        } else {
            rank = hcnt[hx];
            if ((int)hcnt[hx + 1] - rank > 1) {
                for (int x = hx;; x = x + 1 == TX ? 0 : x + 1) {
                    const int kx = keys[x];
                    if (kx == kEmpty) break;
                    rank += kx < key && home(kx) == hx;
                }
            }
        }
        if (MS) {
            order[rank] = (uint16_t)sidx;
        } else {
            // a CSR row goes straight to its place in C
            if (row_fits && rank < want) {
                ccol[rank] = key;
                cval[rank] = vals[sidx];
                if (cl_out) a.oc_mask[o0 + rank] = 1;  // a one-row cluster
            } else {
                atomicOr(a.err, kErrCapacity);
            }
        }
    }
    if (PRED) {
        if (lane == 0) a.c_rp[row0] = U;
        return;
    }
    if (!MS) {
        if (lane == 0 && U != want) atomicOr(a.err, kErrCount);
        return;
    }

    // ---- C in CSR_Cluster form: the union columns in order, their masks and
    // the member values (the accumulator of a member that lacks a column was
    // never touched and holds +0.0)
    if (lane == 0 && nkeys > a.vcap) atomicOr(a.err, kErrCount);  // more keys than the bin allows
    if (cl_out) {
        if (!row_fits) {
            if (lane == 0) atomicOr(a.err, kErrCapacity);
            return;
        }
        if (lane == 0 && U != want) atomicOr(a.err, kErrCount);
        for (int i = lane; i < U && i < want; i += 64) {
            const int sl = order[i];
            const int id = vidx[sl];
            a.oc_col[o0 + i] = keys[sl];
            a.oc_mask[o0 + i] = (uint16_t)masks[id];
#pragma unroll
            for (int l = 0; l < S; ++l)
                if (l < v.s) a.oc_val[vo + (int64_t)i * v.s + l] = vals[l * VS + id];
        }
        return;
    }

    // ---- each member row's entries, in column order: one sweep over the
    // keys writes every member's row (a key goes to the rows of its mask)
    int64_t my_off = 0, my_want = 0;
    if (lane < v.s) {
        const int64_t row = member_row<CL>(a, v, lane);
        my_off = a.c_rp[row] - a.out_base;
        my_want = a.c_rp[row + 1] - a.c_rp[row];
    }
    int64_t roff[S], rwant[S], w[S];
#pragma unroll
    for (int l = 0; l < S; ++l) {
        roff[l] = l < v.s ? readlane_i64(my_off, l) : 0;
        rwant[l] = l < v.s ? readlane_i64(my_want, l) : 0;
        w[l] = 0;
    }
    for (int c0 = 0; c0 < U; c0 += 64) {
        const int i = c0 + lane;
        const int sl = i < U ? (int)order[i] : TX;
        const int id = vidx[sl];
        const uint32_t m = i < U ? (uint32_t)masks[id] : 0u;
        const int key = keys[sl];
#pragma unroll
        for (int l = 0; l < S; ++l) {
            if (l >= v.s) break;
            const bool has = (m >> l) & 1u;
            const uint64_t bal = __ballot(has);
            if (has) {
                const int64_t pos = w[l] + __popcll(bal & lanemask_lt(lane));
                const int64_t dst = roff[l] + pos;
                if (dst >= 0 && dst < a.cap && pos < rwant[l]) {
                    a.c_col[dst] = key;
                    a.c_val[dst] = vals[l * VS + id];
                } else {
                    atomicOr(a.err, kErrCapacity);
                }
            }
            w[l] += __popcll(bal);
        }
    }
#pragma unroll
    for (int l = 0; l < S; ++l)
        if (l < v.s && lane == 0 && w[l] != rwant[l]) atomicOr(a.err, kErrCount);
}

// ================================================================ global-memory path
// Units of a batch whose tables do not fit in shared memory (single products
// take the column-window path below instead).  Each wavefront owns a
// bitmap over all columns of B (and, numeric, a value array of the same
// width) in the workspace and takes units one after another; the products
// are walked in the same 64-wide passes as above.  Cluster members are done
// one after another (a product counts for member l when bit l of its
// column's mask is set).
constexpr int kGmSym = 16 * 64 + 8 * kRoundPasses;     // items + start bits
constexpr int kGmNumCl = kGmSym + 8 * 16 * 64;         // + staged cluster values

template <bool BATCH>
__device__ __forceinline__ int gm_unit(SpArgs &a, const SpArgs &a0, int64_t i)
{
    a = a0;
    return BATCH ? batch_resolve(a, a0.order[i]) : uniform(a0.order[i]);
}

// Symbolic: bits are set with atomic ORs that return nothing (no wait per
// product); the row's count is the popcount of its bitmap, which the same
// sweep clears for the next row.
template <bool CL, bool BATCH>
__global__ void __launch_bounds__(256) k_sym_gm(SpArgs a0)
{
    constexpr int S = CL ? 16 : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = (int)__lane_id();
    const int wib = uniform((int)(threadIdx.x >> 6));
    const int64_t wv = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    unsigned char *base = smem + (size_t)wib * kGmSym;
    ItemRec *items = (ItemRec *)base;
    uint64_t *sbits = (uint64_t *)(base + 16 * 64);
    uint32_t *bm = a0.dense_bits + wv * a0.dense_words;
    const int64_t count = BATCH ? a0.dcount[a0.bin] : a0.count;
    const int64_t begin = BATCH ? a0.dbegin[a0.bin] : a0.bin_begin;
    const uint64_t le = lanemask_le(lane);
    for (int64_t ti = wv; ti < count; ti += nw) {
        SpArgs a;
        const int u = gm_unit<BATCH>(a, a0, begin + ti);
        const UnitView v = unit_view<CL>(a, u);
        for (int l = 0; l < v.s; ++l) {
            int64_t q0 = v.it0;
            int off0 = 0;
            while (q0 < v.it1) {
                const int E = load_round<CL, S, false>(a, v, q0, off0, items, sbits, nullptr, nullptr);
                const int npass = (E + 63) >> 6;
                int cum = 0;
                for (int p = 0; p < npass; ++p) {
                    const uint64_t w = uniform64(sbits[p]);
                    const Pass<CL, false> d = fetch_pass<CL, false>(a, items, w, cum, (p << 6) + lane, E, le);
                    cum += __popcll(w);
                    if (d.j != kDummyKey && (!CL || ((d.m >> l) & 1u))) atomicOr(&bm[d.j >> 5], 1u << (d.j & 31));
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
            int64_t cnt = 0;
            for (int64_t x = lane; x < a.dense_words; x += 64) {
                const uint32_t word = __hip_atomic_load(&bm[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (word) {
                    cnt += __popc(word);
                    bm[x] = 0u;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
            for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
            if (lane == 0) a.c_rp[member_row<CL>(a, v, l)] = cnt;
        }
        if (lane == 0) a.ucount[u] = INT32_MAX;
    }
}

// Numeric: within a pass the products are applied item by item (ascending
// k), and every item waits for its stores before the next item may read the
// same accumulator entries.  The first touch of a column (its bitmap bit)
// starts the entry from +0.0.  Output: the bitmap in column order.
template <bool CL, bool BATCH>
__global__ void __launch_bounds__(256) k_num_gm(SpArgs a0)
{
    constexpr int S = CL ? 16 : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = (int)__lane_id();
    const int wib = uniform((int)(threadIdx.x >> 6));
    const int64_t wv = (int64_t)blockIdx.x * (blockDim.x >> 6) + wib;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    unsigned char *base = smem + (size_t)wib * (CL ? kGmNumCl : kGmSym);
    ItemRec *items = (ItemRec *)base;
    uint64_t *sbits = (uint64_t *)(base + 16 * 64);
    double *aval = (double *)(base + kGmSym);
    uint32_t *bm = a0.dense_bits + wv * a0.dense_words;
    double *acc = a0.dense_vals + wv * a0.ncols;  // stride: the widest B of the launch
    const int64_t count = BATCH ? a0.dcount[a0.bin] : a0.count;
    const int64_t begin = BATCH ? a0.dbegin[a0.bin] : a0.bin_begin;
    const uint64_t le = lanemask_le(lane);
    for (int64_t ti = wv; ti < count; ti += nw) {
        SpArgs a;
        const int u = gm_unit<BATCH>(a, a0, begin + ti);
        if (u < a.unit_lo || u >= a.unit_hi) continue;
        const UnitView v = unit_view<CL>(a, u);
        for (int l = 0; l < v.s; ++l) {
            int64_t q0 = v.it0;
            int off0 = 0;
            while (q0 < v.it1) {
                const int E = load_round<CL, S, true>(a, v, q0, off0, items, sbits, aval, nullptr);
                const int npass = (E + 63) >> 6;
                int cum = 0;
                for (int p = 0; p < npass; ++p) {
                    const uint64_t w = uniform64(sbits[p]);
                    const int last = min(63, E - 1 - (p << 6));
                    const int tf = cum + (int)(w & 1ull) - 1;
                    const int tl = cum + __popcll(w & lanemask_le(last)) - 1;
                    const Pass<CL, true> d = fetch_pass<CL, true>(a, items, w, cum, (p << 6) + lane, E, le);
                    cum += __popcll(w);
                    for (int tt = tf; tt <= tl; ++tt) {
                        double av = CL ? 0.0 : *(const double *)&items[tt].x;  // a_ik of the item
                        if (CL) {
                            if (!((uniform((int)items[tt].x) >> l) & 1)) continue;
                            av = aval[uniform((int)items[tt].y) * S + l];
                        }
                        if (d.t == tt && d.j != kDummyKey) {
                            const uint32_t bit = 1u << (d.j & 31);
                            const uint32_t old = atomicOr(&bm[d.j >> 5], bit);
                            const double prev = (old & bit) ? __hip_atomic_load(&acc[d.j], __ATOMIC_RELAXED,
                                                                                 __HIP_MEMORY_SCOPE_WORKGROUP)
                                                            : 0.0;
                            __hip_atomic_store(&acc[d.j], __fma_rn(av, d.b, prev), __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
            const int64_t row = member_row<CL>(a, v, l);
            const int64_t o0 = a.c_rp[row] - a.out_base;
            const int64_t want = a.c_rp[row + 1] - a.c_rp[row];
            int64_t wsum = 0;
            for (int64_t w0 = 0; w0 < a.dense_words; w0 += 64) {
                const int64_t wi = w0 + lane;
                uint32_t word = wi < a.dense_words
                                    ? __hip_atomic_load(&bm[wi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                    : 0u;
                const int c = __popc(word);
                const int pre = wave_incl_scan(c);
                const int tot = __shfl(pre, 63);
                int64_t dst = o0 + wsum + pre - c;
                if (word) bm[wi] = 0u;
                while (word) {
                    const int b = __ffs(word) - 1;
                    word &= word - 1u;
                    const int j = (int)(wi * 32 + b);
                    if (dst >= 0 && dst < a.cap && dst - o0 < want) {
                        a.c_col[dst] = j;
                        a.c_val[dst] = __hip_atomic_load(&acc[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        atomicOr(a.err, kErrCapacity);
                    }
                    ++dst;
                }
                wsum += tot;
            }
            if (lane == 0 && wsum != want) atomicOr(a.err, kErrCount);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
        }
    }
}

hipError_t launch_sym_dense(bool cluster, bool batch, const SpArgs &a, int blocks, hipStream_t s)
{
    const size_t lds = 4 * (size_t)kGmSym;
    if (cluster && batch) hipLaunchKernelGGL((k_sym_gm<true, true>), dim3(blocks), dim3(256), lds, s, a);
    else if (cluster) hipLaunchKernelGGL((k_sym_gm<true, false>), dim3(blocks), dim3(256), lds, s, a);
    else if (batch) hipLaunchKernelGGL((k_sym_gm<false, true>), dim3(blocks), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((k_sym_gm<false, false>), dim3(blocks), dim3(256), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_num_dense(bool cluster, bool batch, const SpArgs &a, int blocks, hipStream_t s)
{
    const size_t lds = 4 * (size_t)(cluster ? kGmNumCl : kGmSym);
    if (cluster && batch) hipLaunchKernelGGL((k_num_gm<true, true>), dim3(blocks), dim3(256), lds, s, a);
    else if (cluster) hipLaunchKernelGGL((k_num_gm<true, false>), dim3(blocks), dim3(256), lds, s, a);
    else if (batch) hipLaunchKernelGGL((k_num_gm<false, true>), dim3(blocks), dim3(256), lds, s, a);
    else hipLaunchKernelGGL((k_num_gm<false, false>), dim3(blocks), dim3(256), lds, s, a);
    return hipGetLastError();
}

// ================================================================ column windows
// Units of a single product whose tables do not fit in shared memory: their
// rows (a CSR row, or each member row of a cluster) are taken one by one, a
// workgroup each, and their output columns are held in a bitmap in shared
// memory.  The symbolic phase counts a row's columns per column chunk (equal
// column ranges, more for units with more products, win_nchunks); the
// numeric phase takes one chunk per workgroup and writes its entries after
// those of the chunks before it, in windows of the chunk's columns.  A
// window's products are the entries of the rows of B that fall inside it
// (found by binary search or carried over from the window before, the rows
// of B being sorted), walked in ascending k as everywhere else, so every
// output entry still receives its products in ascending k, one fma each
// from +0.0.

// First position in [lo, hi) of B's columns whose column is >= x (hi if none).
__device__ __forceinline__ uint32_t lower_bound_col(const int32_t *col, uint32_t lo, uint32_t hi, int x)
{
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ld_col(col, mid) < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// First position in [lo, hi) of B's columns whose column is >= x (hi if none),
// by doubling steps from lo and then a binary search: a few loads when the
// answer lies near lo, one when lo itself qualifies.
__device__ __forceinline__ uint32_t gallop_col(const int32_t *col, uint32_t lo, uint32_t hi, int x)
{
    uint32_t b = lo, s = 1;
    while (b + s - 1 < hi && ld_col(col, b + s - 1) < x) {
        b += s;
        s <<= 1;
    }
    return lower_bound_col(col, b, min(b + s - 1, hi), x);
}

// A row of the window path: a CSR row (items: its columns), or member l of
// a cluster of s rows (items: the cluster's union columns whose mask has
// bit l; values at vbase + t*s + l for union column t).
struct WinRow {
    int64_t it0, it1, vbase;
    int l, s;
};

// Loads the next round of a window row's items for the window [w0, w1):
// lane i takes item q0+i and the part of row k of B inside the window
// (clip false: the caller knows every row of B reached lies inside).  With
// cursors (cvalid: left by the window before, which ended at w0), item
// t < kWinCurMax of the row starts at cpos[t], the first position of its row
// of B at or after w0, whose column cnext[t] tells without any load whether
// the item reaches this window at all; once an item is done with the window
// both move on to w1.
template <bool NUM, bool CL>
__device__ __forceinline__ int load_round_win(const SpArgs &a, const WinRow &r, int64_t &q0, int &off0,
                                              ItemRec *items, uint64_t *sbits, int w0, int w1, bool clip = true,
                                              int32_t *cpos = nullptr, int32_t *cnext = nullptr, bool cvalid = false)
{
    const int lane = (int)__lane_id();
    sbits[lane] = 0ull;
    const int64_t q = q0 + lane;
    uint32_t lo = 0, hi = 0;
    double a1 = 0.0;
    bool upd = false;
    int32_t npos = 0, nnext = 0;
    if (q < r.it1 && (!CL || ((a.cl_mask[q] >> r.l) & 1u))) {
        const int64_t t = q - r.it0;
        const bool cur = cpos && t < kWinCurMax;
        if (!(cur && cvalid && cnext[t] >= w1)) {
            const int k = CL ? a.cl_col[q] : a.a_col[q];
            lo = (uint32_t)a.b_rp[k];
            const uint32_t end = (uint32_t)a.b_rp[k + 1];
            hi = end;
            if (cur && cvalid) {
                lo = (uint32_t)cpos[t];
                hi = gallop_col(a.b_col, lo, end, w1);
            } else {
                if (clip && lo < hi && ld_col(a.b_col, lo) < w0) lo = lower_bound_col(a.b_col, lo + 1, hi, w0);
                if (clip && lo < hi && ld_col(a.b_col, hi - 1) >= w1) hi = lower_bound_col(a.b_col, lo, hi - 1, w1);
            }
            if (cur) {
                upd = true;
                npos = (int32_t)hi;
                nnext = hi < end ? ld_col(a.b_col, hi) : INT_MAX;
            }
            if (NUM) a1 = CL ? a.cl_val[r.vbase + (q - r.it0) * r.s + r.l] : a.a_val[q];
        }
    }
    const uint64_t ab = (uint64_t)__double_as_longlong(a1);
    bool fin;
    const int E = flatten_round(r.it1, q0, off0, items, sbits, lo, (int)(hi - lo), (uint32_t)ab, (uint32_t)(ab >> 32),
                                nullptr, &fin);
    if (upd && fin) {
        const int64_t t = q - r.it0;
        cpos[t] = npos;
        cnext[t] = nnext;
    }
    return E;
}

// Column range of chunk c of nch equal chunks of the output columns [0, ncols).
__device__ __forceinline__ void win_chunk(int64_t ncols, int nch, int c, int *lo, int *hi)
{
    const int64_t cw = (ncols + nch - 1) / nch;
    *lo = (int)min<int64_t>(ncols, c * cw);
    *hi = (int)min<int64_t>(ncols, (c + 1) * cw);
}

// (row, chunk) pairs of a window launch per unit of the bin: a CSR row, or
// each member row of a cluster, gets win_nchunks(the unit's products)
// chunks in the symbolic launch; in the numeric launch only rows of more
// than kWinCurMax items are split so (the chunks of a row share its work out
// between workgroups, but each walks all of the row's items), the others
// are one task each.
// base[i] = pairs of the bin's i-th unit, base[count] = 0; an exclusive scan
// then gives each unit's first pair.
template <bool SYM, bool CL>
__global__ void __launch_bounds__(256) k_win_prep(SpArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > a.count) return;
    if (i == a.count) {
        a.win_base[i] = 0;
        return;
    }
    const int u = a.order[a.bin_begin + i];
    const int s = CL ? (int)(a.cl_row_ptr[u + 1] - a.cl_row_ptr[u]) : 1;
    const int64_t m = CL ? a.cl_col_ptr[u + 1] - a.cl_col_ptr[u] : a.a_rp[u + 1] - a.a_rp[u];
    const bool split = SYM || (a.ucount[u] == INT32_MAX && m > kWinCurMax);
    a.win_base[i] = (int64_t)s * (split ? win_nchunks(a.probes[u], a.win_log2) : 1);
}

// The (row, chunk) pair i of a window launch: p = the largest position with
// base[p] <= i (base strictly increasing over [0, count]), by a 64-way search
// of the whole wavefront.
__device__ __forceinline__ int64_t win_find(const int64_t *base, int64_t count, int64_t i)
{
    const int lane = (int)__lane_id();
    int64_t lo = 0, hi = count;  // answer in [lo, hi)
    while (hi - lo > 64) {
        const int64_t step = (hi - lo + 63) / 64;
        const int64_t x = lo + lane * step;
        const uint64_t b = __ballot(x < hi && base[x] <= i);
        const int L = 63 - __clzll((long long)b);  // lane 0 always qualifies
        lo += L * step;
        hi = min(hi, lo + step);
    }
    const int64_t x = lo + lane;
    const uint64_t b = __ballot(x < hi && base[x] <= i);
    return lo + (63 - __clzll((long long)b));
}

// Pair i of a window launch resolved: its unit, window row, output row and
// chunk c of nch (wave-uniform).
struct WinPair {
    int u, c, nch;
    int64_t row, first;  // first: the unit's first pair in this launch
    WinRow r;
};

template <bool CL>
__device__ __forceinline__ WinPair win_pair(const SpArgs &a, int64_t i)
{
    WinPair w;
    const int64_t p = (int64_t)uniform64((uint64_t)win_find(a.win_base, a.count, i));
    const int64_t b0 = (int64_t)uniform64((uint64_t)a.win_base[p]);
    const int64_t np = (int64_t)uniform64((uint64_t)a.win_base[p + 1]) - b0;
    w.u = uniform(a.order[a.bin_begin + p]);
    w.first = b0;
    const UnitView v = unit_view<CL>(a, w.u);
    w.nch = (int)(np / v.s);
    const int loc = (int)(i - b0);
    const int l = loc / w.nch;
    w.c = loc - l * w.nch;
    w.r.it0 = v.it0;
    w.r.it1 = v.it1;
    w.r.vbase = v.vbase;
    w.r.l = l;
    w.r.s = v.s;
    w.row = CL ? (int64_t)uniform(a.perm[v.pos0 + l]) : (int64_t)w.u;
    return w;
}

// Symbolic phase of the units too long for shared-memory tables: their
// member rows' output columns are counted in a bitmap instead of a table,
// one workgroup of kSymBmWaves wavefronts per unit (persistent over the bin),
// member rows one after another.  A row's column range [lo, hi] (the first
// and last columns of the rows of B its items reach) is taken in segments of
// 2^kBmLog2Bits columns.  When the range fits one segment (no row of B needs
// clipping) the row's flattened product list is cut into kSymBmWaves equal
// parts, one per wavefront (a few items carry most of the products of a
// power-law row, so items alone would share the work out badly); otherwise
// the wavefronts take the items 64 at a time from a shared counter.  Each
// product sets one bit by an atomic OR that returns nothing (ORs commute, so
// how the work is shared out does not change the bitmap).  The bits are then
// counted per column chunk of the numeric phase -- chunk_cnt[first + l*nch +
// c] for member l, chunk c, first the unit's first pair -- and the row's
// total is added to its count (zeroed by the binning kernel).
constexpr int kBmLog2Bits = 20;  // columns per segment: a 128 KiB bitmap
constexpr int kBmWords = 1 << (kBmLog2Bits - 5);
constexpr int kBmWaveBytes = 16 * 64 + 8 * kRoundPasses;  // a wavefront's item records and start bits

struct BmLayout {
    int bm, ccnt, red, psum, next, waves, bytes;
    __host__ __device__ BmLayout()
    {
        bm = 0;
        ccnt = 4 * kBmWords;             // kWinChunksMax chunk counters
        red = ccnt + 4 * kWinChunksMax;  // per-wavefront partial lo/hi
        psum = red + 8 * kSymBmWaves;    // per-wavefront partial product counts
        next = psum + 8 * kSymBmWaves;   // the next item group to take
        waves = align16(next + 4);
        bytes = waves + kSymBmWaves * kBmWaveBytes;
    }
};

int64_t sym_bm_bytes() { return BmLayout().bytes; }

// Item and offset holding product X of member row l's flattened product
// list (items without bit l count no products); (it1, 0) if X is past the end.
// Called by a whole wavefront.
template <bool CL>
__device__ __forceinline__ void bm_locate(const SpArgs &a, const UnitView &v, int l, int64_t X, int64_t &q0,
                                          int &off0)
{
    const int lane = (int)__lane_id();
    int64_t before = 0;  // products of the items before this group
    for (int64_t g = v.it0; g < v.it1; g += 64) {
        const int64_t q = g + lane;
        int len = 0;
        if (q < v.it1 && (!CL || ((a.cl_mask[q] >> l) & 1u))) {
            const int k = CL ? a.cl_col[q] : a.a_col[q];
            len = (int)(a.b_rp[k + 1] - a.b_rp[k]);
        }
        const int incl = wave_incl_scan(len);
        const uint64_t past = __ballot(before + incl > X);
        if (past) {
            const int L = __ffsll((unsigned long long)past) - 1;
            q0 = g + L;
            off0 = (int)(X - before - (__shfl(incl, L) - __shfl(len, L)));
            return;
        }
        before += __shfl(incl, 63);
    }
    q0 = v.it1;
    off0 = 0;
}

// A member row's column range [lo, hi] (the first and last columns of the
// rows of B its items reach) and product count, reduced over the workgroup
// (lo > hi for a row without products), over a workgroup of W wavefronts.
// Contains a barrier.
template <bool CL, int W>
__device__ __forceinline__ void bm_range(const SpArgs &a, const UnitView &v, int l, int *red, int64_t *psum, int &lo,
                                         int &hi, int64_t &np)
{
    constexpr int NT = 64 * W;
    const int wave = (int)(threadIdx.x >> 6), lane = (int)__lane_id();
    lo = INT_MAX;
    hi = -1;
    np = 0;
    for (int64_t q = v.it0 + threadIdx.x; q < v.it1; q += NT) {
        if (CL && !((a.cl_mask[q] >> l) & 1u)) continue;
        const int k = CL ? a.cl_col[q] : a.a_col[q];
        const int64_t b0 = a.b_rp[k], b1 = a.b_rp[k + 1];
        if (b1 > b0) {
            lo = min(lo, ld_col(a.b_col, (uint32_t)b0));
            hi = max(hi, ld_col(a.b_col, (uint32_t)(b1 - 1)));
            np += b1 - b0;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o));
        hi = max(hi, __shfl_xor(hi, o));
        np += __shfl_xor(np, o);
    }
    if (lane == 0) {
        red[wave] = lo;
        red[W + wave] = hi;
        psum[wave] = np;
    }
    __syncthreads();
    np = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        lo = min(lo, red[w]);
        hi = max(hi, red[W + w]);
        np += psum[w];
    }
    lo = uniform(lo);
    hi = uniform(hi);
    np = (int64_t)uniform64((uint64_t)np);
}

// Sets the bits of member row l's output columns inside the segment [w0, w1)
// (bit x of bm: column w0 + x), clearing the segment's words first.  clip
// false: the row's np products are cut into W equal parts, one per
// wavefront, and those outside the segment are passed over (none when the
// segment holds the row's whole range); clip: the wavefronts take the items
// 64 at a time from *next and find each item's part inside the segment by
// binary search.  A workgroup of W wavefronts; starts and ends with a barrier.
template <bool CL, int W>
__device__ __forceinline__ void bm_fill(const SpArgs &a, const UnitView &v, int l, int64_t np, int w0, int w1,
                                        bool clip, uint32_t *bm, int *next, ItemRec *items, uint64_t *sbits)
{
    constexpr int kR = 8, NT = 64 * W;
    const int wave = (int)(threadIdx.x >> 6), lane = (int)__lane_id();
    const uint64_t le = lanemask_le(lane);
    const int nw = (w1 - w0 + 31) >> 5;
    const int m = (int)(v.it1 - v.it0);
    for (int x = (int)threadIdx.x; x < ((nw + 3) >> 2); x += NT) ((uint4 *)bm)[x] = make_uint4(0u, 0u, 0u, 0u);
    if (threadIdx.x == 0) *next = 0;
    __syncthreads();
    int64_t x0 = 0, x1 = INT64_MAX;
    if (!clip) {
        x0 = np * wave / W;
        x1 = np * (wave + 1) / W;
    }
    for (;;) {
        int64_t q0;
        int off0 = 0;
        WinRow r{v.it0, v.it1, v.vbase, l, v.s};
        if (clip) {
            int g = 0;
            if (lane == 0) g = atomicAdd(next, 64);
            g = uniform(__shfl(g, 0));
            if (g >= m) break;
            r.it0 = v.it0 + g;
            r.it1 = min(v.it1, v.it0 + g + 64);
            q0 = r.it0;
        } else {
            if (x0 >= x1) break;
            bm_locate<CL>(a, v, l, x0, q0, off0);
            q0 = (int64_t)uniform64((uint64_t)q0);
            off0 = uniform(off0);
        }
        int64_t rem = x1 - x0;
        while (q0 < r.it1 && rem > 0) {
            const int E =
                (int)min<int64_t>(load_round_win<false, CL>(a, r, q0, off0, items, sbits, w0, w1, clip), rem);
            rem -= E;
            const int npass = (E + 63) >> 6;
            int cum = 0;
            for (int p = 0; p < npass; p += kR) {
                Pass<false, false> d[kR];
#pragma unroll
                for (int rr = 0; rr < kR; ++rr) {
                    if (p + rr < npass) {
                        const uint64_t w = uniform64(sbits[p + rr]);
                        d[rr] = fetch_pass<false, false>(a, items, w, cum, ((p + rr) << 6) + lane, E, le);
                        cum += __popcll(w);
                    } else {
                        d[rr].j = kDummyKey;
                    }
                }
#pragma unroll
                for (int rr = 0; rr < kR; ++rr) {
                    const uint32_t x = (uint32_t)(d[rr].j - w0);
                    if (d[rr].j != kDummyKey && x < (uint32_t)(w1 - w0)) atomicOr(&bm[x >> 5], 1u << (x & 31u));
                }
            }
        }
        if (!clip) break;
    }
    __syncthreads();
}

template <bool CL>
__global__ void __launch_bounds__(64 * kSymBmWaves) k_sym_bm(SpArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NT = 64 * kSymBmWaves;
    const BmLayout L;
    uint32_t *bm = (uint32_t *)(smem + L.bm);
    int *ccnt = (int *)(smem + L.ccnt);
    int *red = (int *)(smem + L.red);
    int64_t *psum = (int64_t *)(smem + L.psum);
    int *next = (int *)(smem + L.next);
    const int wave = (int)(threadIdx.x >> 6), lane = (int)__lane_id();
    ItemRec *items = (ItemRec *)(smem + L.waves + wave * kBmWaveBytes);
    uint64_t *sbits = (uint64_t *)(smem + L.waves + wave * kBmWaveBytes + 16 * 64);
    for (int64_t i = xcd_block(); i < a.count; i += gridDim.x) {
        const int u = uniform(a.order[a.bin_begin + i]);
        const UnitView v = unit_view<CL>(a, u);
        const int64_t first = (int64_t)uniform64((uint64_t)a.win_base[i]);
        const int nch = (int)(((int64_t)uniform64((uint64_t)a.win_base[i + 1]) - first) / v.s);
        const bool room = first + (int64_t)v.s * nch <= a.win_cap;
        const int64_t cw = (a.ncols + nch - 1) / nch;  // chunk width (win_chunk)
        for (int l = 0; l < v.s; ++l) {
            for (int c = (int)threadIdx.x; c < nch; c += NT) ccnt[c] = 0;
            int lo, hi;
            int64_t np;
            bm_range<CL, kSymBmWaves>(a, v, l, red, psum, lo, hi, np);
            for (int64_t g0 = lo; g0 <= (int64_t)hi; g0 += (int64_t)1 << kBmLog2Bits) {
                const int w0 = (int)g0;
                const int w1 = (int)min<int64_t>((int64_t)hi + 1, g0 + ((int64_t)1 << kBmLog2Bits));
                const int nw = (w1 - w0 + 31) >> 5;
                bm_fill<CL, kSymBmWaves>(a, v, l, np, w0, w1, g0 > lo || w1 <= hi, bm, next, items, sbits);
                // count the bits per chunk: a wavefront's 64 words usually lie in one chunk
                for (int x0 = wave * 64; x0 < nw; x0 += NT) {
                    const int wd = x0 + lane;
                    const uint32_t bits = wd < nw ? bm[wd] : 0u;
                    const int64_t col0 = g0 + 32 * (int64_t)wd;
                    const int c0 = (int)(col0 / cw);
                    const int c1 = (int)(min<int64_t>(col0 + 31, a.ncols - 1) / cw);
                    const int cf = uniform(__shfl(c0, 0));
                    if (__ballot(wd < nw && (c0 != cf || c1 != cf)) == 0ull) {
                        int n = __popc(bits);
                        for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
                        if (lane == 0 && n) atomicAdd(&ccnt[cf], n);
                    } else {
                        uint32_t y = bits;
                        while (y) {
                            const int c = (int)((col0 + (__ffs((int)y) - 1)) / cw);
                            const int64_t nb = (int64_t)(c + 1) * cw - col0;  // this word's bits before chunk c+1
                            const uint32_t mk = nb >= 32 ? 0xffffffffu : ((1u << nb) - 1u);
                            atomicAdd(&ccnt[c], __popc(y & mk));
                            y &= ~mk;
                        }
                    }
                }
                __syncthreads();
            }
            int64_t tot = 0;
            for (int c = (int)threadIdx.x; c < nch; c += NT) {
                const int n = ccnt[c];
                tot += n;
                if (room) a.chunk_cnt[first + (int64_t)l * nch + c] = n;
            }
            for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
            if (lane == 0 && tot) {
                const int64_t row = CL ? (int64_t)a.perm[v.pos0 + l] : (int64_t)u;
                atomicAdd((unsigned long long *)&a.c_rp[row], (unsigned long long)tot);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (!room) atomicOr(a.err, kErrWindows);
            a.ucount[u] = INT32_MAX;
            a.sym_base[u] = first;
        }
    }
}

// Numeric phase of the units too long for shared-memory tables: one
// workgroup of kNumBmWaves wavefronts per member row, or, for rows of many
// items, per (member row, column chunk) of the symbolic phase (the chunk's
// entries follow those of the chunks before it).  The
// task's columns are taken in segments of 2^kNbLog2Bits columns; for
// each, the row's output columns are first set in a bitmap (as in the
// symbolic phase), whose keys are then shared out between the wavefronts in
// equal parts of whole words.  A wavefront takes its words in windows of at
// most kNbK keys and kNbSpan words: a key's slot in the window's values is its
// rank, the keys before it in the window (a per-word prefix plus a popcount),
// so there is no probing, no table that can fill and no sort -- the values
// come out in column order, and the columns are read off the bitmap.  The
// window's products are walked in the usual way (items in ascending k,
// 64-product passes, each item's entries applied in turn), with the items'
// positions in B carried from one window to the next.
constexpr int kNbLog2Bits = 19;  // columns per segment: a 64 KiB bitmap
constexpr int kNbWords = 1 << (kNbLog2Bits - 5);
constexpr int kNbK = 1024;       // keys per window at most (a value each)
constexpr int kNbSpan = 512;     // words per window at most
constexpr int kNbValBytes = (8 * (kNbK + 1) + 15) & ~15;
constexpr int kNbPreBytes = (2 * (kNbSpan + 1) + 15) & ~15;
constexpr int kNbWaveBytes = kNbValBytes + kNbPreBytes + 16 * 64 + 8 * kRoundPasses;

struct NbLayout {
    int bm, tpre, red, psum, next, waves, bytes;
    __host__ __device__ NbLayout()
    {
        bm = 0;
        tpre = 4 * kNbWords;                   // per-thread key prefix [64 * kNumBmWaves]
        red = tpre + 4 * 64 * kNumBmWaves;     // per-wavefront partial lo/hi, then key sums
        psum = red + 8 * kNumBmWaves;          // per-wavefront partial product counts
        next = psum + 8 * kNumBmWaves;         // the next item group to take
        waves = align16(next + 4);
        bytes = waves + kNumBmWaves * kNbWaveBytes;
    }
};

int64_t num_bm_bytes() { return NbLayout().bytes; }

// The smallest word W in [0, nw] whose key prefix P(W) (keys of the segment
// before word W) is at least x, and P(W).  tpre[t]: keys before thread t's
// words [t*wpt, (t+1)*wpt); total: keys of the segment.  Whole wavefront.
__device__ __forceinline__ void nb_split(const uint32_t *bm, const int *tpre, int wpt, int nw, int total, int x,
                                         int &W, int &PW)
{
    constexpr int NT = 64 * kNumBmWaves;
    const int lane = (int)__lane_id();
    int below = 0;  // threads whose words start below the prefix x
    for (int t = lane; t < NT; t += 64) below += tpre[t] < x;
    for (int o = 32; o > 0; o >>= 1) below += __shfl_xor(below, o);
    below = uniform(below);
    if (below == 0) {
        W = 0;
        PW = 0;
        return;
    }
    const int T = below - 1;
    const int wd = T * wpt + lane;
    const bool valid = lane < wpt && wd < nw;
    const int pc = valid ? __popc(bm[wd]) : 0;
    const int P = tpre[T] + wave_incl_scan(pc) - pc;
    const uint64_t q = __ballot(valid && P >= x);
    if (q) {
        const int L = __ffsll((unsigned long long)q) - 1;
        W = T * wpt + L;
        PW = uniform(__shfl(P, L));
    } else {
        W = min(nw, (T + 1) * wpt);
        PW = T + 1 < NT ? tpre[T + 1] : total;
    }
}

template <bool CL>
__global__ void __launch_bounds__(64 * kNumBmWaves) k_num_bm(SpArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NT = 64 * kNumBmWaves, kR = 4;
    const NbLayout L;
    uint32_t *bm = (uint32_t *)(smem + L.bm);
    int *tpre = (int *)(smem + L.tpre);
    int *red = (int *)(smem + L.red);
    int64_t *psum = (int64_t *)(smem + L.psum);
    int *next = (int *)(smem + L.next);
    const int wave = (int)(threadIdx.x >> 6), lane = (int)__lane_id();
    unsigned char *wb = smem + L.waves + wave * kNbWaveBytes;
    double *vals = (double *)wb;
    uint16_t *lpre = (uint16_t *)(wb + kNbValBytes);
    ItemRec *items = (ItemRec *)(wb + kNbValBytes + kNbPreBytes);
    uint64_t *sbits = (uint64_t *)(wb + kNbValBytes + kNbPreBytes + 16 * 64);
    const uint64_t le = lanemask_le(lane);
    // this wavefront's carried positions in B and the columns there
    int32_t *const cpos = a.win_cur ? a.win_cur + ((size_t)blockIdx.x * kNumBmWaves + wave) * (2 * kWinCurMax) : nullptr;
    int32_t *const cnext = cpos ? cpos + kWinCurMax : nullptr;
    const int64_t pairs = (int64_t)uniform64((uint64_t)a.win_base[a.count]);
    for (int64_t i = xcd_block(); i < pairs; i += gridDim.x) {
        const WinPair w = win_pair<CL>(a, i);
        if (w.u < a.unit_lo || w.u >= a.unit_hi) continue;
        const int u = w.u, l = w.r.l;
        const UnitView v = unit_view<CL>(a, u);
        {
            const int64_t row = w.row;
            // this task's columns [clo, chi), its first entry in C and its entries
            int64_t off = (int64_t)uniform64((uint64_t)a.c_rp[row]) - a.out_base, cnt;
            int clo, chi;
            if (w.nch > 1) {
                win_chunk(a.ncols, w.nch, w.c, &clo, &chi);
                const int64_t cb = (int64_t)uniform64((uint64_t)a.sym_base[u]) + (int64_t)l * w.nch;
                if (cb < 0 || cb + w.nch > a.win_cap) {
                    if (threadIdx.x == 0) atomicOr(a.err, kErrWindows);
                    continue;
                }
                const int32_t *cc = a.chunk_cnt + cb;
                int64_t before = 0;
                for (int x = lane; x < w.c; x += 64) before += cc[x];
                for (int o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o);
                off += (int64_t)uniform64((uint64_t)before);
                cnt = uniform(cc[w.c]);
            } else {
                clo = 0;
                chi = (int)a.ncols;
                cnt = (int64_t)uniform64((uint64_t)a.c_rp[row + 1]) - (off + a.out_base);
            }
            if (cnt <= 0) continue;
            if (off < 0 || off + cnt > a.cap) {
                if (threadIdx.x == 0) atomicOr(a.err, kErrCapacity);
                continue;
            }
            int rlo, rhi;
            int64_t np;
            bm_range<CL, kNumBmWaves>(a, v, l, red, psum, rlo, rhi, np);
            // the row's columns inside the task's; one segment over all of the
            // row's products needs no clipping
            const int lo = max(rlo, clo), hi = min(rhi, chi - 1);
            int64_t done = 0;  // keys of the segments before
            for (int64_t g0 = lo; g0 <= (int64_t)hi; g0 += (int64_t)1 << kNbLog2Bits) {
                const int w0 = (int)g0;
                const int w1 = (int)min<int64_t>((int64_t)hi + 1, g0 + ((int64_t)1 << kNbLog2Bits));
                const int nw = (w1 - w0 + 31) >> 5;
                // a chunk of a row searches its items' parts; a whole row walks
                // all of its products once per segment
                bm_fill<CL, kNumBmWaves>(a, v, l, np, w0, w1, w.nch > 1 && (w0 > rlo || w1 <= rhi), bm, next, items, sbits);
                // keys per thread's words, and their exclusive prefix over the workgroup
                const int wpt = (nw + NT - 1) / NT;
                int mine = 0;
                for (int x = (int)threadIdx.x * wpt; x < min(nw, ((int)threadIdx.x + 1) * wpt); ++x) mine += __popc(bm[x]);
                const int incl = wave_incl_scan(mine);
                if (lane == 63) red[wave] = incl;
                __syncthreads();
                int before = 0, total = 0;
#pragma unroll
                for (int w = 0; w < kNumBmWaves; ++w) {
                    const int rw = red[w];
                    before += w < wave ? rw : 0;
                    total += rw;
                }
                total = uniform(total);
                tpre[threadIdx.x] = before + incl - mine;
                __syncthreads();
                if (done + total > cnt) {  // more keys than the symbolic phase counted
                    if (threadIdx.x == 0) atomicOr(a.err, kErrCount);
                    done = cnt + 1;
                    break;
                }
                // this wavefront's words [wa, we) and the keys before wa
                int wa, pa, we, pe;
                nb_split(bm, tpre, wpt, nw, total, (int)((int64_t)total * wave / kNumBmWaves), wa, pa);
                if (wave + 1 < kNumBmWaves) {
                    nb_split(bm, tpre, wpt, nw, total, (int)((int64_t)total * (wave + 1) / kNumBmWaves), we, pe);
                } else {
                    we = nw;
                    pe = total;
                }
                const WinRow r{v.it0, v.it1, v.vbase, l, v.s};
                bool cvalid = false;  // the first window searches
                int pos = pa;
                for (int a0 = wa; a0 < we;) {
                    // the window: words [a0, b0) holding nk <= kNbK keys, their prefix in lpre
                    int nk = 0, b0 = a0;
                    for (;;) {
                        const int wd = b0 + lane;
                        const bool valid = wd < we && wd - a0 < kNbSpan;
                        const int pc = valid ? __popc(bm[wd]) : 0;
                        const int inc = wave_incl_scan(pc);
                        const bool fits = valid && nk + inc <= kNbK;
                        if (fits) lpre[wd - a0] = (uint16_t)(nk + inc - pc);
                        const int nf = __popcll(__ballot(fits));
                        if (nf == 0) break;
                        nk += __shfl(inc, nf - 1);
                        b0 += nf;
                        if (nf < 64) break;
                    }
                    nk = uniform(nk);
                    b0 = uniform(b0);
                    if (lane == 0) lpre[b0 - a0] = (uint16_t)nk;
                    for (int x = lane; x < nk; x += 64) vals[x] = 0.0;
                    if (lane == 0) vals[kNbK] = 0.0;
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    const int c0 = w0 + 32 * a0, c1 = min(w1, w0 + 32 * b0);
                    auto apply = [&](const Pass<false, true> &d, int h, int tf, int tl) {
                        for (int tt = tf; tt <= tl; ++tt) {
                            if (d.t != tt) continue;
                            const double av = *(const double *)&items[tt].x;
                            vals[h] = __fma_rn(av, d.b, vals[h]);
                        }
                    };
                    int64_t q0 = v.it0;
                    int off0 = 0;
                    while (q0 < v.it1) {
                        const int E =
                            load_round_win<true, CL>(a, r, q0, off0, items, sbits, c0, c1, true, cpos, cnext, cvalid);
                        const int npass = (E + 63) >> 6;
                        int cum = 0;
                        for (int p = 0; p < npass; p += kR) {
                            Pass<false, true> d[kR];
                            int tf[kR], tl[kR], h[kR];
#pragma unroll
                            for (int rr = 0; rr < kR; ++rr) {
                                if (p + rr < npass) {
                                    const uint64_t w = uniform64(sbits[p + rr]);
                                    const int last = min(63, E - 1 - ((p + rr) << 6));
                                    tf[rr] = cum + (int)(w & 1ull) - 1;
                                    tl[rr] = cum + __popcll(w & lanemask_le(last)) - 1;
                                    d[rr] = fetch_pass<false, true>(a, items, w, cum, ((p + rr) << 6) + lane, E, le);
                                    cum += __popcll(w);
                                }
                            }
#pragma unroll
                            for (int rr = 0; rr < kR; ++rr) {
                                if (p + rr < npass) {
                                    h[rr] = kNbK;
                                    if (d[rr].j != kDummyKey) {
                                        const uint32_t x = (uint32_t)(d[rr].j - c0);
                                        const int wd = (int)(x >> 5);
                                        h[rr] = (int)lpre[wd] + __popc(bm[a0 + wd] & ((1u << (x & 31u)) - 1u));
                                    }
                                    apply(d[rr], h[rr], tf[rr], tl[rr]);
                                }
                            }
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    // the window's entries: values in rank order, columns off the bitmap
                    const int64_t base = off + done + pos;
                    for (int x = lane; x < nk; x += 64) a.c_val[base + x] = vals[x];
                    for (int t = lane; t < b0 - a0; t += 64) {
                        uint32_t bits = bm[a0 + t];
                        int pr = lpre[t];
                        while (bits) {
                            a.c_col[base + pr] = c0 + 32 * t + (__ffs((int)bits) - 1);
                            ++pr;
                            bits &= bits - 1u;
                        }
                    }
                    cvalid = true;
                    pos += nk;
                    a0 = b0;
                }
                if (lane == 0 && pos != pe) atomicOr(a.err, kErrCount);  // windows did not tile the share
                __syncthreads();
                done += total;
            }
            if (threadIdx.x == 0 && done != cnt) atomicOr(a.err, kErrCount);
            __syncthreads();
        }
    }
}

hipError_t launch_win_prep(bool sym, bool cluster, const SpArgs &a, hipStream_t s)
{
    const unsigned blocks = (unsigned)((a.count + 1 + 255) / 256);
    if (sym && cluster) hipLaunchKernelGGL((k_win_prep<true, true>), dim3(blocks), dim3(256), 0, s, a);
    else if (sym) hipLaunchKernelGGL((k_win_prep<true, false>), dim3(blocks), dim3(256), 0, s, a);
    else if (cluster) hipLaunchKernelGGL((k_win_prep<false, true>), dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_win_prep<false, false>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sym_bm(bool cluster, const SpArgs &a, int blocks, hipStream_t s)
{
    const dim3 g(blocks), t(64 * kSymBmWaves);
    if (cluster) hipLaunchKernelGGL(k_sym_bm<true>, g, t, (size_t)sym_bm_bytes(), s, a);
    else hipLaunchKernelGGL(k_sym_bm<false>, g, t, (size_t)sym_bm_bytes(), s, a);
    return hipGetLastError();
}

hipError_t launch_num_bm(bool cluster, const SpArgs &a, int blocks, hipStream_t s)
{
    const dim3 g(blocks), t(64 * kNumBmWaves);
    if (cluster) hipLaunchKernelGGL(k_num_bm<true>, g, t, (size_t)num_bm_bytes(), s, a);
    else hipLaunchKernelGGL(k_num_bm<false>, g, t, (size_t)num_bm_bytes(), s, a);
    return hipGetLastError();
}

// ================================================================ kernels
// A bin's units: one per wavefront with the grid sized to the bin, or, for a
// batch (BATCH), a persistent grid whose wavefronts each take one contiguous
// slice of the bin, whose size and start are read from device memory; each
// unit is then resolved to its product first.
template <int S, bool CL, bool BATCH, bool NUM, bool PRED = false, bool HASHED = false>
__device__ __forceinline__ void run_bin(const SpArgs &a0)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int wpb = blockDim.x >> 6;
    const int wib = uniform((int)(threadIdx.x >> 6));
    unsigned char *base = smem + (size_t)wib * a0.group_bytes;
    const int64_t lw = xcd_block() * wpb + wib;
    if (!BATCH) {
        if (lw >= a0.count) return;
        const int u = uniform(a0.order[a0.bin_begin + lw]);
        if (NUM) num_unit<S, CL, PRED, true, HASHED>(a0, u, base);
        else sym_unit<S, CL>(a0, u, base);
        return;
    }
    const int64_t count = a0.dcount[a0.bin], begin = a0.dbegin[a0.bin];
    const int64_t W = (int64_t)gridDim.x * wpb;
    const int64_t e = begin + (lw + 1) * count / W;
    for (int64_t i = begin + lw * count / W; i < e; ++i) {
        SpArgs a = a0;
        const int u = batch_resolve(a, a0.order[i]);
        if (NUM) num_unit<S, CL, false, false, HASHED>(a, u, base);
        else sym_unit<S, CL>(a, u, base);
    }
}

template <int S, bool CL, bool BATCH>
__global__ void __launch_bounds__(256) k_sym(SpArgs a) { run_bin<S, CL, BATCH, false>(a); }

// Wavefronts per SIMD the numeric kernels must allow (their register budget):
// CSR rows 8 (64 vector registers), two-row clusters 7 (72); in batches,
// whose unit arguments are resolved per unit, 6 (80).  Large (hashed) tables
// leave room for a few wavefronts per compute unit only, so their kernels
// get 4 (128 registers).
template <int S, bool BATCH, bool HASHED>
struct NumOcc {
    static constexpr int W = HASHED ? 4 : S == 1 && !BATCH ? 8 : S <= 2 ? (BATCH ? 6 : 7) : 1;
};

template <int S, bool CL, bool BATCH, bool HASHED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NumOcc<S, BATCH, HASHED>::W)))
k_num(SpArgs a) { run_bin<S, CL, BATCH, true, false, HASHED>(a); }

template <bool HASHED>
__global__ void __launch_bounds__(256) k_num_pred(SpArgs a) { run_bin<1, false, false, true, true, HASHED>(a); }

hipError_t launch_num_pred(const SpArgs &a, int blocks, int threads, size_t lds, hipStream_t s)
{
    if (hashed_table(a.T)) hipLaunchKernelGGL(k_num_pred<true>, dim3(blocks), dim3(threads), lds, s, a);
    else hipLaunchKernelGGL(k_num_pred<false>, dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// ================================================================ launchers
template <int S, bool CL>
static hipError_t go_sym(bool batch, const SpArgs &a, int blocks, int threads, size_t lds, hipStream_t s)
{
    if (batch) hipLaunchKernelGGL((k_sym<S, CL, true>), dim3(blocks), dim3(threads), lds, s, a);
    else hipLaunchKernelGGL((k_sym<S, CL, false>), dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <int S, bool CL>
static hipError_t go_num(bool batch, const SpArgs &a, int blocks, int threads, size_t lds, hipStream_t s)
{
    const bool h = hashed_table(a.T);
    if (batch && h) hipLaunchKernelGGL((k_num<S, CL, true, true>), dim3(blocks), dim3(threads), lds, s, a);
    else if (batch) hipLaunchKernelGGL((k_num<S, CL, true, false>), dim3(blocks), dim3(threads), lds, s, a);
    else if (h) hipLaunchKernelGGL((k_num<S, CL, false, true>), dim3(blocks), dim3(threads), lds, s, a);
    else hipLaunchKernelGGL((k_num<S, CL, false, false>), dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_sym(int sclass, bool cluster, bool batch, const SpArgs &a, int blocks, int threads, size_t lds,
                      hipStream_t s)
{
    if (!cluster) return go_sym<1, false>(batch, a, blocks, threads, lds, s);
    switch (sclass) {
    case 0: return go_sym<1, true>(batch, a, blocks, threads, lds, s);
    case 1: return go_sym<2, true>(batch, a, blocks, threads, lds, s);
    case 2: return go_sym<4, true>(batch, a, blocks, threads, lds, s);
    case 3: return go_sym<8, true>(batch, a, blocks, threads, lds, s);
    default: return go_sym<16, true>(batch, a, blocks, threads, lds, s);
    }
}

hipError_t launch_num(int sclass, bool cluster, bool batch, const SpArgs &a, int blocks, int threads, size_t lds,
                      hipStream_t s)
{
    if (!cluster) return go_num<1, false>(batch, a, blocks, threads, lds, s);
    switch (sclass) {
    case 0: return go_num<1, true>(batch, a, blocks, threads, lds, s);
    case 1: return go_num<2, true>(batch, a, blocks, threads, lds, s);
    case 2: return go_num<4, true>(batch, a, blocks, threads, lds, s);
    case 3: return go_num<8, true>(batch, a, blocks, threads, lds, s);
    default: return go_num<16, true>(batch, a, blocks, threads, lds, s);
    }
}

}  // namespace hcsp
