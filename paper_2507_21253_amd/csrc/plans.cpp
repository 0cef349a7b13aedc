// Host-side cluster plans: fixed-length, variable-length (paper, Alg. 2) and
// hierarchical (paper, Alg. 3).  They read host copies of A's pattern and
// return a row order plus cluster boundaries; the device then builds the
// CSR_Cluster form from them.
//
// The candidate search of the hierarchical plan (SpGEMM_TopK over A A^T) is
// split over host threads; the merge loop that follows is sequential by
// nature (each merge changes later decisions).  Every comparison of
// similarities is exact: J = ov/un is compared by cross-multiplication.
#include <algorithm>
#include <cstring>
#include <new>
#include <queue>
#include <thread>
#include <vector>

#include "internal.h"

namespace hcsp {
namespace {

struct Sim {
    int64_t ov, un;  // similarity ov/un; an empty union reads as 0
};

inline int cmp_sim(Sim a, Sim b)
{
    if (a.un == 0) a = {0, 1};
    if (b.un == 0) b = {0, 1};
    const __int128 l = (__int128)a.ov * b.un, r = (__int128)b.ov * a.un;
    return (l > r) - (l < r);
}

inline int cmp_thr(Sim a, int64_t num, int64_t den) { return cmp_sim(a, Sim{num, den}); }

struct Pattern {
    // rows of A in plan order: position p holds original row row[p]
    const int64_t *rp;
    const int32_t *col;
    std::vector<int32_t> row;
    int64_t n, ncols;
    int64_t len(int64_t p) const { return rp[row[p] + 1] - rp[row[p]]; }
    const int32_t *cols(int64_t p) const { return col + rp[row[p]]; }
};

// A's rows copied in plan order (position p's columns contiguous), for the
// merge loop, whose pairs are near each other in that order.
struct PosPattern {
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    explicit PosPattern(const Pattern &P) : rp((size_t)P.n + 1, 0)
    {
        for (int64_t p = 0; p < P.n; ++p) rp[(size_t)p + 1] = rp[(size_t)p] + P.len(p);
        col.resize((size_t)rp[(size_t)P.n]);
        for (int64_t p = 0; p < P.n; ++p) std::copy(P.cols(p), P.cols(p) + P.len(p), col.begin() + rp[(size_t)p]);
    }
    int64_t len(int64_t p) const { return rp[(size_t)p + 1] - rp[(size_t)p]; }
    const int32_t *cols(int64_t p) const { return col.data() + rp[(size_t)p]; }
};

template <class Pat>
Sim jaccard(const Pat &P, int64_t i, int64_t j)
{
    const int32_t *a = P.cols(i), *b = P.cols(j);
    const int64_t na = P.len(i), nb = P.len(j);
    int64_t x = 0, y = 0, ov = 0;
    while (x < na && y < nb) {
        if (a[x] == b[y]) {
            ++ov;
            ++x;
            ++y;
        } else if (a[x] < b[y]) {
            ++x;
        } else {
            ++y;
        }
    }
    return Sim{ov, na + nb - ov};
}

int make_pattern(const hcsp_csr *A, const int32_t *perm_in, Pattern *P)
{
    if (!A || A->nrows < 0 || !A->row_ptr || (A->nnz > 0 && !A->col)) return fail(HCSP_E_INVALID, "bad host A");
    P->rp = A->row_ptr;
    P->col = A->col;
    P->n = A->nrows;
    P->ncols = A->ncols;
    try {
        P->row.resize((size_t)A->nrows);
    } catch (const std::bad_alloc &) {
        return fail(HCSP_E_NOMEM, "host allocation failed");
    }
    if (perm_in) {
        std::vector<uint8_t> seen((size_t)A->nrows, 0);
        for (int64_t p = 0; p < A->nrows; ++p) {
            const int32_t r = perm_in[p];
            if (r < 0 || r >= A->nrows || seen[r]) return fail(HCSP_E_INVALID, "perm_in is not a permutation");
            seen[r] = 1;
            P->row[p] = r;
        }
    } else {
        for (int64_t p = 0; p < A->nrows; ++p) P->row[p] = (int32_t)p;
    }
    return HCSP_OK;
}

struct Cand {
    Sim s;
    int32_t i, j;  // i < j
};

// heap order: larger similarity first, then smaller i, then smaller j
struct CandLess {
    bool operator()(const Cand &a, const Cand &b) const
    {
        const int c = cmp_sim(a.s, b.s);
        if (c) return c < 0;
        if (a.i != b.i) return a.i > b.i;
        return a.j > b.j;
    }
};

// Open-addressing set of unordered position pairs.
class PairSet {
  public:
    explicit PairSet(size_t expect)
    {
        size_t cap = 1024;
        while (cap < 2 * expect + 16) cap <<= 1;
        keys_.assign(cap, kNone);
    }
    bool insert(uint64_t k)
    {
        if (2 * (n_ + 1) > keys_.size()) grow();
        return put(keys_, k);
    }
    bool contains(uint64_t k) const
    {
        const size_t m = keys_.size() - 1;
        for (size_t h = mix(k) & m;; h = (h + 1) & m) {
            if (keys_[h] == k) return true;
            if (keys_[h] == kNone) return false;
        }
    }

  private:
    static constexpr uint64_t kNone = ~0ull;
    static uint64_t mix(uint64_t x)
    {
        x ^= x >> 31;
        x *= 0x7fb5d329728ea185ull;
        x ^= x >> 27;
        x *= 0x81dadef4bc2dd44dull;
        return x ^ (x >> 33);
    }
    bool put(std::vector<uint64_t> &t, uint64_t k)
    {
        const size_t m = t.size() - 1;
        for (size_t h = mix(k) & m;; h = (h + 1) & m) {
            if (t[h] == k) return false;
            if (t[h] == kNone) {
                t[h] = k;
                if (&t == &keys_) ++n_;
                return true;
            }
        }
    }
    void grow()
    {
        std::vector<uint64_t> old;
        old.swap(keys_);
        keys_.assign(old.size() * 2, kNone);
        n_ = 0;
        for (uint64_t k : old)
            if (k != kNone) put(keys_, k);
    }
    std::vector<uint64_t> keys_;
    size_t n_ = 0;
};

inline uint64_t pair_key(int32_t i, int32_t j) { return ((uint64_t)(uint32_t)i << 32) | (uint32_t)j; }

// Per-row top-k candidate partners: rows of a slice [lo, hi) of positions.
void topk_rows(const Pattern &P, const std::vector<int64_t> &tp, const std::vector<int32_t> &tr, int64_t num,
               int64_t den, int topk, int64_t lo, int64_t hi, std::vector<int32_t> &cnt, std::vector<int32_t> &nbr,
               std::vector<Sim> &nsim)
{
    std::vector<int32_t> ov((size_t)P.n, 0);
    std::vector<int32_t> touched;
    touched.reserve(1024);
    std::vector<Cand> best((size_t)topk);
    for (int64_t i = lo; i < hi; ++i) {
        touched.clear();
        const int32_t *c = P.cols(i);
        const int64_t li = P.len(i);
        for (int64_t q = 0; q < li; ++q) {
            const int32_t k = c[q];
            for (int64_t t = tp[k]; t < tp[k + 1]; ++t) {
                const int32_t j = tr[t];
                if (j == i) continue;
                if (ov[j]++ == 0) touched.push_back(j);
            }
        }
        int nb = 0;
        for (int32_t j : touched) {
            const Sim s{ov[j], li + P.len(j) - ov[j]};
            ov[j] = 0;
            if (cmp_thr(s, num, den) <= 0) continue;
            // keep the topk best by (similarity desc, j asc)
            int pos = nb;
            while (pos > 0) {
                const Cand &b = best[pos - 1];
                const int cmp = cmp_sim(s, b.s);
                if (cmp > 0 || (cmp == 0 && j < b.j)) --pos;
                else break;
            }
            if (pos >= topk) continue;
            const int last = nb < topk ? nb : topk - 1;
            for (int x = last; x > pos; --x) best[x] = best[x - 1];
            best[pos] = Cand{s, (int32_t)i, j};
            if (nb < topk) ++nb;
        }
        cnt[i] = nb;
        for (int x = 0; x < nb; ++x) {
            nbr[(size_t)i * topk + x] = best[x].j;
            nsim[(size_t)i * topk + x] = best[x].s;
        }
    }
}

int32_t uf_find(std::vector<int32_t> &parent, int32_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

int emit(const Pattern &P, const std::vector<int32_t> &parent, const std::vector<int32_t> &next, int32_t *perm_out,
         int64_t *cl_row_ptr, int64_t *ncl)
{
    int64_t c = 0, p = 0;
    cl_row_ptr[0] = 0;
    std::vector<int32_t> mem;
    for (int64_t r = 0; r < P.n; ++r) {
        if (parent[r] != r) continue;
        mem.clear();
        for (int32_t m = (int32_t)r; m >= 0; m = next[m]) mem.push_back(m);
        std::sort(mem.begin(), mem.end());
        for (int32_t m : mem) perm_out[p++] = P.row[m];
        cl_row_ptr[++c] = p;
    }
    *ncl = c;
    return HCSP_OK;
}

}  // namespace
}  // namespace hcsp

using namespace hcsp;

extern "C" {

int hcsp_plan_fixed(int64_t nrows, int32_t K, const int32_t *perm_in_h, int32_t *perm_out_h, int64_t *cl_row_ptr_h,
                    int64_t *ncl)
{
    clear_error();
    if (nrows < 0 || K < 1 || K > 16 || (nrows > 0 && !perm_out_h) || !cl_row_ptr_h || !ncl)
        return fail(HCSP_E_INVALID, "fixed plan: bad arguments (K must be 1..16)");
    int64_t c = 0;
    cl_row_ptr_h[0] = 0;
    for (int64_t p = 0; p < nrows; ++p) {
        perm_out_h[p] = perm_in_h ? perm_in_h[p] : (int32_t)p;
        if ((p + 1) % K == 0 || p + 1 == nrows) cl_row_ptr_h[++c] = p + 1;
    }
    *ncl = c;
    return HCSP_OK;
}

int hcsp_plan_variable(const hcsp_csr *A_h, hcsp_ratio jacc_th, int32_t max_cluster, const int32_t *perm_in_h,
                       int32_t *perm_out_h, int64_t *cl_row_ptr_h, int64_t *ncl)
{
    clear_error();
    if (jacc_th.den <= 0 || jacc_th.num < 0 || max_cluster < 1 || max_cluster > 16 || !cl_row_ptr_h || !ncl)
        return fail(HCSP_E_INVALID, "variable plan: bad arguments");
    Pattern P;
    int rc = make_pattern(A_h, perm_in_h, &P);
    if (rc) return rc;
    if (P.n > 0 && !perm_out_h) return fail(HCSP_E_INVALID, "null perm_out");
    cl_row_ptr_h[0] = 0;
    if (P.n == 0) {
        *ncl = 0;
        return HCSP_OK;
    }
    int64_t c = 0, rep = 0, size = 1;
    perm_out_h[0] = P.row[0];
    for (int64_t p = 1; p < P.n; ++p) {
        const Sim s = jaccard(P, rep, p);
        if (cmp_thr(s, jacc_th.num, jacc_th.den) < 0 || size == max_cluster) {
            cl_row_ptr_h[++c] = p;
            rep = p;
            size = 1;
        } else {
            ++size;
        }
        perm_out_h[p] = P.row[p];
    }
    cl_row_ptr_h[++c] = P.n;
    *ncl = c;
    return HCSP_OK;
}

}  // extern "C"

namespace hcsp {
namespace {

// The merge loop of Alg. 3 over per-position candidate lists (cnt[p]
// partners in nbr[p*topk ..] with similarities nsim[p*topk ..]): candidate
// pairs go into the heap once each, then pairs are popped best first and
// merged, lifted to their roots, rescored and pushed again.
int merge_phase(const Pattern &P, int64_t num, int64_t den, int32_t max_cluster, uint32_t sim_flags, int topk,
                const std::vector<int32_t> &cnt, const std::vector<int32_t> &nbr, const std::vector<Sim> &nsim,
                int32_t *perm_out_h, int64_t *cl_row_ptr_h, int64_t *ncl);

}  // namespace
}  // namespace hcsp

extern "C" {

int hcsp_plan_hierarchical(const hcsp_csr *A_h, hcsp_ratio jacc_th, int32_t max_cluster, uint32_t sim_flags,
                           int32_t nthreads, const int32_t *perm_in_h, int32_t *perm_out_h, int64_t *cl_row_ptr_h,
                           int64_t *ncl)
{
    clear_error();
    if (jacc_th.den <= 0 || jacc_th.num < 0 || max_cluster < 1 || max_cluster > 16 || !cl_row_ptr_h || !ncl ||
        sim_flags > HCSP_SIM_UNION)
        return fail(HCSP_E_INVALID, "hierarchical plan: bad arguments");
    Pattern P;
    int rc = make_pattern(A_h, perm_in_h, &P);
    if (rc) return rc;
    if (P.n > 0 && !perm_out_h) return fail(HCSP_E_INVALID, "null perm_out");
    const int64_t n = P.n, num = jacc_th.num, den = jacc_th.den;
    const int topk = max_cluster - 1;
    try {
        std::vector<int32_t> cnt((size_t)n, 0), nbr((size_t)n * std::max(topk, 1), -1);
        std::vector<Sim> nsim((size_t)n * std::max(topk, 1));
        if (topk > 0 && n > 0) {
            // transpose of the pattern in plan order: column -> positions holding it
            std::vector<int64_t> tp((size_t)P.ncols + 1, 0);
            for (int64_t p = 0; p < n; ++p)
                for (int64_t q = 0; q < P.len(p); ++q) tp[P.cols(p)[q] + 1]++;
            for (int64_t c = 0; c < P.ncols; ++c) tp[c + 1] += tp[c];
            std::vector<int32_t> tr((size_t)tp[P.ncols]);
            {
                std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
                for (int64_t p = 0; p < n; ++p)
                    for (int64_t q = 0; q < P.len(p); ++q) tr[fill[P.cols(p)[q]]++] = (int32_t)p;
            }
            int nt = nthreads > 0 ? nthreads : (int)std::thread::hardware_concurrency();
            nt = std::max(1, std::min<int>(nt, 64));
            if (n < 4096) nt = 1;
            std::vector<std::thread> th;
            for (int t = 0; t < nt; ++t) {
                const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
                th.emplace_back([&, lo, hi] { topk_rows(P, tp, tr, num, den, topk, lo, hi, cnt, nbr, nsim); });
            }
            for (auto &x : th) x.join();
        }
        return merge_phase(P, num, den, max_cluster, sim_flags, topk, cnt, nbr, nsim, perm_out_h, cl_row_ptr_h, ncl);
    } catch (const std::bad_alloc &) {
        return fail(HCSP_E_NOMEM, "hierarchical plan: host allocation failed");
    }
}

int hcsp_plan_hierarchical_candidates(const hcsp_csr *A_h, hcsp_ratio jacc_th, int32_t max_cluster,
                                      uint32_t sim_flags, const int32_t *perm_in_h, const int32_t *cnt_h,
                                      const int32_t *nbr_h, const int64_t *ov_h, int32_t *perm_out_h,
                                      int64_t *cl_row_ptr_h, int64_t *ncl)
{
    clear_error();
    if (jacc_th.den <= 0 || jacc_th.num < 0 || max_cluster < 1 || max_cluster > 16 || !cl_row_ptr_h || !ncl ||
        sim_flags > HCSP_SIM_UNION)
        return fail(HCSP_E_INVALID, "hierarchical plan: bad arguments");
    Pattern P;
    int rc = make_pattern(A_h, perm_in_h, &P);
    if (rc) return rc;
    if (P.n > 0 && !perm_out_h) return fail(HCSP_E_INVALID, "null perm_out");
    const int64_t n = P.n;
    const int topk = max_cluster - 1;
    if (topk > 0 && n > 0 && (!cnt_h || !nbr_h || !ov_h)) return fail(HCSP_E_INVALID, "null candidate lists");
    try {
        std::vector<int32_t> cnt((size_t)n, 0), nbr((size_t)n * std::max(topk, 1), -1);
        std::vector<Sim> nsim((size_t)n * std::max(topk, 1));
        for (int64_t i = 0; i < n && topk > 0; ++i) {
            if (cnt_h[i] < 0 || cnt_h[i] > topk) return fail(HCSP_E_INVALID, "candidate count out of range");
            cnt[i] = cnt_h[i];
            for (int x = 0; x < cnt[i]; ++x) {
                const size_t k = (size_t)i * topk + x;
                const int32_t j = nbr_h[k];
                if (j < 0 || j >= n || j == i) return fail(HCSP_E_INVALID, "candidate partner out of range");
                const int64_t ov = ov_h[k];
                if (ov < 0 || ov > std::min(P.len(i), P.len(j))) return fail(HCSP_E_INVALID, "overlap out of range");
                nbr[k] = j;
                nsim[k] = Sim{ov, P.len(i) + P.len(j) - ov};
            }
        }
        return merge_phase(P, jacc_th.num, jacc_th.den, max_cluster, sim_flags, topk, cnt, nbr, nsim, perm_out_h,
                           cl_row_ptr_h, ncl);
    } catch (const std::bad_alloc &) {
        return fail(HCSP_E_NOMEM, "hierarchical plan: host allocation failed");
    }
}

}  // extern "C"

namespace hcsp {
namespace {

int merge_phase(const Pattern &P, int64_t num, int64_t den, int32_t max_cluster, uint32_t sim_flags, int topk,
                const std::vector<int32_t> &cnt, const std::vector<int32_t> &nbr, const std::vector<Sim> &nsim,
                int32_t *perm_out_h, int64_t *cl_row_ptr_h, int64_t *ncl)
{
    const int64_t n = P.n;
    try {
        std::vector<int32_t> parent((size_t)n), size((size_t)n, 1), next((size_t)n, -1), tail((size_t)n);
        for (int64_t i = 0; i < n; ++i) parent[i] = tail[i] = (int32_t)i;
        // The initial candidate pairs (each row's list, pairs listed from both
        // ends once) are sorted best first and merged with a heap that only
        // holds the pairs pushed during the loop: the same pop order as one
        // heap over everything, without its cache misses.
        const CandLess less;
        std::vector<Cand> init;
        size_t ninit = 0;
        for (int64_t i = 0; i < n && topk > 0; ++i) ninit += (size_t)cnt[i];
        init.reserve(ninit);
        for (int64_t i = 0; i < n && topk > 0; ++i)
            for (int x = 0; x < cnt[i]; ++x) {
                int32_t a = (int32_t)i, b = nbr[(size_t)i * topk + x];
                if (a > b) std::swap(a, b);
                init.push_back(Cand{nsim[(size_t)i * topk + x], a, b});
            }
        {
            // order = similarity (exact ratio) descending, then i, then j: the
            // distinct similarities are ranked once (equal ratios share a
            // rank), then (rank, i, j) integer keys are sorted
            std::vector<Sim> vals;
            {
                PairSet seen(1024);
                for (const Cand &c : init)
                    if (seen.insert(((uint64_t)c.s.ov << 32) | (uint64_t)c.s.un)) vals.push_back(c.s);
            }
            std::sort(vals.begin(), vals.end(), [](const Sim &x, const Sim &y) { return cmp_sim(x, y) > 0; });
            std::vector<uint64_t> vkey(vals.size());
            std::vector<uint32_t> vrank(vals.size());
            for (size_t x = 0; x < vals.size(); ++x) {
                vkey[x] = ((uint64_t)vals[x].ov << 32) | (uint64_t)vals[x].un;
                vrank[x] = x > 0 && cmp_sim(vals[x], vals[x - 1]) == 0 ? vrank[x - 1] : (uint32_t)x;
            }
            // (ov, un) -> rank through a sorted key table
            std::vector<size_t> vo(vals.size());
            for (size_t x = 0; x < vo.size(); ++x) vo[x] = x;
            std::sort(vo.begin(), vo.end(), [&](size_t x, size_t y) { return vkey[x] < vkey[y]; });
            std::vector<uint64_t> skey(vals.size());
            std::vector<uint32_t> srank(vals.size());
            for (size_t x = 0; x < vo.size(); ++x) {
                skey[x] = vkey[vo[x]];
                srank[x] = vrank[vo[x]];
            }
            struct Key {
                uint64_t hi;  // rank, i
                uint32_t j;
            };
            std::vector<Key> keys(init.size());
            for (size_t x = 0; x < init.size(); ++x) {
                const uint64_t k = ((uint64_t)init[x].s.ov << 32) | (uint64_t)init[x].s.un;
                const uint32_t r = srank[(size_t)(std::lower_bound(skey.begin(), skey.end(), k) - skey.begin())];
                keys[x] = Key{((uint64_t)r << 32) | (uint32_t)init[x].i, (uint32_t)init[x].j};
            }
            std::sort(keys.begin(), keys.end(),
                      [](const Key &x, const Key &y) { return x.hi != y.hi ? x.hi < y.hi : x.j < y.j; });
            for (size_t x = 0; x < keys.size(); ++x)
                init[x] = Cand{vals[keys[x].hi >> 32], (int32_t)(uint32_t)keys[x].hi, (int32_t)keys[x].j};
        }
        // a pair listed by both rows has the same similarity: the copies are adjacent
        init.erase(std::unique(init.begin(), init.end(),
                               [](const Cand &x, const Cand &y) { return x.i == y.i && x.j == y.j; }),
                   init.end());
        std::priority_queue<Cand, std::vector<Cand>, CandLess> heap;
        PairSet pushed(1024);
        // was (a, b) ever a candidate: in a's or b's initial list, or pushed
        auto listed = [&](int32_t a, int32_t b) -> bool {
            for (int x = 0; x < cnt[a]; ++x)
                if (nbr[(size_t)a * topk + x] == b) return true;
            for (int x = 0; x < cnt[b]; ++x)
                if (nbr[(size_t)b * topk + x] == a) return true;
            return pushed.contains(pair_key(a, b));
        };
        const PosPattern Q(P);
        std::vector<int64_t> mark;
        int64_t stamp = 0;
        if (sim_flags == HCSP_SIM_UNION) mark.assign((size_t)std::max<int64_t>(P.ncols, 1), -1);
        auto union_sim = [&](int32_t a, int32_t b) -> Sim {
            const int64_t sa = ++stamp;
            int64_t na = 0;
            for (int32_t m = a; m >= 0; m = next[m])
                for (int64_t q = 0; q < Q.len(m); ++q) {
                    const int32_t c = Q.cols(m)[q];
                    if (mark[c] != sa) {
                        mark[c] = sa;
                        ++na;
                    }
                }
            const int64_t sb = ++stamp;
            int64_t nb = 0, ov = 0;
            for (int32_t m = b; m >= 0; m = next[m])
                for (int64_t q = 0; q < Q.len(m); ++q) {
                    const int32_t c = Q.cols(m)[q];
                    if (mark[c] == sb) continue;
                    if (mark[c] == sa) ++ov;
                    mark[c] = sb;
                    ++nb;
                }
            return Sim{ov, na + nb - ov};
        };
        size_t ip = 0;
        while (ip < init.size() || !heap.empty()) {
            Cand top;
            if (heap.empty() || (ip < init.size() && less(heap.top(), init[ip]))) {
                top = init[ip++];
            } else {
                top = heap.top();
                heap.pop();
            }
            const int32_t i = top.i, j = top.j;
            if (parent[i] == i && parent[j] == j) {
                if (size[i] + size[j] <= max_cluster) {
                    parent[j] = i;  // i < j: the smaller position stays root
                    size[i] += size[j];
                    next[tail[i]] = j;
                    tail[i] = tail[j];
                }
                continue;
            }
            const int32_t ri = uf_find(parent, i), rj = uf_find(parent, j);
            if (ri == rj) continue;
            const int32_t a = std::min(ri, rj), b = std::max(ri, rj);
            if (topk > 0 && listed(a, b)) continue;
            const Sim s = sim_flags == HCSP_SIM_UNION ? union_sim(a, b) : jaccard(Q, a, b);
            if (cmp_thr(s, num, den) > 0) {
                heap.push(Cand{s, a, b});
                pushed.insert(pair_key(a, b));
            }
        }
        return emit(P, parent, next, perm_out_h, cl_row_ptr_h, ncl);
    } catch (const std::bad_alloc &) {
        return fail(HCSP_E_NOMEM, "hierarchical plan: host allocation failed");
    }
}

}  // namespace
}  // namespace hcsp
