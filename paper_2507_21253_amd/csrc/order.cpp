// Host row orderings and the symmetric permutation of a CSR matrix: the
// reordering step the paper applies before row-wise or cluster-wise SpGEMM
// (Sec. "Matrix Reordering", Table of reordering algorithms): reverse
// Cuthill-McKee (bandwidth reduction by breadth-first search) and degree
// order (rows by descending length).  A random order is an input, not an
// algorithm, and comes from the caller.
//
// Reverse Cuthill-McKee here works on the pattern of A + A^T without the
// diagonal.  Each connected component starts from a pseudo-peripheral vertex
// found the George-Liu way (breadth-first level structures from a vertex of
// minimum degree, moving to a minimum-degree vertex of the last level while
// that deepens the structure); the breadth-first search visits unvisited
// neighbours by ascending degree, ties by id; components follow each other
// in the order of their lowest-(degree, id) vertex, and the whole sequence
// is reversed at the end.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "internal.h"

namespace hcsp {
namespace {

struct Graph {
    std::vector<int64_t> ptr;
    std::vector<int32_t> adj;  // neighbours sorted by (degree, id)
    std::vector<int64_t> deg;
};

// f(lo, hi) over [0, n) split into contiguous ranges on the host's threads.
template <class F>
void parallel_ranges(int64_t n, F f)
{
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>({(int64_t)std::thread::hardware_concurrency(), 64,
                                                               (n + 65535) / 65536}));
    if (nt == 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    for (int64_t t = 0; t < nt; ++t) th.emplace_back(f, n * t / nt, n * (t + 1) / nt);
    for (auto &x : th) x.join();
}

// Whether A's pattern is symmetric (j in row i iff i in row j; rows sorted):
// each entry looks itself up in the other row, rows split over the threads.
bool pattern_symmetric(const hcsp_csr &A)
{
    std::atomic<bool> ok(true);
    parallel_ranges(A.nrows, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi && ok.load(std::memory_order_relaxed); ++i)
            for (int64_t p = A.row_ptr[i]; p < A.row_ptr[i + 1]; ++p) {
                const int64_t j = A.col[p];
                const int32_t *b = A.col + A.row_ptr[j], *e = A.col + A.row_ptr[j + 1];
                const int32_t *f = std::lower_bound(b, e, (int32_t)i);
                if (f == e || *f != (int32_t)i) {
                    ok.store(false, std::memory_order_relaxed);
                    break;
                }
            }
    });
    return ok.load();
}

// Pattern of A + A^T without the diagonal, duplicate-free.
void build_graph(const hcsp_csr &A, Graph &g)
{
    const int64_t n = A.nrows;
    if (pattern_symmetric(A)) {
        // A + A^T has A's pattern: rows copied without the diagonal
        g.ptr.assign((size_t)n + 1, 0);
        g.deg.assign((size_t)n, 0);
        parallel_ranges(n, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) {
                int64_t d = A.row_ptr[i + 1] - A.row_ptr[i];
                const int32_t *b = A.col + A.row_ptr[i], *e = A.col + A.row_ptr[i + 1];
                if (std::binary_search(b, e, (int32_t)i)) --d;
                g.deg[(size_t)i] = d;
            }
        });
        for (int64_t i = 0; i < n; ++i) g.ptr[(size_t)i + 1] = g.ptr[(size_t)i] + g.deg[(size_t)i];
        g.adj.resize((size_t)g.ptr[(size_t)n]);
        parallel_ranges(n, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) {
                auto o = g.adj.begin() + g.ptr[(size_t)i];
                for (int64_t p = A.row_ptr[i]; p < A.row_ptr[i + 1]; ++p)
                    if (A.col[p] != i) *o++ = A.col[p];
                std::sort(g.adj.begin() + g.ptr[(size_t)i], o, [&](int32_t x, int32_t y) {
                    return g.deg[(size_t)x] != g.deg[(size_t)y] ? g.deg[(size_t)x] < g.deg[(size_t)y] : x < y;
                });
            }
        });
        return;
    }
    std::vector<int64_t> cnt((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = A.row_ptr[i]; p < A.row_ptr[i + 1]; ++p) {
            const int64_t j = A.col[p];
            if (j == i) continue;
            ++cnt[(size_t)i + 1];
            ++cnt[(size_t)j + 1];
        }
    for (int64_t i = 0; i < n; ++i) cnt[(size_t)i + 1] += cnt[(size_t)i];
    std::vector<int32_t> raw((size_t)cnt[(size_t)n]);
    std::vector<int64_t> cur(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = A.row_ptr[i]; p < A.row_ptr[i + 1]; ++p) {
            const int64_t j = A.col[p];
            if (j == i) continue;
            raw[(size_t)cur[(size_t)i]++] = (int32_t)j;
            raw[(size_t)cur[(size_t)j]++] = (int32_t)i;
        }
    g.ptr.assign((size_t)n + 1, 0);
    g.deg.assign((size_t)n, 0);
    // rows are independent: sorted and de-duplicated on the host's threads
    parallel_ranges(n, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            auto b = raw.begin() + cnt[(size_t)i], e = raw.begin() + cnt[(size_t)i + 1];
            std::sort(b, e);
            g.deg[(size_t)i] = std::unique(b, e) - b;
        }
    });
    for (int64_t i = 0; i < n; ++i) g.ptr[(size_t)i + 1] = g.ptr[(size_t)i] + g.deg[(size_t)i];
    g.adj.resize((size_t)g.ptr[(size_t)n]);
    parallel_ranges(n, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            std::copy(raw.begin() + cnt[(size_t)i], raw.begin() + cnt[(size_t)i] + g.deg[(size_t)i],
                      g.adj.begin() + g.ptr[(size_t)i]);
            auto b = g.adj.begin() + g.ptr[(size_t)i], e = g.adj.begin() + g.ptr[(size_t)i + 1];
            std::sort(b, e, [&](int32_t x, int32_t y) {
                return g.deg[(size_t)x] != g.deg[(size_t)y] ? g.deg[(size_t)x] < g.deg[(size_t)y] : x < y;
            });
        }
    });
}

inline bool before(const Graph &g, int64_t x, int64_t y)
{
    return g.deg[(size_t)x] != g.deg[(size_t)y] ? g.deg[(size_t)x] < g.deg[(size_t)y] : x < y;
}

// Breadth-first search from s over unvisited (stamp != mark) vertices; fills
// `out` in visit order and returns the number of levels.  `last` receives the
// first vertex of the deepest level with the least (degree, id).
int64_t bfs(const Graph &g, int64_t s, std::vector<int32_t> &stamp, int32_t mark, std::vector<int32_t> &out,
            int64_t *last)
{
    out.clear();
    out.push_back((int32_t)s);
    stamp[(size_t)s] = mark;
    int64_t head = 0, levels = 0;
    while (head < (int64_t)out.size()) {
        const int64_t lb = head, le = (int64_t)out.size();
        ++levels;
        int64_t best = out[(size_t)lb];
        for (int64_t q = lb; q < le; ++q) {
            const int64_t u = out[(size_t)q];
            if (before(g, u, best)) best = u;
            for (int64_t p = g.ptr[(size_t)u]; p < g.ptr[(size_t)u + 1]; ++p) {
                const int32_t w = g.adj[(size_t)p];
                if (stamp[(size_t)w] != mark) {
                    stamp[(size_t)w] = mark;
                    out.push_back(w);
                }
            }
        }
        head = le;
        *last = best;
    }
    return levels;
}

}  // namespace
}  // namespace hcsp

using namespace hcsp;

extern "C" {

int hcsp_order_rcm(const hcsp_csr *A, int32_t *perm_out)
{
    clear_error();
    if (!A || !perm_out || !A->row_ptr || (A->nnz > 0 && !A->col)) return fail(HCSP_E_INVALID, "null argument");
    if (A->nrows != A->ncols) return fail(HCSP_E_INVALID, "reverse Cuthill-McKee needs a square matrix");
    const int64_t n = A->nrows;
    try {
        Graph g;
        build_graph(*A, g);
        std::vector<int32_t> byd((size_t)n);
        for (int64_t i = 0; i < n; ++i) byd[(size_t)i] = (int32_t)i;
        std::sort(byd.begin(), byd.end(), [&](int32_t x, int32_t y) { return before(g, x, y); });
        std::vector<int32_t> probe((size_t)n, -1), lev;
        std::vector<uint8_t> done((size_t)n, 0);
        std::vector<int32_t> order;
        order.reserve((size_t)n);
        int32_t pmark = 0;
        int64_t next = 0;
        while ((int64_t)order.size() < n) {
            while (done[(size_t)byd[(size_t)next]]) ++next;
            int64_t s = byd[(size_t)next], last = s;
            // pseudo-peripheral start (searches stay inside the component: its
            // vertices are exactly the unvisited ones reachable from s)
            int64_t h = bfs(g, s, probe, ++pmark, lev, &last);
            for (;;) {
                int64_t last2 = last;
                const int64_t h2 = bfs(g, last, probe, ++pmark, lev, &last2);
                if (h2 <= h) break;
                s = last;
                h = h2;
                last = last2;
            }
            // Cuthill-McKee order of the component
            const size_t base = order.size();
            order.push_back((int32_t)s);
            done[(size_t)s] = 1;
            for (size_t q = base; q < order.size(); ++q) {
                const int64_t u = order[q];
                for (int64_t p = g.ptr[(size_t)u]; p < g.ptr[(size_t)u + 1]; ++p) {
                    const int32_t w = g.adj[(size_t)p];
                    if (!done[(size_t)w]) {
                        done[(size_t)w] = 1;
                        order.push_back(w);
                    }
                }
            }
        }
        for (int64_t i = 0; i < n; ++i) perm_out[i] = order[(size_t)(n - 1 - i)];
    } catch (const std::bad_alloc &) {
        return fail(HCSP_E_NOMEM, "out of host memory");
    }
    return HCSP_OK;
}

int hcsp_order_degree(const hcsp_csr *A, int32_t *perm_out)
{
    clear_error();
    if (!A || !perm_out || !A->row_ptr) return fail(HCSP_E_INVALID, "null argument");
    const int64_t n = A->nrows;
    try {
        std::vector<int32_t> p((size_t)n);
        for (int64_t i = 0; i < n; ++i) p[(size_t)i] = (int32_t)i;
        std::stable_sort(p.begin(), p.end(), [&](int32_t x, int32_t y) {
            return A->row_ptr[x + 1] - A->row_ptr[x] > A->row_ptr[y + 1] - A->row_ptr[y];
        });
        std::memcpy(perm_out, p.data(), sizeof(int32_t) * (size_t)n);
    } catch (const std::bad_alloc &) {
        return fail(HCSP_E_NOMEM, "out of host memory");
    }
    return HCSP_OK;
}

int hcsp_permute_h(const hcsp_csr *A, const int32_t *rperm, const int32_t *cperm, hcsp_csr *out, int32_t nthreads)
{
    clear_error();
    if (!A || !out || !A->row_ptr || (A->nnz > 0 && (!A->col || !A->val)) || !out->row_ptr ||
        (A->nnz > 0 && (!out->col || !out->val)))
        return fail(HCSP_E_INVALID, "null argument");
    if (out->nrows != A->nrows || out->ncols != A->ncols || out->nnz != A->nnz)
        return fail(HCSP_E_INVALID, "output shape differs from A");
    const int64_t n = A->nrows, m = A->ncols;
    try {
        // position maps: new row r holds old row rperm[r]; old column c becomes inv[c]
        std::vector<int32_t> cinv((size_t)m);
        std::vector<uint8_t> seen((size_t)std::max(n, m), 0);
        if (rperm) {
            for (int64_t r = 0; r < n; ++r) {
                const int64_t o = rperm[r];
                if (o < 0 || o >= n || seen[(size_t)o]) return fail(HCSP_E_INVALID, "rperm is not a permutation");
                seen[(size_t)o] = 1;
            }
            std::fill(seen.begin(), seen.end(), 0);
        }
        for (int64_t c = 0; c < m; ++c) {
            const int64_t o = cperm ? cperm[c] : c;
            if (o < 0 || o >= m || seen[(size_t)o]) return fail(HCSP_E_INVALID, "cperm is not a permutation");
            seen[(size_t)o] = 1;
            cinv[(size_t)o] = (int32_t)c;
        }
        out->row_ptr[0] = 0;
        for (int64_t r = 0; r < n; ++r) {
            const int64_t o = rperm ? rperm[r] : r;
            out->row_ptr[r + 1] = out->row_ptr[r] + (A->row_ptr[o + 1] - A->row_ptr[o]);
        }
        const int nt = std::max(1, std::min<int>(nthreads > 0 ? nthreads : 1, 64));
        auto work = [&](int t) {
            std::vector<std::pair<int32_t, double>> row;
            for (int64_t r = (int64_t)t; r < n; r += nt) {
                const int64_t o = rperm ? rperm[r] : r;
                row.clear();
                for (int64_t p = A->row_ptr[o]; p < A->row_ptr[o + 1]; ++p)
                    row.emplace_back(cinv[(size_t)A->col[p]], A->val[p]);
                std::sort(row.begin(), row.end(),
                          [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
                              return x.first < y.first;
                          });
                int64_t q = out->row_ptr[r];
                for (const auto &e : row) {
                    out->col[q] = e.first;
                    out->val[q] = e.second;
                    ++q;
                }
            }
        };
        std::vector<std::thread> th;
        for (int t = 1; t < nt; ++t) th.emplace_back(work, t);
        work(0);
        for (auto &x : th) x.join();
    } catch (const std::bad_alloc &) {
        return fail(HCSP_E_NOMEM, "out of host memory");
    } catch (const std::system_error &) {
        return fail(HCSP_E_NOMEM, "could not start host threads");
    }
    return HCSP_OK;
}

}  // extern "C"
