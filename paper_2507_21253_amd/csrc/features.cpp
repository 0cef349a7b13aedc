// Structure-only features of a product C = A x B, read from host copies of
// the patterns (values are never read).  They describe what decides the
// speed of the row-wise product and of its clustered forms: sizes, row
// lengths, the per-row product counts (the work of Gustavson's algorithm),
// locality (column distance from the diagonal), similarity of neighbouring
// rows (what variable-length clustering, Alg. 2, can merge), the best
// similarity a row finds anywhere (what hierarchical clustering, Alg. 3,
// can merge) and the compression of products into output entries.  Sampled
// quantities use a fixed, evenly spaced row sample, so the features are
// deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace hcsp {
namespace {

inline double lg(double x) { return std::log2(x + 1.0); }

int64_t overlap(const int32_t *a, int64_t na, const int32_t *b, int64_t nb)
{
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
    return ov;
}

double quantile(std::vector<int64_t> v, double q)
{
    if (v.empty()) return 0.0;
    const size_t k = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + (ptrdiff_t)k, v.end());
    return (double)v[k];
}

}  // namespace
}  // namespace hcsp

using namespace hcsp;

extern "C" int hcsp_features(const hcsp_csr *A, const hcsp_csr *B, float *out)
{
    clear_error();
    if (!A || !B || !out || !A->row_ptr || !B->row_ptr || (A->nnz > 0 && !A->col) || (B->nnz > 0 && !B->col))
        return fail(HCSP_E_INVALID, "null argument");
    if (A->ncols != B->nrows) return fail(HCSP_E_INVALID, "A.ncols != B.nrows");
    const int64_t n = A->nrows;
    const int64_t *rp = A->row_ptr, *brp = B->row_ptr;
    const int32_t *col = A->col;
    double f[HCSP_NFEATURES];
    std::memset(f, 0, sizeof f);
    try {
        std::vector<int64_t> len((size_t)n), ub((size_t)n);
        double sl = 0, sl2 = 0, su = 0, su2 = 0, sb = 0, sb2 = 0;
        int64_t maxl = 0, maxu = 0, empty = 0, nb = 0;
        int64_t bins[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t i = 0; i < n; ++i) {
            const int64_t l = rp[i + 1] - rp[i];
            int64_t u = 0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                const int32_t k = col[p];
                u += brp[k + 1] - brp[k];
                const double d = std::fabs((double)k - (double)i) / (double)std::max<int64_t>(A->ncols, 1);
                sb += d;
                sb2 += d * d;
                ++nb;
            }
            len[(size_t)i] = l;
            ub[(size_t)i] = u;
            sl += (double)l;
            sl2 += (double)l * (double)l;
            su += (double)u;
            su2 += (double)u * (double)u;
            maxl = std::max(maxl, l);
            maxu = std::max(maxu, u);
            empty += l == 0;
            const int b = u < 64 ? 0 : u < 256 ? 1 : u < 1024 ? 2 : u < 4096 ? 3 : u < 16384 ? 4 : 5;
            ++bins[b];
        }
        const double dn = (double)std::max<int64_t>(n, 1);
        const double ml = sl / dn, mu = su / dn;
        f[0] = lg((double)n);
        f[1] = lg((double)A->nnz);
        f[2] = ml;
        f[3] = std::sqrt(std::max(0.0, sl2 / dn - ml * ml));
        f[4] = lg((double)maxl);
        const double qs[5] = {0.10, 0.25, 0.50, 0.75, 0.90};
        for (int q = 0; q < 5; ++q) f[5 + q] = lg(quantile(len, qs[q]));
        f[10] = lg(su);
        f[11] = lg(mu);
        f[12] = mu > 0 ? std::sqrt(std::max(0.0, su2 / dn - mu * mu)) / mu : 0.0;
        f[13] = lg((double)maxu);
        const double dnb = (double)std::max<int64_t>(nb, 1);
        f[14] = sb / dnb;
        f[15] = std::sqrt(std::max(0.0, sb2 / dnb - (sb / dnb) * (sb / dnb)));

        // neighbouring rows: Jaccard of (i, i+1), pair and block-of-8 compression
        const int64_t npairs = std::min<int64_t>(4096, std::max<int64_t>(n - 1, 0));
        double sj = 0, j3 = 0, j5 = 0, pin = 0, pun = 0;
        for (int64_t s = 0; s < npairs; ++s) {
            const int64_t i = npairs == n - 1 ? s : s * (n - 1) / npairs;
            const int64_t la = rp[i + 1] - rp[i], lb = rp[i + 2] - rp[i + 1];
            const int64_t ov = overlap(col + rp[i], la, col + rp[i + 1], lb);
            const int64_t un = la + lb - ov;
            const double J = un ? (double)ov / (double)un : 0.0;
            sj += J;
            j3 += J >= 0.3;
            j5 += J >= 0.5;
            if (J >= 0.3) {
                pin += (double)(la + lb);
                pun += (double)un;
            }
        }
        f[16] = npairs ? sj / (double)npairs : 0.0;
        f[17] = npairs ? j3 / (double)npairs : 0.0;
        f[18] = npairs ? j5 / (double)npairs : 0.0;
        f[19] = pun > 0 ? pin / pun : 1.0;
        const int64_t nblk = std::min<int64_t>(512, n / 8);
        double slots = 0, ent = 0;
        std::vector<int32_t> u8;
        for (int64_t s = 0; s < nblk; ++s) {
            const int64_t i0 = s * (n / 8) / std::max<int64_t>(nblk, 1) * 8;
            u8.clear();
            for (int64_t i = i0; i < i0 + 8; ++i) u8.insert(u8.end(), col + rp[i], col + rp[i + 1]);
            ent += (double)u8.size();
            std::sort(u8.begin(), u8.end());
            slots += 8.0 * (double)(std::unique(u8.begin(), u8.end()) - u8.begin());
        }
        f[20] = ent > 0 ? slots / ent : 1.0;

        // sampled rows: best Jaccard with any row sharing a column (A^T lists
        // capped at 64 rows per column), and exact output count of the row
        const int64_t ns = std::min<int64_t>(256, n);
        std::vector<int64_t> cp((size_t)A->ncols + 1, 0);
        for (int64_t p = 0; p < A->nnz; ++p) ++cp[(size_t)col[p] + 1];
        for (int64_t k = 0; k < A->ncols; ++k) cp[(size_t)k + 1] += cp[(size_t)k];
        std::vector<int32_t> rows_of((size_t)A->nnz);
        {
            std::vector<int64_t> cur(cp.begin(), cp.end() - 1);
            for (int64_t i = 0; i < n; ++i)
                for (int64_t p = rp[i]; p < rp[i + 1]; ++p) rows_of[(size_t)cur[(size_t)col[p]]++] = (int32_t)i;
        }
        std::vector<int32_t> mark((size_t)std::max<int64_t>(std::max(n, B->ncols), 1), -1);
        std::vector<int32_t> cnt((size_t)std::max<int64_t>(n, 1), 0), touched;
        double best = 0, sub = 0, sout = 0;
        for (int64_t s = 0; s < ns; ++s) {
            const int64_t i = s * n / ns;
            const int64_t la = rp[i + 1] - rp[i];
            touched.clear();
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                const int32_t k = col[p];
                const int64_t e = std::min(cp[(size_t)k + 1], cp[(size_t)k] + 64);
                for (int64_t q = cp[(size_t)k]; q < e; ++q) {
                    const int32_t r = rows_of[(size_t)q];
                    if (r == i) continue;
                    if (cnt[(size_t)r]++ == 0) touched.push_back(r);
                }
            }
            double bj = 0;
            for (int32_t r : touched) {
                const int64_t ov = overlap(col + rp[i], la, col + rp[r], rp[r + 1] - rp[r]);
                const int64_t un = la + (rp[r + 1] - rp[r]) - ov;
                if (un) bj = std::max(bj, (double)ov / (double)un);
                cnt[(size_t)r] = 0;
            }
            best += bj;
            int64_t outs = 0;
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
                const int32_t k = col[p];
                for (int64_t q = brp[k]; q < brp[k + 1]; ++q) {
                    const int32_t j = B->col[q];
                    if (mark[(size_t)j] != (int32_t)s) {
                        mark[(size_t)j] = (int32_t)s;
                        ++outs;
                    }
                }
            }
            sub += (double)ub[(size_t)i];
            sout += (double)outs;
        }
        f[21] = ns ? best / (double)ns : 0.0;
        f[22] = sout > 0 ? sub / sout : 1.0;
        f[23] = (double)empty / dn;
        for (int b = 0; b < 6; ++b) f[24 + b] = (double)bins[b] / dn;
        f[30] = lg((double)B->ncols);
        int64_t wide = 0;
        for (int64_t i = 0; i < n; ++i) wide += (double)len[(size_t)i] > 2.0 * ml;
        f[31] = (double)wide / dn;
    } catch (const std::bad_alloc &) {
        return fail(HCSP_E_NOMEM, "out of host memory");
    }
    for (int i = 0; i < HCSP_NFEATURES; ++i) out[i] = (float)f[i];
    return HCSP_OK;
}
