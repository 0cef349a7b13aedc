/*
 * Seeded synthetic sparse-matrix generators (inputs only).
 *
 * This module produces the input matrices that both the CPU oracle and the
 * GPU library are run on.  It holds none of the SpGEMM method's arithmetic:
 * no products, no accumulators, no clustering.  Every random draw comes from
 * one counter-based generator so a (seed, stream, counter) triple always
 * yields the same number on every machine.
 *
 * Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014, in the public-domain formulation by
 * S. Vigna).  Its n-th output from state s is mix(s + (n+1)*gamma), which is
 * already counter-based: synth_u64(key, n) below is exactly that.
 *
 * Matrices are CSR with int64 row offsets, int32 column indices (strictly
 * increasing inside a row) and float64 values.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define SM_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* n-th SplitMix64 output for a generator whose state starts at `key`. */
uint64_t synth_u64(uint64_t key, uint64_t n)
{
    return sm_mix(key + (n + 1) * SM_GAMMA);
}

/* Independent stream key for (seed, tag). */
uint64_t synth_key(uint64_t seed, uint64_t tag)
{
    return sm_mix(sm_mix(seed + SM_GAMMA) ^ sm_mix(tag * 0xD1342543DE82EF95ULL + 1));
}

/* Uniform double in [0,1) with 53 random bits. */
double synth_u01(uint64_t key, uint64_t n)
{
    return (double)(synth_u64(key, n) >> 11) * 0x1.0p-53;
}

/* Uniform double in [-1,1). */
static inline double uval(uint64_t key, uint64_t n)
{
    return 2.0 * synth_u01(key, n) - 1.0;
}

/* Integer in [0, m) by the multiply-high map (m >= 1). */
static inline uint64_t below(uint64_t key, uint64_t n, uint64_t m)
{
    return (uint64_t)(((unsigned __int128)synth_u64(key, n) * m) >> 64);
}

enum { TAG_COL = 1, TAG_VAL = 2, TAG_PERM = 3, TAG_RMAT = 4, TAG_FRONTIER = 5 };  /* 5 and 6 */

static void isort_i32(int32_t *a, int64_t n)
{
    for (int64_t i = 1; i < n; ++i) {
        int32_t x = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
        a[j + 1] = x;
    }
}

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

static void sort_i32(int32_t *a, int64_t n)
{
    if (n <= 32) isort_i32(a, n);
    else qsort(a, (size_t)n, sizeof(int32_t), cmp_i32);
}

/*
 * Uniform-random matrix: every row holds exactly d distinct columns drawn
 * uniformly from [0, ncols) by Floyd's sampling algorithm (Bentley & Floyd,
 * CACM 1987), values U(-1,1).  Returns 0, or -1 on bad sizes.
 */
int synth_uniform(int64_t nrows, int64_t ncols, int32_t d, uint64_t seed,
                  int64_t *rp, int32_t *col, double *val)
{
    if (nrows < 0 || ncols < 1 || d < 0 || d > ncols || ncols > INT32_MAX) return -1;
    uint64_t kc = synth_key(seed, TAG_COL), kv = synth_key(seed, TAG_VAL);
    rp[0] = 0;
    for (int64_t r = 0; r < nrows; ++r) {
        int32_t *row = col + r * (int64_t)d;
        int32_t cnt = 0;
        uint64_t base = (uint64_t)r * (uint64_t)d;
        for (int64_t j = ncols - d; j < ncols; ++j) {
            int32_t t = (int32_t)below(kc, base + (uint64_t)(j - (ncols - d)), (uint64_t)j + 1);
            int seen = 0;
            for (int32_t q = 0; q < cnt; ++q) if (row[q] == t) { seen = 1; break; }
            row[cnt++] = seen ? (int32_t)j : t;
        }
        sort_i32(row, d);
        for (int32_t q = 0; q < d; ++q) val[base + (uint64_t)q] = uval(kv, base + (uint64_t)q);
        rp[r + 1] = rp[r] + d;
    }
    return 0;
}

/* Grid shape of a stencil kind: 5 -> 2D, 7 and 27 -> 3D. */
static int stencil_dims(int kind)
{
    if (kind == 5) return 2;
    if (kind == 7 || kind == 27) return 3;
    return 0;
}

static int64_t ipow(int64_t b, int e) { int64_t r = 1; while (e-- > 0) r *= b; return r; }

/* Number of non-zeros of a stencil matrix on an m^dim grid (counted, not a formula). */
int64_t synth_stencil_nnz(int kind, int64_t m)
{
    int dims = stencil_dims(kind);
    if (!dims || m < 1) return -1;
    int64_t n = ipow(m, dims), nnz = 0;
    for (int64_t r = 0; r < n; ++r) {
        int64_t x = r % m, y = (r / m) % m, z = dims == 3 ? r / (m * m) : 0;
        if (kind == 27) {
            int64_t cx = 1 + (x > 0) + (x < m - 1), cy = 1 + (y > 0) + (y < m - 1), cz = 1 + (z > 0) + (z < m - 1);
            nnz += cx * cy * cz;
        } else {
            nnz += 1 + (x > 0) + (x < m - 1) + (y > 0) + (y < m - 1);
            if (dims == 3) nnz += (z > 0) + (z < m - 1);
        }
    }
    return nnz;
}

/*
 * Stencil matrix on an m^dim grid, row index x + m*(y + m*z) (x fastest).
 * kind 5: 2D 5-point; 7: 3D 7-point; 27: 3D 27-point (all 3x3x3 neighbours).
 * Values U(-1,1), one draw per stored entry in CSR order.
 */
int synth_stencil(int kind, int64_t m, uint64_t seed, int64_t *rp, int32_t *col, double *val)
{
    int dims = stencil_dims(kind);
    if (!dims || m < 1) return -1;
    int64_t n = ipow(m, dims);
    if (n > INT32_MAX) return -1;
    uint64_t kv = synth_key(seed, TAG_VAL);
    int64_t p = 0;
    rp[0] = 0;
    for (int64_t r = 0; r < n; ++r) {
        int64_t x = r % m, y = (r / m) % m, z = dims == 3 ? r / (m * m) : 0;
        for (int dz = -1; dz <= 1; ++dz) {
            if (dims == 2 && dz != 0) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                for (int dx = -1; dx <= 1; ++dx) {
                    int nzc = (dx != 0) + (dy != 0) + (dz != 0);
                    if (kind != 27 && nzc > 1) continue;
                    int64_t xx = x + dx, yy = y + dy, zz = z + dz;
                    if (xx < 0 || xx >= m || yy < 0 || yy >= m || zz < 0 || zz >= m) continue;
                    col[p] = (int32_t)(xx + m * (yy + m * zz));
                    val[p] = uval(kv, (uint64_t)p);
                    ++p;
                }
            }
        }
        rp[r + 1] = p;
    }
    return 0;
}

/* Seeded uniform permutation of [0, n) by the Fisher-Yates shuffle. */
int synth_perm(int64_t n, uint64_t seed, int32_t *perm)
{
    if (n < 0 || n > INT32_MAX) return -1;
    uint64_t k = synth_key(seed, TAG_PERM);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)below(k, (uint64_t)i, (uint64_t)i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    return 0;
}

typedef struct { int32_t c; int64_t src; } cpair;

static int cmp_cpair(const void *x, const void *y)
{
    const cpair *a = (const cpair *)x, *b = (const cpair *)y;
    return (a->c > b->c) - (a->c < b->c);
}

/*
 * Relabel a matrix: output row rmap[u] holds input row u, and (if cmap is
 * non-null) every column v becomes cmap[v]; rows are re-sorted by column with
 * values carried along.  rmap == cmap gives the symmetric relabel Q S Q^T;
 * cmap == NULL gives a row permutation only.  Output arrays have the input's
 * sizes.  Returns 0, or -1 if the input has unsorted rows after mapping
 * collisions (cannot happen for permutations).
 */
int synth_relabel(int64_t nrows, const int64_t *rp, const int32_t *col, const double *val,
                  const int32_t *rmap, const int32_t *cmap,
                  int64_t *rp2, int32_t *col2, double *val2)
{
    int32_t *inv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nrows > 0 ? nrows : 1));
    if (!inv) return -1;
    for (int64_t u = 0; u < nrows; ++u) inv[rmap[u]] = (int32_t)u;
    rp2[0] = 0;
    for (int64_t r = 0; r < nrows; ++r) rp2[r + 1] = rp2[r] + (rp[inv[r] + 1] - rp[inv[r]]);
    int64_t cap = 0;
    cpair *buf = NULL;
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t u = inv[r], b = rp[u], len = rp[u + 1] - b, o = rp2[r];
        if (!cmap) {
            memcpy(col2 + o, col + b, sizeof(int32_t) * (size_t)len);
            memcpy(val2 + o, val + b, sizeof(double) * (size_t)len);
            continue;
        }
        if (len > cap) {
            cap = len * 2;
            free(buf);
            buf = (cpair *)malloc(sizeof(cpair) * (size_t)cap);
            if (!buf) { free(inv); return -1; }
        }
        for (int64_t q = 0; q < len; ++q) { buf[q].c = cmap[col[b + q]]; buf[q].src = b + q; }
        if (len <= 32) {
            for (int64_t i = 1; i < len; ++i) {
                cpair x = buf[i]; int64_t j = i - 1;
                while (j >= 0 && buf[j].c > x.c) { buf[j + 1] = buf[j]; --j; }
                buf[j + 1] = x;
            }
        } else {
            qsort(buf, (size_t)len, sizeof(cpair), cmp_cpair);
        }
        for (int64_t q = 0; q < len; ++q) { col2[o + q] = buf[q].c; val2[o + q] = val[buf[q].src]; }
    }
    free(buf);
    free(inv);
    return 0;
}

/*
 * R-MAT graph (Chakrabarti, Zhan & Faloutsos, SDM 2004): 2^scale vertices,
 * `nedges` generated edges, quadrant probabilities (a, b, c, 1-a-b-c), no
 * noise.  Self-loops are dropped, the edge set is symmetrised and
 * de-duplicated.  Writes rp[n+1] and up to `cap` sorted columns; returns the
 * final nnz, or -1 on bad arguments / -2 if cap is too small.
 */
int64_t synth_rmat(int scale, int64_t nedges, double a, double b, double c, uint64_t seed,
                   int64_t *rp, int32_t *col, int64_t cap)
{
    if (scale < 1 || scale > 30 || nedges < 0) return -1;
    int64_t n = (int64_t)1 << scale;
    uint64_t k = synth_key(seed, TAG_RMAT);
    int32_t *eu = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nedges > 0 ? nedges : 1));
    int32_t *ev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nedges > 0 ? nedges : 1));
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!eu || !ev || !deg) { free(eu); free(ev); free(deg); return -1; }
    double ab = a + b, abc = a + b + c;
    int64_t m = 0;
    for (int64_t e = 0; e < nedges; ++e) {
        int64_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
            double r = synth_u01(k, (uint64_t)e * (uint64_t)scale + (uint64_t)l);
            int ru = r >= ab, rv = (r >= a && r < ab) || r >= abc;
            u = 2 * u + ru;
            v = 2 * v + rv;
        }
        if (u == v) continue;
        eu[m] = (int32_t)u; ev[m] = (int32_t)v; ++m;
        deg[u + 1]++; deg[v + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
    int64_t tot = deg[n];
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!tmp || !fill) { free(eu); free(ev); free(deg); free(tmp); free(fill); return -1; }
    memcpy(fill, deg, sizeof(int64_t) * (size_t)n);
    for (int64_t e = 0; e < m; ++e) {
        tmp[fill[eu[e]]++] = ev[e];
        tmp[fill[ev[e]]++] = eu[e];
    }
    free(eu); free(ev); free(fill);
    int64_t out = 0;
    rp[0] = 0;
    int rc = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t *row = tmp + deg[i];
        int64_t len = deg[i + 1] - deg[i];
        sort_i32(row, len);
        for (int64_t q = 0; q < len; ++q) {
            if (q > 0 && row[q] == row[q - 1]) continue;
            if (out >= cap) { rc = -2; break; }
            col[out++] = row[q];
        }
        if (rc) break;
        rp[i + 1] = out;
    }
    free(tmp); free(deg);
    return rc ? rc : out;
}

static int cmp_u64(const void *x, const void *y)
{
    const uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return a < b ? -1 : a > b;
}

/*
 * Multi-source BFS frontier matrix of a square graph A (CSR pattern, values
 * ignored): nsrc sources (the first nsrc entries of a seeded permutation of
 * the vertices); column s of the n x nsrc result holds the vertices at
 * distance exactly `level` from source s (the frontier of a breadth-first
 * search after `level` steps), values U(-1,1).  Writes out_rp[n+1] and up to
 * `cap` entries; returns the entry count, -1 on bad arguments or -2 when cap
 * is too small (call again with a larger one).
 */
int64_t synth_frontiers(int64_t n, const int64_t *rp, const int32_t *col, int32_t nsrc, int32_t level,
                        uint64_t seed, int64_t *out_rp, int32_t *out_col, double *out_val, int64_t cap)
{
    if (n <= 0 || nsrc <= 0 || nsrc > n || level < 0 || !rp || !col || !out_rp) return -1;
    int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *nxt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *seen = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t pcap = 1 << 16, np_ = 0;
    uint64_t *pairs = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)pcap);
    if (!src || !dist || !cur || !nxt || !seen || !pairs || synth_perm(n, synth_key(seed, TAG_FRONTIER), src) != 0) {
        free(src); free(dist); free(cur); free(nxt); free(seen); free(pairs);
        return -1;
    }
    for (int64_t v = 0; v < n; ++v) dist[v] = -1;
    for (int32_t s = 0; s < nsrc; ++s) {
        int64_t ncur = 1, nseen = 1;
        cur[0] = src[s];
        seen[0] = src[s];
        dist[src[s]] = 0;
        for (int32_t d = 1; d <= level && ncur > 0; ++d) {
            int64_t nn = 0;
            for (int64_t t = 0; t < ncur; ++t) {
                const int32_t u = cur[t];
                for (int64_t q = rp[u]; q < rp[u + 1]; ++q) {
                    const int32_t w = col[q];
                    if (dist[w] >= 0) continue;
                    dist[w] = d;
                    nxt[nn++] = w;
                    seen[nseen++] = w;
                }
            }
            int32_t *tmp = cur; cur = nxt; nxt = tmp;
            ncur = nn;
        }
        if (np_ + ncur > pcap) {
            while (np_ + ncur > pcap) pcap *= 2;
            uint64_t *p2 = (uint64_t *)realloc(pairs, sizeof(uint64_t) * (size_t)pcap);
            if (!p2) { free(src); free(dist); free(cur); free(nxt); free(seen); free(pairs); return -1; }
            pairs = p2;
        }
        for (int64_t t = 0; t < ncur; ++t) pairs[np_++] = (uint64_t)cur[t] * (uint64_t)nsrc + (uint64_t)s;
        for (int64_t t = 0; t < nseen; ++t) dist[seen[t]] = -1;
    }
    int64_t rc = np_;
    if (np_ <= cap) {
        qsort(pairs, (size_t)np_, sizeof(uint64_t), cmp_u64);
        const uint64_t kv = synth_key(seed, TAG_FRONTIER + 1);
        for (int64_t v = 0; v <= n; ++v) out_rp[v] = 0;
        for (int64_t t = 0; t < np_; ++t) {
            out_rp[pairs[t] / (uint64_t)nsrc + 1]++;
            out_col[t] = (int32_t)(pairs[t] % (uint64_t)nsrc);
            out_val[t] = uval(kv, pairs[t]);
        }
        for (int64_t v = 0; v < n; ++v) out_rp[v + 1] += out_rp[v];
    } else {
        rc = -2;
    }
    free(src); free(dist); free(cur); free(nxt); free(seen); free(pairs);
    return rc;
}
