/*
 * CPU ORACLE — test infrastructure only.
 *
 * A plain, slow, obviously-correct C implementation of what the clustered
 * SpGEMM path computes.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; the GPU library never does, and the
 * two share no code, headers or tables.
 *
 * Contents (paper sections in brackets):
 *   orc_spgemm*          Gustavson row-wise product C = A*B        [Background: SpGEMM Kernel, Fig. 1]
 *   orc_dense_product    brute-force dense triple loop (pin for the above)
 *   orc_jaccard          |Si n Sj| and |Si u Sj| of two rows        [Variable-length Clusters]
 *   orc_spgemm_count     row counts of C only (structure)           [Background, SpGEMM Kernel]
 *   orc_plan_fixed       fixed-length clusters                      [Fixed-length Clusters]
 *   orc_plan_variable    variable-length clusters                   [Alg. 2]
 *   orc_topk_candidates  SpGEMM_TopK(A, A^T, topk, jacc_th)          [Alg. 3, Hierarchical Clusters]
 *   orc_plan_hierarchical hierarchical clusters                     [Alg. 3]
 *   orc_cluster_count / orc_cluster_fill   CSR_Cluster layout        [Access Pattern and Matrix Format, Fig. csr_cluster]
 *   orc_cluster_spgemm   cluster-wise product                       [Alg. 1]
 *   orc_order_rcm / orc_order_degree   row orderings                 [Matrix Reordering, Table of reorderings]
 *
 * Numerical convention (the paper does not fix one): every output entry
 * c_ij starts at +0.0 and takes its contributions in ascending k, each by
 * one fused multiply-add; entries are kept even if their value cancels to
 * zero (the structure is the boolean product); output rows list their
 * columns in ascending order.  Compiled with -ffp-contract=off.
 *
 * Matrices are CSR: int64 row offsets, int32 strictly increasing columns,
 * float64 values.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>

/* ------------------------------------------------------------------ helpers */

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

static void sort_i32(int32_t *a, int64_t n)
{
    if (n <= 24) {
        for (int64_t i = 1; i < n; ++i) {
            int32_t x = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
            a[j + 1] = x;
        }
    } else {
        qsort(a, (size_t)n, sizeof(int32_t), cmp_i32);
    }
}

/* ------------------------------------------------ Gustavson row-wise product */

typedef struct {
    int64_t p;        /* columns of B */
    double *acc;      /* dense accumulator, one slot per column of B */
    int64_t *mark;    /* mark[j] == stamp  <=>  column j touched in the current row */
    int32_t *list;    /* touched columns of the current row */
    int64_t stamp;
} rowws;

static int rowws_init(rowws *w, int64_t p)
{
    w->p = p;
    w->acc = (double *)malloc(sizeof(double) * (size_t)(p > 0 ? p : 1));
    w->mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)(p > 0 ? p : 1));
    w->list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(p > 0 ? p : 1));
    w->stamp = 0;
    if (!w->acc || !w->mark || !w->list) return -1;
    for (int64_t j = 0; j < p; ++j) w->mark[j] = -1;
    return 0;
}

static void rowws_free(rowws *w)
{
    free(w->acc); free(w->mark); free(w->list);
}

/*
 * Row i of C = sum over stored a_ik (ascending k) of a_ik * (row k of B):
 * Gustavson's algorithm.  Returns the number of distinct columns touched and
 * leaves them sorted in w->list with their sums in w->acc.
 */
static int64_t gustavson_row(rowws *w, int64_t i,
                             const int64_t *Arp, const int32_t *Acol, const double *Aval,
                             const int64_t *Brp, const int32_t *Bcol, const double *Bval)
{
    int64_t cnt = 0, stamp = ++w->stamp;
    for (int64_t q = Arp[i]; q < Arp[i + 1]; ++q) {
        int64_t k = Acol[q];
        double a = Aval ? Aval[q] : 1.0;
        for (int64_t r = Brp[k]; r < Brp[k + 1]; ++r) {
            int32_t j = Bcol[r];
            if (w->mark[j] != stamp) {
                w->mark[j] = stamp;
                w->acc[j] = 0.0;
                w->list[cnt++] = j;
            }
            w->acc[j] = fma(a, Bval ? Bval[r] : 1.0, w->acc[j]);
        }
    }
    sort_i32(w->list, cnt);
    return cnt;
}

/*
 * C = A*B over rows [row_lo, row_hi) of A.  C_rp receives (row_hi-row_lo+1)
 * offsets starting at 0.  If C_col is NULL only C_rp is written (structure
 * count).  Returns nnz of the slice, -1 on allocation failure, -2 if `cap`
 * is too small for the output.
 */
int64_t orc_spgemm(int64_t p,
                   const int64_t *Arp, const int32_t *Acol, const double *Aval,
                   const int64_t *Brp, const int32_t *Bcol, const double *Bval,
                   int64_t row_lo, int64_t row_hi,
                   int64_t *C_rp, int32_t *C_col, double *C_val, int64_t cap)
{
    rowws w;
    if (rowws_init(&w, p)) { rowws_free(&w); return -1; }
    int64_t out = 0;
    C_rp[0] = 0;
    for (int64_t i = row_lo; i < row_hi; ++i) {
        int64_t cnt = gustavson_row(&w, i, Arp, Acol, Aval, Brp, Bcol, Bval);
        if (C_col) {
            if (out + cnt > cap) { rowws_free(&w); return -2; }
            for (int64_t t = 0; t < cnt; ++t) {
                C_col[out + t] = w.list[t];
                C_val[out + t] = w.acc[w.list[t]];
            }
        }
        out += cnt;
        C_rp[i - row_lo + 1] = out;
    }
    rowws_free(&w);
    return out;
}

/* ---------------------------------- the same product on several host threads */

typedef struct {
    int64_t p, lo, hi, phase;
    int64_t *next;    /* shared cursor: the next unclaimed row */
    const int64_t *Arp; const int32_t *Acol; const double *Aval;
    const int64_t *Brp; const int32_t *Bcol; const double *Bval;
    int64_t *C_rp; int32_t *C_col; double *C_val;
    int64_t *row_nnz;
    uint64_t *row_hash; double *row_sum;
    int rc;
} mtjob;

static uint64_t hash_cols(const int32_t *c, int64_t n)
{
    /* FNV-1a over the little-endian bytes of the sorted column list */
    uint64_t h = 0xcbf29ce484222325ULL;
    for (int64_t t = 0; t < n; ++t) {
        uint32_t v = (uint32_t)c[t];
        for (int b = 0; b < 4; ++b) { h ^= (v >> (8 * b)) & 0xffu; h *= 0x100000001b3ULL; }
    }
    return h;
}

/* Rows are handed out in chunks of MT_CHUNK from a shared cursor, so threads
 * stay busy on inputs whose work is concentrated in a few rows; each row is
 * computed exactly as by orc_spgemm. */
#define MT_CHUNK 64

static void *mt_worker(void *arg)
{
    mtjob *j = (mtjob *)arg;
    rowws w;
    if (rowws_init(&w, j->p)) { rowws_free(&w); j->rc = -1; return NULL; }
    for (;;) {
        int64_t c0 = __atomic_fetch_add(j->next, MT_CHUNK, __ATOMIC_RELAXED);
        if (c0 >= j->hi) break;
        int64_t c1 = c0 + MT_CHUNK < j->hi ? c0 + MT_CHUNK : j->hi;
        for (int64_t i = c0; i < c1; ++i) {
            int64_t cnt = gustavson_row(&w, i, j->Arp, j->Acol, j->Aval, j->Brp, j->Bcol, j->Bval);
            if (j->phase == 0) {
                j->row_nnz[i] = cnt;
            } else if (j->phase == 1) {
                int64_t o = j->C_rp[i];
                for (int64_t t = 0; t < cnt; ++t) {
                    j->C_col[o + t] = w.list[t];
                    j->C_val[o + t] = w.acc[w.list[t]];
                }
            } else {
                double s = 0.0;
                for (int64_t t = 0; t < cnt; ++t) s += w.acc[w.list[t]];
                j->row_nnz[i] = cnt;
                j->row_hash[i] = hash_cols(w.list, cnt);
                j->row_sum[i] = s;
            }
        }
    }
    rowws_free(&w);
    j->rc = 0;
    return NULL;
}

static int run_threads(int nthreads, int64_t lo, int64_t hi, mtjob proto)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    mtjob jobs[256];
    int64_t next = lo;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = proto;
        jobs[t].lo = lo;
        jobs[t].hi = hi;
        jobs[t].next = &next;
        jobs[t].rc = 0;
        if (pthread_create(&th[t], NULL, mt_worker, &jobs[t])) { nthreads = t; break; }
    }
    int rc = nthreads > 0 ? 0 : -1;
    for (int t = 0; t < nthreads; ++t) { pthread_join(th[t], NULL); if (jobs[t].rc) rc = jobs[t].rc; }
    return rc;
}

/*
 * Full product on `nthreads` host threads (rows handed out in chunks); the
 * same per-row Gustavson as orc_spgemm.  C_rp has nrows+1
 * entries.  Phase 0 counts, a host prefix sum sizes C, phase 1 fills.  If
 * C_col is NULL only C_rp is produced.  Returns nnz(C) or a negative code.
 */
int64_t orc_spgemm_mt(int64_t nrows, int64_t p,
                      const int64_t *Arp, const int32_t *Acol, const double *Aval,
                      const int64_t *Brp, const int32_t *Bcol, const double *Bval,
                      int64_t *C_rp, int32_t *C_col, double *C_val, int64_t cap, int nthreads)
{
    mtjob proto;
    memset(&proto, 0, sizeof proto);
    proto.p = p; proto.Arp = Arp; proto.Acol = Acol; proto.Aval = Aval;
    proto.Brp = Brp; proto.Bcol = Bcol; proto.Bval = Bval;
    proto.row_nnz = C_rp + 1;
    proto.phase = 0;
    if (run_threads(nthreads, 0, nrows, proto)) return -1;
    C_rp[0] = 0;
    for (int64_t i = 0; i < nrows; ++i) C_rp[i + 1] += C_rp[i];
    if (!C_col) return C_rp[nrows];
    if (C_rp[nrows] > cap) return -2;
    proto.C_rp = C_rp; proto.C_col = C_col; proto.C_val = C_val;
    proto.phase = 1;
    if (run_threads(nthreads, 0, nrows, proto)) return -1;
    return C_rp[nrows];
}

/*
 * Streaming per-row summary of C over rows [lo, hi): nnz, FNV-1a hash of the
 * sorted column list, and the sum of the row's values in ascending column
 * order.  For outputs too large to store.  Arrays are indexed by absolute row.
 */
int orc_spgemm_rowstats(int64_t p,
                        const int64_t *Arp, const int32_t *Acol, const double *Aval,
                        const int64_t *Brp, const int32_t *Bcol, const double *Bval,
                        int64_t lo, int64_t hi, int64_t *row_nnz, uint64_t *row_hash, double *row_sum,
                        int nthreads)
{
    mtjob proto;
    memset(&proto, 0, sizeof proto);
    proto.p = p; proto.Arp = Arp; proto.Acol = Acol; proto.Aval = Aval;
    proto.Brp = Brp; proto.Bcol = Bcol; proto.Bval = Bval;
    proto.row_nnz = row_nnz; proto.row_hash = row_hash; proto.row_sum = row_sum;
    proto.phase = 2;
    return run_threads(nthreads, lo, hi, proto);
}

/*
 * Structure of C = A*B only: row i's count is the number of distinct columns
 * j in the rows of B that row i of A selects (the boolean product, the first
 * phase of the two-phase product).  A bitmap over the columns of B marks the
 * columns seen in the current row; it is cleared again by walking the same
 * products.  Rows are handed out to `nthreads` threads in chunks.  Writes
 * row_nnz[lo..hi) (absolute row index); returns 0, or -1 on allocation
 * failure.
 */
typedef struct {
    int64_t p, hi, *next, *row_nnz;
    const int64_t *Arp, *Brp;
    const int32_t *Acol, *Bcol;
    int rc;
} cntjob;

static void *count_worker(void *arg)
{
    cntjob *j = (cntjob *)arg;
    uint64_t *seen = (uint64_t *)calloc((size_t)(j->p / 64 + 1), sizeof(uint64_t));
    if (!seen) { j->rc = -1; return NULL; }
    for (;;) {
        int64_t c0 = __atomic_fetch_add(j->next, MT_CHUNK, __ATOMIC_RELAXED);
        if (c0 >= j->hi) break;
        int64_t c1 = c0 + MT_CHUNK < j->hi ? c0 + MT_CHUNK : j->hi;
        for (int64_t i = c0; i < c1; ++i) {
            int64_t cnt = 0;
            for (int64_t q = j->Arp[i]; q < j->Arp[i + 1]; ++q) {
                int64_t k = j->Acol[q];
                for (int64_t r = j->Brp[k]; r < j->Brp[k + 1]; ++r) {
                    uint32_t c = (uint32_t)j->Bcol[r];
                    uint64_t bit = 1ull << (c & 63);
                    if (!(seen[c >> 6] & bit)) { seen[c >> 6] |= bit; ++cnt; }
                }
            }
            for (int64_t q = j->Arp[i]; q < j->Arp[i + 1]; ++q) {
                int64_t k = j->Acol[q];
                for (int64_t r = j->Brp[k]; r < j->Brp[k + 1]; ++r) seen[(uint32_t)j->Bcol[r] >> 6] = 0;
            }
            j->row_nnz[i] = cnt;
        }
    }
    free(seen);
    j->rc = 0;
    return NULL;
}

int orc_spgemm_count(int64_t p, const int64_t *Arp, const int32_t *Acol, const int64_t *Brp, const int32_t *Bcol,
                     int64_t lo, int64_t hi, int64_t *row_nnz, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    cntjob jobs[256];
    int64_t next = lo;
    for (int t = 0; t < nthreads; ++t) {
        cntjob z = {p, hi, &next, row_nnz, Arp, Brp, Acol, Bcol, 0};
        jobs[t] = z;
        if (pthread_create(&th[t], NULL, count_worker, &jobs[t])) { nthreads = t; break; }
    }
    int rc = nthreads > 0 ? 0 : -1;
    for (int t = 0; t < nthreads; ++t) { pthread_join(th[t], NULL); if (jobs[t].rc) rc = jobs[t].rc; }
    return rc;
}

/* Hash of a sorted column list, the same FNV-1a the row summary uses. */
uint64_t orc_hash_cols(const int32_t *c, int64_t n) { return hash_cols(c, n); }

/* ------------------------------------------------- brute-force dense product */

/*
 * Dense triple loop over n x m and m x p arrays with explicit presence
 * patterns: C[i][j] exists iff some k has A[i][k] and B[k][j] both stored;
 * its value is the fused multiply-add chain over those k in ascending order,
 * starting from +0.0.
 */
int orc_dense_product(int64_t n, int64_t m, int64_t p,
                      const double *A, const uint8_t *Ap, const double *B, const uint8_t *Bp,
                      double *C, uint8_t *Cp)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < p; ++j) {
            double c = 0.0;
            uint8_t present = 0;
            for (int64_t k = 0; k < m; ++k)
                if (Ap[i * m + k] && Bp[k * p + j]) {
                    c = fma(A[i * m + k], B[k * p + j], c);
                    present = 1;
                }
            C[i * p + j] = present ? c : 0.0;
            Cp[i * p + j] = present;
        }
    return 0;
}

/* ------------------------------------------------------------ Jaccard index */

/*
 * Jaccard similarity of rows i and j: |Si n Sj| / |Si u Sj| over their column
 * sets (Variable-length Clusters).  Returns the two integer counts; the
 * ratio is never formed in floating point.  J(empty, empty) is read as 0.
 */
void orc_jaccard(const int64_t *rp, const int32_t *col, int64_t i, int64_t j, int64_t *ov, int64_t *un)
{
    int64_t a = rp[i], ae = rp[i + 1], b = rp[j], be = rp[j + 1], o = 0;
    while (a < ae && b < be) {
        if (col[a] == col[b]) { ++o; ++a; ++b; }
        else if (col[a] < col[b]) ++a;
        else ++b;
    }
    *ov = o;
    *un = (rp[i + 1] - rp[i]) + (rp[j + 1] - rp[j]) - o;
}

/* sign of ov/un - num/den; an empty union counts as similarity 0 */
static int jac_cmp(int64_t ov, int64_t un, int64_t num, int64_t den)
{
    if (un == 0) { ov = 0; un = 1; }
    __int128 l = (__int128)ov * den, r = (__int128)un * num;
    return (l > r) - (l < r);
}

/* sign of ov1/un1 - ov2/un2 */
static int jac_cmp2(int64_t ov1, int64_t un1, int64_t ov2, int64_t un2)
{
    if (un1 == 0) { ov1 = 0; un1 = 1; }
    if (un2 == 0) { ov2 = 0; un2 = 1; }
    __int128 l = (__int128)ov1 * un2, r = (__int128)ov2 * un1;
    return (l > r) - (l < r);
}

/* ------------------------------------------------------------ cluster plans */

/*
 * Every plan works on the rows in the order given by perm_in (position p
 * holds original row perm_in[p]; NULL = identity) and reports clusters as
 * consecutive position ranges of perm_out: cluster c holds original rows
 * perm_out[cl_row_ptr[c] .. cl_row_ptr[c+1]).  Returns the cluster count.
 */

static int32_t row_at(const int32_t *perm_in, int64_t p) { return perm_in ? perm_in[p] : (int32_t)p; }

/* Fixed-length clusters: consecutive blocks of K rows; the last holds the remainder. */
int64_t orc_plan_fixed(int64_t n, int32_t K, const int32_t *perm_in, int32_t *perm_out, int64_t *cl_row_ptr)
{
    if (K < 1 || n < 0) return -1;
    int64_t c = 0;
    cl_row_ptr[0] = 0;
    for (int64_t p = 0; p < n; ++p) {
        perm_out[p] = row_at(perm_in, p);
        if ((p + 1) % K == 0 || p + 1 == n) cl_row_ptr[++c] = p + 1;
    }
    return c;
}

/*
 * Variable-length clusters (Alg. 2).  The first row of a cluster is its
 * representative; each following row joins while its Jaccard similarity to
 * the representative is at least num/den and the cluster holds fewer than
 * max_cluster rows, otherwise it starts a new cluster.  (The listing never
 * increments the size counter; it is incremented on every join here.)
 */
int64_t orc_plan_variable(int64_t n, const int64_t *rp, const int32_t *col, int64_t num, int64_t den,
                          int32_t max_cluster, const int32_t *perm_in, int32_t *perm_out, int64_t *cl_row_ptr)
{
    if (n < 0 || den <= 0 || num < 0 || max_cluster < 1) return -1;
    if (n == 0) { cl_row_ptr[0] = 0; return 0; }
    int64_t c = 0, rep = row_at(perm_in, 0), size = 1;
    cl_row_ptr[0] = 0;
    perm_out[0] = (int32_t)rep;
    for (int64_t p = 1; p < n; ++p) {
        int64_t r = row_at(perm_in, p), ov, un;
        orc_jaccard(rp, col, rep, r, &ov, &un);
        if (jac_cmp(ov, un, num, den) < 0 || size == max_cluster) {
            cl_row_ptr[++c] = p;
            rep = r;
            size = 1;
        } else {
            size += 1;
        }
        perm_out[p] = (int32_t)r;
    }
    cl_row_ptr[++c] = n;
    return c;
}

/* ------------------------------------------------------ hierarchical clusters */

typedef struct { int64_t ov, un; int32_t i, j; } cand;   /* i < j, similarity ov/un */

/* heap order: larger similarity first, then smaller i, then smaller j */
static int cand_before(const cand *x, const cand *y)
{
    int s = jac_cmp2(x->ov, x->un, y->ov, y->un);
    if (s) return s > 0;
    if (x->i != y->i) return x->i < y->i;
    return x->j < y->j;
}

typedef struct { cand *a; int64_t n, cap; } heap;

static int heap_push(heap *h, cand c)
{
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        cand *na = (cand *)realloc(h->a, sizeof(cand) * (size_t)nc);
        if (!na) return -1;
        h->a = na; h->cap = nc;
    }
    int64_t k = h->n++;
    h->a[k] = c;
    while (k > 0) {
        int64_t par = (k - 1) / 2;
        if (!cand_before(&h->a[k], &h->a[par])) break;
        cand t = h->a[k]; h->a[k] = h->a[par]; h->a[par] = t;
        k = par;
    }
    return 0;
}

static cand heap_pop(heap *h)
{
    cand top = h->a[0];
    h->a[0] = h->a[--h->n];
    int64_t k = 0;
    for (;;) {
        int64_t l = 2 * k + 1, r = l + 1, b = k;
        if (l < h->n && cand_before(&h->a[l], &h->a[b])) b = l;
        if (r < h->n && cand_before(&h->a[r], &h->a[b])) b = r;
        if (b == k) break;
        cand t = h->a[k]; h->a[k] = h->a[b]; h->a[b] = t;
        k = b;
    }
    return top;
}

/* open-addressing set of unordered pairs (i < j) */
typedef struct { uint64_t *k; int64_t cap, n; } pairset;

static uint64_t pkey(int32_t i, int32_t j) { return ((uint64_t)(uint32_t)i << 32) | (uint32_t)j; }

static uint64_t phash(uint64_t x)
{
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL; x ^= x >> 33;
    return x;
}

static int pset_has(const pairset *s, uint64_t key)
{
    int64_t m = s->cap - 1, h = (int64_t)(phash(key) & (uint64_t)m);
    while (s->k[h] != UINT64_MAX) {
        if (s->k[h] == key) return 1;
        h = (h + 1) & m;
    }
    return 0;
}

static int pset_add(pairset *s, uint64_t key);

static int pset_grow(pairset *s)
{
    pairset t;
    t.cap = s->cap ? 2 * s->cap : 1024;
    t.n = 0;
    t.k = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)t.cap);
    if (!t.k) return -1;
    memset(t.k, 0xff, sizeof(uint64_t) * (size_t)t.cap);
    for (int64_t q = 0; q < s->cap; ++q) if (s->k[q] != UINT64_MAX) pset_add(&t, s->k[q]);
    free(s->k);
    *s = t;
    return 0;
}

static int pset_add(pairset *s, uint64_t key)
{
    if (2 * (s->n + 1) > s->cap && pset_grow(s)) return -1;
    int64_t m = s->cap - 1, h = (int64_t)(phash(key) & (uint64_t)m);
    while (s->k[h] != UINT64_MAX) {
        if (s->k[h] == key) return 0;
        h = (h + 1) & m;
    }
    s->k[h] = key;
    s->n++;
    return 1;
}

/*
 * SpGEMM_TopK (Alg. 3): with every value of A taken as 1, (A A^T)_ij counts
 * the columns rows i and j share.  For each row i, every j != i with a
 * non-zero overlap gets J_ij = ov / (|Si| + |Sj| - ov); the row keeps its
 * `topk` best partners with J strictly above num/den, best first (ties to
 * the smaller j).  Rows here are positions of the perm_in order.  Writes
 * cnt[i] partners into nbr[i*topk ..], with ov/un; returns 0.
 */
int orc_topk_candidates(int64_t n, int64_t ncols, const int64_t *rp, const int32_t *col,
                        int64_t num, int64_t den, int32_t topk, const int32_t *perm_in,
                        int32_t *cnt, int32_t *nbr, int64_t *nbr_ov, int64_t *nbr_un)
{
    /* Transpose of the (position-ordered) pattern: for each column, the positions holding it. */
    int64_t *tp = (int64_t *)calloc((size_t)ncols + 1, sizeof(int64_t));
    int64_t nnz = 0;
    for (int64_t p = 0; p < n; ++p) nnz += rp[row_at(perm_in, p) + 1] - rp[row_at(perm_in, p)];
    int32_t *tr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *len = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *ovc = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!tp || !tr || !len || !ovc || !touched) { free(tp); free(tr); free(len); free(ovc); free(touched); return -1; }
    for (int64_t p = 0; p < n; ++p) {
        int32_t r = row_at(perm_in, p);
        len[p] = rp[r + 1] - rp[r];
        for (int64_t q = rp[r]; q < rp[r + 1]; ++q) tp[col[q] + 1]++;
    }
    for (int64_t c = 0; c < ncols; ++c) tp[c + 1] += tp[c];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncols > 0 ? ncols : 1));
        memcpy(fill, tp, sizeof(int64_t) * (size_t)ncols);
        for (int64_t p = 0; p < n; ++p) {
            int32_t r = row_at(perm_in, p);
            for (int64_t q = rp[r]; q < rp[r + 1]; ++q) tr[fill[col[q]]++] = (int32_t)p;
        }
        free(fill);
    }
    for (int64_t i = 0; i < n; ++i) {
        int32_t r = row_at(perm_in, i);
        int64_t nt = 0;
        for (int64_t q = rp[r]; q < rp[r + 1]; ++q) {
            int32_t c = col[q];
            for (int64_t t = tp[c]; t < tp[c + 1]; ++t) {
                int32_t j = tr[t];
                if (j == i) continue;
                if (ovc[j] == 0) touched[nt++] = j;
                ovc[j] += 1;
            }
        }
        int32_t k = 0;
        for (int64_t t = 0; t < nt; ++t) {
            int32_t j = touched[t];
            int64_t ov = ovc[j], un = len[i] + len[j] - ov;
            ovc[j] = 0;
            if (jac_cmp(ov, un, num, den) <= 0) continue;
            /* insert into the sorted top list: (J desc, j asc) */
            int32_t pos = k;
            while (pos > 0) {
                int64_t *po = &nbr_ov[i * topk + pos - 1], *pu = &nbr_un[i * topk + pos - 1];
                int s = jac_cmp2(ov, un, *po, *pu);
                if (s > 0 || (s == 0 && j < nbr[i * topk + pos - 1])) --pos;
                else break;
            }
            if (pos >= topk) continue;
            int32_t last = k < topk ? k : topk - 1;
            for (int32_t s2 = last; s2 > pos; --s2) {
                nbr[i * topk + s2] = nbr[i * topk + s2 - 1];
                nbr_ov[i * topk + s2] = nbr_ov[i * topk + s2 - 1];
                nbr_un[i * topk + s2] = nbr_un[i * topk + s2 - 1];
            }
            nbr[i * topk + pos] = j;
            nbr_ov[i * topk + pos] = ov;
            nbr_un[i * topk + pos] = un;
            if (k < topk) ++k;
        }
        cnt[i] = k;
    }
    free(tp); free(tr); free(len); free(ovc); free(touched);
    return 0;
}

#define ORC_SIM_UNION 1u

static int32_t uf_find(int32_t *parent, int32_t x)
{
    while (parent[x] != x) { parent[x] = parent[parent[x]]; x = parent[x]; }
    return x;
}

/* Column set of a cluster (root position r): union of its members' rows. */
static int64_t cluster_cols(int32_t r, const int32_t *next, const int64_t *rp, const int32_t *col,
                            const int32_t *perm_in, int64_t *mark, int64_t stamp, int32_t *out)
{
    int64_t m = 0;
    for (int32_t p = r; p >= 0; p = next[p]) {
        int32_t row = row_at(perm_in, p);
        for (int64_t q = rp[row]; q < rp[row + 1]; ++q)
            if (mark[col[q]] != stamp) { mark[col[q]] = stamp; out[m++] = col[q]; }
    }
    return m;
}

/*
 * Hierarchical clusters (Alg. 3).
 *   1. Candidate pairs from SpGEMM_TopK with topk = max_cluster - 1.
 *   2. A max-heap of the candidates (similarity, then smaller ids first) and
 *      a union-find forest, every row its own root.
 *   3. Pop until the heap is empty.  If both rows are still roots they are
 *      merged when the merged size stays within max_cluster (the smaller id
 *      becomes the root).  Otherwise the pair is lifted to its two roots;
 *      if those differ and that root pair was never a candidate, its
 *      similarity is computed and, when strictly above the threshold, the
 *      pair is pushed and recorded as a candidate.
 *   4. Clusters ordered by root (their smallest position), members ascending.
 * Similarity of a lifted pair: the two root rows' own patterns (default), or
 * with ORC_SIM_UNION the union of each cluster's member patterns.
 */
int64_t orc_plan_hierarchical(int64_t n, int64_t ncols, const int64_t *rp, const int32_t *col,
                              int64_t num, int64_t den, int32_t max_cluster, uint32_t flags,
                              const int32_t *perm_in, int32_t *perm_out, int64_t *cl_row_ptr)
{
    if (n < 0 || den <= 0 || num < 0 || max_cluster < 1) return -1;
    if (n == 0) { cl_row_ptr[0] = 0; return 0; }
    int32_t topk = max_cluster - 1;
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *size = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);   /* member lists */
    int32_t *tail = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    heap h = {0, 0, 0};
    pairset cs = {0, 0, 0};
    if (!parent || !size || !next || !tail || pset_grow(&cs)) goto fail;
    for (int64_t i = 0; i < n; ++i) { parent[i] = (int32_t)i; size[i] = 1; next[i] = -1; tail[i] = (int32_t)i; }
    if (topk > 0) {
        int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)topk);
        int64_t *nov = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * (size_t)topk);
        int64_t *nun = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * (size_t)topk);
        if (!cnt || !nbr || !nov || !nun ||
            orc_topk_candidates(n, ncols, rp, col, num, den, topk, perm_in, cnt, nbr, nov, nun)) {
            free(cnt); free(nbr); free(nov); free(nun);
            goto fail;
        }
        for (int64_t i = 0; i < n; ++i)
            for (int32_t t = 0; t < cnt[i]; ++t) {
                int32_t a = (int32_t)i, b = nbr[i * topk + t];
                if (a > b) { int32_t x = a; a = b; b = x; }
                int added = pset_add(&cs, pkey(a, b));
                if (added < 0) { free(cnt); free(nbr); free(nov); free(nun); goto fail; }
                if (added) {
                    cand c = {nov[i * topk + t], nun[i * topk + t], a, b};
                    if (heap_push(&h, c)) { free(cnt); free(nbr); free(nov); free(nun); goto fail; }
                }
            }
        free(cnt); free(nbr); free(nov); free(nun);
    }
    {
        int64_t *mark = NULL, stamp = 0;
        int32_t *ca = NULL, *cb = NULL;
        if (flags & ORC_SIM_UNION) {
            mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncols > 0 ? ncols : 1));
            ca = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncols > 0 ? ncols : 1));
            cb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncols > 0 ? ncols : 1));
            if (!mark || !ca || !cb) { free(mark); free(ca); free(cb); goto fail; }
            for (int64_t c = 0; c < ncols; ++c) mark[c] = -1;
        }
        while (h.n > 0) {
            cand top = heap_pop(&h);
            int32_t i = top.i, j = top.j;
            if (parent[i] == i && parent[j] == j) {
                if (size[i] + size[j] <= max_cluster) {
                    int32_t r = i < j ? i : j, o = i < j ? j : i;
                    parent[o] = r;
                    size[r] += size[o];
                    next[tail[r]] = o;
                    tail[r] = tail[o];
                }
                continue;
            }
            int32_t ri = uf_find(parent, i), rj = uf_find(parent, j);
            if (ri == rj) continue;
            int32_t a = ri < rj ? ri : rj, b = ri < rj ? rj : ri;
            if (pset_has(&cs, pkey(a, b))) continue;
            int64_t ov, un;
            if (flags & ORC_SIM_UNION) {
                int64_t na = cluster_cols(a, next, rp, col, perm_in, mark, ++stamp, ca);
                int64_t nb = cluster_cols(b, next, rp, col, perm_in, mark, ++stamp, cb);
                int64_t o = 0;
                for (int64_t t = 0; t < na; ++t) if (mark[ca[t]] == stamp) ++o;
                ov = o; un = na + nb - o;
            } else {
                orc_jaccard(rp, col, row_at(perm_in, a), row_at(perm_in, b), &ov, &un);
            }
            if (jac_cmp(ov, un, num, den) > 0) {
                cand c = {ov, un, a, b};
                if (heap_push(&h, c) || pset_add(&cs, pkey(a, b)) < 0) { free(mark); free(ca); free(cb); goto fail; }
            }
        }
        free(mark); free(ca); free(cb);
    }
    {
        /* members are positions; list each cluster's positions ascending, then map to rows */
        int64_t c = 0, p = 0;
        cl_row_ptr[0] = 0;
        for (int64_t r = 0; r < n; ++r) {
            if (parent[r] != r) continue;
            int64_t b = p;
            for (int32_t m = (int32_t)r; m >= 0; m = next[m]) perm_out[p++] = m;
            for (int64_t x = b + 1; x < p; ++x) {
                int32_t v = perm_out[x];
                int64_t y = x - 1;
                while (y >= b && perm_out[y] > v) { perm_out[y + 1] = perm_out[y]; --y; }
                perm_out[y + 1] = v;
            }
            cl_row_ptr[++c] = p;
        }
        for (int64_t q = 0; q < n; ++q) perm_out[q] = row_at(perm_in, perm_out[q]);
        free(parent); free(size); free(next); free(tail); free(h.a); free(cs.k);
        return c;
    }
fail:
    free(parent); free(size); free(next); free(tail); free(h.a); free(cs.k);
    return -1;
}

/* ------------------------------------------------------- CSR_Cluster layout */

/*
 * CSR_Cluster of A for clusters given as position ranges of perm
 * (Access Pattern and Matrix Format).  For cluster c of s rows:
 *   cl_col[cl_col_ptr[c] ..]  the sorted union of its rows' columns;
 *   cl_mask[t]                bit l set iff member row l stores column cl_col[t];
 *   cl_val[cl_val_ptr[c] + t*s + l]  that value, or +0.0 as a placeholder.
 * orc_cluster_count fills cl_col_ptr and cl_val_ptr (ncl+1 entries each);
 * orc_cluster_fill fills the rest.  Clusters are limited to 16 rows.
 */
static int64_t cluster_union(int64_t c, const int64_t *rp, const int32_t *col, const int32_t *perm,
                             const int64_t *cl_row_ptr, int32_t *ucol, uint16_t *umask, int64_t *cur)
{
    int64_t b = cl_row_ptr[c], s = cl_row_ptr[c + 1] - b, m = 0;
    for (int64_t l = 0; l < s; ++l) cur[l] = rp[perm[b + l]];
    for (;;) {
        int64_t best = INT64_MAX;
        for (int64_t l = 0; l < s; ++l) {
            int32_t r = perm[b + l];
            if (cur[l] < rp[r + 1] && col[cur[l]] < best) best = col[cur[l]];
        }
        if (best == INT64_MAX) break;
        uint16_t mk = 0;
        for (int64_t l = 0; l < s; ++l) {
            int32_t r = perm[b + l];
            if (cur[l] < rp[r + 1] && col[cur[l]] == best) { mk |= (uint16_t)(1u << l); }
        }
        if (ucol) { ucol[m] = (int32_t)best; umask[m] = mk; }
        ++m;
        for (int64_t l = 0; l < s; ++l) {
            int32_t r = perm[b + l];
            if (cur[l] < rp[r + 1] && col[cur[l]] == best) cur[l]++;
        }
    }
    return m;
}

int orc_cluster_count(int64_t ncl, const int64_t *rp, const int32_t *col, const int32_t *perm,
                      const int64_t *cl_row_ptr, int64_t *cl_col_ptr, int64_t *cl_val_ptr)
{
    int64_t cur[16];
    cl_col_ptr[0] = 0; cl_val_ptr[0] = 0;
    for (int64_t c = 0; c < ncl; ++c) {
        int64_t s = cl_row_ptr[c + 1] - cl_row_ptr[c];
        if (s < 1 || s > 16) return -1;
        int64_t m = cluster_union(c, rp, col, perm, cl_row_ptr, NULL, NULL, cur);
        cl_col_ptr[c + 1] = cl_col_ptr[c] + m;
        cl_val_ptr[c + 1] = cl_val_ptr[c] + m * s;
    }
    return 0;
}

int orc_cluster_fill(int64_t ncl, const int64_t *rp, const int32_t *col, const double *val, const int32_t *perm,
                     const int64_t *cl_row_ptr, const int64_t *cl_col_ptr, const int64_t *cl_val_ptr,
                     int32_t *cl_col, uint16_t *cl_mask, double *cl_val)
{
    int64_t cur[16];
    for (int64_t c = 0; c < ncl; ++c) {
        int64_t b = cl_row_ptr[c], s = cl_row_ptr[c + 1] - b, o = cl_col_ptr[c];
        if (s < 1 || s > 16) return -1;
        int64_t m = cluster_union(c, rp, col, perm, cl_row_ptr, cl_col + o, cl_mask + o, cur);
        if (m != cl_col_ptr[c + 1] - o) return -2;
        double *v = cl_val + cl_val_ptr[c];
        for (int64_t t = 0; t < m * s; ++t) v[t] = 0.0;
        for (int64_t l = 0; l < s; ++l) {
            int32_t r = perm[b + l];
            int64_t t = 0;
            for (int64_t q = rp[r]; q < rp[r + 1]; ++q) {
                while (cl_col[o + t] != col[q]) ++t;
                v[t * s + l] = val[q];
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------- cluster-wise product */

/*
 * Alg. 1 over a CSR_Cluster operand: for each cluster, for each union column
 * k in ascending order, for each b_kj of row k of B, for each member row l
 * whose mask bit is set: c_lj = fma(a_lk, b_kj, c_lj).  Row l of the cluster
 * is written to output row perm[...] of C (A's original order), columns
 * ascending.  C_rp has nrows+1 entries.  With C_col NULL only C_rp is made.
 * Returns nnz(C), or a negative code.
 */
int64_t orc_cluster_spgemm(int64_t nrows, int64_t p, int64_t ncl,
                           const int64_t *cl_row_ptr, const int32_t *perm,
                           const int64_t *cl_col_ptr, const int32_t *cl_col, const uint16_t *cl_mask,
                           const int64_t *cl_val_ptr, const double *cl_val,
                           const int64_t *Brp, const int32_t *Bcol, const double *Bval,
                           int64_t *C_rp, int32_t *C_col, double *C_val, int64_t cap)
{
    double *acc = (double *)malloc(sizeof(double) * 16 * (size_t)(p > 0 ? p : 1));
    int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * 16 * (size_t)(p > 0 ? p : 1));
    int32_t *list = (int32_t *)malloc(sizeof(int32_t) * 16 * (size_t)(p > 0 ? p : 1));
    int64_t cnt[16];
    if (!acc || !mark || !list) { free(acc); free(mark); free(list); return -1; }
    for (int64_t t = 0; t < 16 * p; ++t) mark[t] = -1;
    int pass_rc = 0;
    int64_t stamp = 0;
    for (int pass = 0; pass < (C_col ? 2 : 1) && !pass_rc; ++pass) {
        if (pass == 1) {
            /* C_rp currently holds per-row counts at [r+1]; make offsets */
            C_rp[0] = 0;
            for (int64_t r = 0; r < nrows; ++r) C_rp[r + 1] += C_rp[r];
            if (C_rp[nrows] > cap) { pass_rc = -2; break; }
        } else {
            for (int64_t r = 0; r <= nrows; ++r) C_rp[r] = 0;
        }
        for (int64_t c = 0; c < ncl; ++c) {
            int64_t b = cl_row_ptr[c], s = cl_row_ptr[c + 1] - b;
            ++stamp;
            for (int64_t l = 0; l < s; ++l) cnt[l] = 0;
            for (int64_t t = cl_col_ptr[c]; t < cl_col_ptr[c + 1]; ++t) {
                int64_t k = cl_col[t];
                uint16_t mk = cl_mask[t];
                const double *a = cl_val + cl_val_ptr[c] + (t - cl_col_ptr[c]) * s;
                for (int64_t r = Brp[k]; r < Brp[k + 1]; ++r) {
                    int32_t j = Bcol[r];
                    for (int64_t l = 0; l < s; ++l) {
                        if (!((mk >> l) & 1)) continue;
                        int64_t x = l * p + j;
                        if (mark[x] != stamp) {
                            mark[x] = stamp;
                            acc[x] = 0.0;
                            list[l * p + cnt[l]++] = j;
                        }
                        acc[x] = fma(a[l], Bval[r], acc[x]);
                    }
                }
            }
            for (int64_t l = 0; l < s; ++l) {
                int64_t row = perm[b + l];
                if (pass == 0) { C_rp[row + 1] = cnt[l]; continue; }
                sort_i32(list + l * p, cnt[l]);
                int64_t o = C_rp[row];
                for (int64_t q = 0; q < cnt[l]; ++q) {
                    int32_t j = list[l * p + q];
                    C_col[o + q] = j;
                    C_val[o + q] = acc[l * p + j];
                }
            }
        }
    }
    if (!C_col && !pass_rc) {
        for (int64_t r = 0; r < nrows; ++r) C_rp[r + 1] += C_rp[r];
    }
    free(acc); free(mark); free(list);
    return pass_rc ? pass_rc : C_rp[nrows];
}

/* ------------------------------------------------------------- row orderings */
/* Reverse Cuthill-McKee [Sec. "Matrix Reordering": bandwidth reduction by
 * breadth-first search].  The paper takes RCM from a library and states no
 * details; this follows the textbook procedure:
 *   graph   = pattern of A + A^T, diagonal dropped
 *   start   = per connected component, the unvisited vertex of least degree
 *             (ties: least id), moved to a pseudo-peripheral vertex: from the
 *             current start build the breadth-first level structure, take the
 *             least-(degree, id) vertex x of its last level; if x's level
 *             structure is deeper, x becomes the start and the step repeats
 *   visit   = breadth-first; a dequeued vertex appends its unvisited
 *             neighbours in ascending (degree, id)
 *   result  = the concatenated visit order, reversed.
 * perm[p] = the vertex placed at position p.  Returns 0, or -1 on
 * allocation failure. */
static const int64_t *g_deg;

static int cmp_deg_id(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    if (g_deg[a] != g_deg[b]) return g_deg[a] < g_deg[b] ? -1 : 1;
    return (a > b) - (a < b);
}

/* breadth-first levels from s, over vertices whose stamp differs from mark;
 * returns the depth and the least-(degree, id) vertex of the deepest level */
static int64_t orc_levels(int64_t s, const int64_t *gp, const int32_t *ga, const int64_t *deg, int32_t *stamp,
                          int32_t mark, int32_t *queue, int32_t *lastv)
{
    int64_t head = 0, tail = 0, depth = 0;
    queue[tail++] = (int32_t)s;
    stamp[s] = mark;
    while (head < tail) {
        int64_t end = tail;
        int32_t best = queue[head];
        depth++;
        for (; head < end; ++head) {
            int32_t u = queue[head];
            if (deg[u] < deg[best] || (deg[u] == deg[best] && u < best)) best = u;
            for (int64_t p = gp[u]; p < gp[u + 1]; ++p) {
                int32_t w = ga[p];
                if (stamp[w] != mark) { stamp[w] = mark; queue[tail++] = w; }
            }
        }
        *lastv = best;
    }
    return depth;
}

int orc_order_rcm(int64_t n, const int64_t *rp, const int32_t *col, int32_t *perm)
{
    int64_t *cnt = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *gp = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *deg = calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *stamp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *queue = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *order = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *byd = malloc(sizeof(int32_t) * (size_t)(n + 1));
    char *done = calloc((size_t)n + 1, 1);
    int32_t *raw = NULL, *ga = NULL;
    int rc = -1;
    if (!cnt || !gp || !deg || !stamp || !queue || !order || !byd || !done) goto out;
    /* symmetric adjacency with duplicates, then sorted and deduplicated */
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (col[p] != i) { cnt[i]++; cnt[col[p]]++; }
    int64_t tot = 0;
    for (int64_t i = 0; i < n; ++i) { int64_t c = cnt[i]; cnt[i] = tot; tot += c; }
    cnt[n] = tot;
    raw = malloc(sizeof(int32_t) * (size_t)(tot + 1));
    ga = malloc(sizeof(int32_t) * (size_t)(tot + 1));
    if (!raw || !ga) goto out;
    {
        int64_t *fill = gp;  /* borrowed as a cursor, rebuilt below */
        for (int64_t i = 0; i < n; ++i) fill[i] = cnt[i];
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
                if (col[p] != i) { raw[fill[i]++] = col[p]; raw[fill[col[p]]++] = (int32_t)i; }
    }
    gp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t *a = raw + cnt[i];
        int64_t m = cnt[i + 1] - cnt[i], k = 0;
        sort_i32(a, m);
        for (int64_t q = 0; q < m; ++q)
            if (q == 0 || a[q] != a[q - 1]) a[k++] = a[q];
        deg[i] = k;
    }
    for (int64_t i = 0; i < n; ++i) {
        gp[i + 1] = gp[i] + deg[i];
        memcpy(ga + gp[i], raw + cnt[i], sizeof(int32_t) * (size_t)deg[i]);
    }
    g_deg = deg;
    for (int64_t i = 0; i < n; ++i) qsort(ga + gp[i], (size_t)deg[i], sizeof(int32_t), cmp_deg_id);
    for (int64_t i = 0; i < n; ++i) { byd[i] = (int32_t)i; stamp[i] = -1; }
    qsort(byd, (size_t)n, sizeof(int32_t), cmp_deg_id);
    {
        int64_t placed = 0, next = 0;
        int32_t mark = 0;
        while (placed < n) {
            while (done[byd[next]]) next++;
            int32_t start = byd[next], x;
            int64_t depth = orc_levels(start, gp, ga, deg, stamp, ++mark, queue, &x);
            for (;;) {
                int32_t y;
                int64_t d2 = orc_levels(x, gp, ga, deg, stamp, ++mark, queue, &y);
                if (d2 <= depth) break;
                start = x; depth = d2; x = y;
            }
            int64_t head = placed;
            order[placed++] = start;
            done[start] = 1;
            while (head < placed) {
                int32_t u = order[head++];
                for (int64_t p = gp[u]; p < gp[u + 1]; ++p)
                    if (!done[ga[p]]) { done[ga[p]] = 1; order[placed++] = ga[p]; }
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) perm[i] = order[n - 1 - i];
    rc = 0;
out:
    free(cnt); free(gp); free(deg); free(stamp); free(queue); free(order); free(byd); free(done);
    free(raw); free(ga);
    return rc;
}

/* Degree order [Sec. "Matrix Reordering": rows in descending order of their
 * degree]: descending row length, equal lengths in ascending row id. */
int orc_order_degree(int64_t n, const int64_t *rp, int32_t *perm)
{
    /* counting sort by length, longest first, stable in row id */
    int64_t maxl = 0;
    for (int64_t i = 0; i < n; ++i) if (rp[i + 1] - rp[i] > maxl) maxl = rp[i + 1] - rp[i];
    int64_t *start = calloc((size_t)maxl + 2, sizeof(int64_t));
    if (!start) return -1;
    for (int64_t i = 0; i < n; ++i) start[maxl - (rp[i + 1] - rp[i]) + 1]++;
    for (int64_t l = 0; l <= maxl; ++l) start[l + 1] += start[l];
    for (int64_t i = 0; i < n; ++i) perm[start[maxl - (rp[i + 1] - rp[i])]++] = (int32_t)i;
    free(start);
    return 0;
}
