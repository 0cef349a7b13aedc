// Host side of the autotuner (matrix classes, the per-class choice rule and
// the table file) and of the learned selector's model (a host copy of the
// parameters and feature normalization, and its file).  Neither touches the
// GPU.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace hcsp;

static const int kSymFill[HCSP_TUNE_NSYM] = {50, 70, 100};
static const int kNumFill[HCSP_TUNE_NNUM] = {50, 60, 70};
static const int kClusterSize[HCSP_TUNE_NMC] = {2, 4, 8};
static const int kClFill[HCSP_TUNE_NCL] = {50, 60, 70, 75, 80, 85};

struct hcsp_tune_table {
    std::map<std::string, std::vector<hcsp_tune_run>> classes;
};

struct hcsp_mlp {
    float params[HCSP_MLP_NPARAMS];
    float norm[2 * HCSP_MLP_NIN];
    std::string tag;
};

namespace {

// number of edges <= x (edges ascending)
int bucket(double x, std::initializer_list<double> edges)
{
    int n = 0;
    for (double e : edges) n += e <= x;
    return n;
}

std::string class_key(const float *f)
{
    char buf[64];
    std::snprintf(buf, sizeof buf, "rl%d_cv%d_cr%d_sim%d_loc%d", bucket(f[2], {6.0, 16.0, 40.0}),
                  bucket(f[12], {0.5, 2.0}), bucket(f[22], {1.3, 3.0}), bucket(f[21], {0.3, 0.6}),
                  bucket(f[14], {0.05}));
    return buf;
}

bool measured(double x) { return std::isfinite(x) && x > 0.0; }

// a run's time for clusters of size index i: its best measured fill (NaN if none)
double hc_best(const hcsp_tune_run &r, int i)
{
    double b = NAN;
    for (int j = 0; j < HCSP_TUNE_NCL; ++j)
        if (measured(r.hc_ms[i][j]) && !(b <= r.hc_ms[i][j])) b = r.hc_ms[i][j];
    return b;
}

// a run's best time over the plain grid and the cluster sizes
double run_best(const hcsp_tune_run &r)
{
    double b = NAN;
    for (int i = 0; i < HCSP_TUNE_NSYM; ++i)
        for (int j = 0; j < HCSP_TUNE_NNUM; ++j)
            if (measured(r.plain_ms[i][j]) && !(b <= r.plain_ms[i][j])) b = r.plain_ms[i][j];
    for (int i = 0; i < HCSP_TUNE_NMC; ++i) {
        const double h = hc_best(r, i);
        if (measured(h) && !(b <= h)) b = h;
    }
    return b;
}

// Sum over the runs of time / the run's best time; NaN unless every run
// measured the candidate.
template <class F>
double score(const std::vector<hcsp_tune_run> &runs, F time_of)
{
    double s = 0.0;
    for (const hcsp_tune_run &r : runs) {
        const double t = time_of(r), b = run_best(r);
        if (!measured(t) || !measured(b)) return NAN;
        s += t / b;
    }
    return s;
}

void defaults(hcsp_tune_choice *c)
{
    std::memset(c, 0, sizeof *c);
    c->path = 0;
    c->max_cluster = 0;
    c->best_cluster_size = 2;
    c->sym_load_pct = 70;
    c->load_pct = 60;
    c->cl_load_pct = 60;
}

// The class's choice (the rule in include/hcsp.h): the first candidate in grid
// order wins ties.
void choose(const std::vector<hcsp_tune_run> &runs, hcsp_tune_choice *c)
{
    defaults(c);
    c->runs = (int32_t)runs.size();
    if (runs.empty()) return;
    double best_plain = NAN;
    int si = -1, ni = -1;
    for (int i = 0; i < HCSP_TUNE_NSYM; ++i)
        for (int j = 0; j < HCSP_TUNE_NNUM; ++j) {
            const double s = score(runs, [&](const hcsp_tune_run &r) { return r.plain_ms[i][j]; });
            if (measured(s) && !(best_plain <= s)) {
                best_plain = s;
                si = i;
                ni = j;
            }
        }
    if (si < 0) return;  // no plain candidate measured by every run
    c->tuned = 1;
    c->sym_load_pct = kSymFill[si];
    c->load_pct = kNumFill[ni];
    double best_hc = NAN;
    int mi = -1;
    for (int i = 0; i < HCSP_TUNE_NMC; ++i) {
        const double s = score(runs, [&](const hcsp_tune_run &r) { return hc_best(r, i); });
        if (measured(s) && !(best_hc <= s)) {
            best_hc = s;
            mi = i;
        }
    }
    c->best_cluster_size = mi < 0 ? 2 : kClusterSize[mi];
    c->cl_load_pct = c->load_pct;
    if (mi >= 0) {
        double best_cl = NAN;
        for (int j = 0; j < HCSP_TUNE_NCL; ++j) {
            const double s = score(runs, [&](const hcsp_tune_run &r) { return r.hc_ms[mi][j]; });
            if (measured(s) && !(best_cl <= s)) {
                best_cl = s;
                c->cl_load_pct = kClFill[j];
            }
        }
    }
    if (mi >= 0 && best_hc < best_plain) {
        c->path = 1;
        c->max_cluster = kClusterSize[mi];
    }
}

bool valid_key(const char *key)
{
    if (!key || !*key) return false;
    for (const char *p = key; *p; ++p)
        if (*p <= ' ' || *p > '~') return false;
    return std::strlen(key) < 64;
}

}  // namespace

extern "C" {

int hcsp_tune_create(hcsp_tune_table **out)
{
    clear_error();
    if (!out) return fail(HCSP_E_INVALID, "tune_create: null output");
    *out = new (std::nothrow) hcsp_tune_table();
    return *out ? HCSP_OK : fail(HCSP_E_NOMEM, "tune_create: out of host memory");
}

int hcsp_tune_destroy(hcsp_tune_table *t)
{
    clear_error();
    delete t;
    return HCSP_OK;
}

int hcsp_tune_class(const float *features, char *key, size_t len)
{
    clear_error();
    if (!features || !key) return fail(HCSP_E_INVALID, "tune_class: null argument");
    const std::string k = class_key(features);
    if (len < k.size() + 1) return fail(HCSP_E_CAPACITY, "tune_class: key buffer too small");
    std::memcpy(key, k.c_str(), k.size() + 1);
    return HCSP_OK;
}

int hcsp_tune_add(hcsp_tune_table *t, const char *key, const hcsp_tune_run *run)
{
    clear_error();
    if (!t || !run || !valid_key(key)) return fail(HCSP_E_INVALID, "tune_add: bad argument");
    if (!measured(run_best(*run))) return fail(HCSP_E_INVALID, "tune_add: the run has no measured time");
    t->classes[key].push_back(*run);
    return HCSP_OK;
}

int hcsp_tune_get(const hcsp_tune_table *t, const char *key, hcsp_tune_choice *out)
{
    clear_error();
    if (!t || !key || !out) return fail(HCSP_E_INVALID, "tune_get: null argument");
    const auto it = t->classes.find(key);
    if (it == t->classes.end()) defaults(out);
    else choose(it->second, out);
    return HCSP_OK;
}

int hcsp_tune_lookup(const hcsp_tune_table *t, const float *features, hcsp_tune_choice *out)
{
    clear_error();
    if (!t || !features || !out) return fail(HCSP_E_INVALID, "tune_lookup: null argument");
    return hcsp_tune_get(t, class_key(features).c_str(), out);
}

int hcsp_tune_classes(const hcsp_tune_table *t, char *keys, size_t len, int32_t *count)
{
    clear_error();
    if (!t || !count) return fail(HCSP_E_INVALID, "tune_classes: null argument");
    std::string all;
    for (const auto &kv : t->classes) all += kv.first + "\n";
    *count = (int32_t)t->classes.size();
    if (keys) {
        if (len < all.size() + 1) return fail(HCSP_E_CAPACITY, "tune_classes: buffer too small");
        std::memcpy(keys, all.c_str(), all.size() + 1);
    }
    return HCSP_OK;
}

int hcsp_tune_runs(const hcsp_tune_table *t, const char *key, hcsp_tune_run *runs, int32_t cap, int32_t *count)
{
    clear_error();
    if (!t || !key || !count || cap < 0 || (cap > 0 && !runs)) return fail(HCSP_E_INVALID, "tune_runs: bad argument");
    const auto it = t->classes.find(key);
    const int32_t n = it == t->classes.end() ? 0 : (int32_t)it->second.size();
    *count = n;
    if (!runs) return HCSP_OK;  // the count only
    if (n > cap) return fail(HCSP_E_CAPACITY, "tune_runs: more runs than the buffer holds");
    for (int32_t i = 0; i < n; ++i) runs[i] = it->second[i];
    return HCSP_OK;
}

// Text file: a header line, then per class "class <key> <runs>" followed by
// one line per run: nrows nnz, the plain grid (row-major), rcm, the cluster
// grid (row-major); %.17g, "nan" where not measured.
int hcsp_tune_save(const hcsp_tune_table *t, const char *path)
{
    clear_error();
    if (!t || !path) return fail(HCSP_E_INVALID, "tune_save: null argument");
    FILE *fp = std::fopen(path, "w");
    if (!fp) return fail(HCSP_E_INVALID, std::string("tune_save: cannot open ") + path);
    std::fprintf(fp, "hcsp-tune 1 %d %d %d %d\n", HCSP_TUNE_NSYM, HCSP_TUNE_NNUM, HCSP_TUNE_NMC, HCSP_TUNE_NCL);
    for (const auto &kv : t->classes) {
        std::fprintf(fp, "class %s %d\n", kv.first.c_str(), (int)kv.second.size());
        for (const hcsp_tune_run &r : kv.second) {
            std::fprintf(fp, "%lld %lld", (long long)r.nrows, (long long)r.nnz);
            for (int i = 0; i < HCSP_TUNE_NSYM; ++i)
                for (int j = 0; j < HCSP_TUNE_NNUM; ++j) std::fprintf(fp, " %.17g", r.plain_ms[i][j]);
            std::fprintf(fp, " %.17g", r.rcm_ms);
            for (int i = 0; i < HCSP_TUNE_NMC; ++i)
                for (int j = 0; j < HCSP_TUNE_NCL; ++j) std::fprintf(fp, " %.17g", r.hc_ms[i][j]);
            std::fprintf(fp, "\n");
        }
    }
    const bool ok = std::fflush(fp) == 0 && !std::ferror(fp);
    std::fclose(fp);
    return ok ? HCSP_OK : fail(HCSP_E_INVALID, std::string("tune_save: write failed: ") + path);
}

int hcsp_tune_load(const char *path, hcsp_tune_table **out)
{
    clear_error();
    if (!path || !out) return fail(HCSP_E_INVALID, "tune_load: null argument");
    *out = nullptr;
    FILE *fp = std::fopen(path, "r");
    if (!fp) return fail(HCSP_E_INVALID, std::string("tune_load: cannot open ") + path);
    hcsp_tune_table *t = new (std::nothrow) hcsp_tune_table();
    if (!t) {
        std::fclose(fp);
        return fail(HCSP_E_NOMEM, "tune_load: out of host memory");
    }
    auto bad = [&](const char *why) {
        std::fclose(fp);
        delete t;
        return fail(HCSP_E_INVALID, std::string("tune_load: ") + path + ": " + why);
    };
    int v = 0, ns = 0, nn = 0, nm = 0, nc = 0;
    if (std::fscanf(fp, " hcsp-tune %d %d %d %d %d", &v, &ns, &nn, &nm, &nc) != 5 || v != 1 ||
        ns != HCSP_TUNE_NSYM || nn != HCSP_TUNE_NNUM || nm != HCSP_TUNE_NMC || nc != HCSP_TUNE_NCL)
        return bad("not a table of this version and grid");
    char key[64];
    int nruns = 0;
    while (true) {
        const int got = std::fscanf(fp, " class %63s %d", key, &nruns);
        if (got == EOF) break;
        if (got != 2 || nruns < 0 || !valid_key(key)) return bad("malformed class line");
        std::vector<hcsp_tune_run> &runs = t->classes[key];
        for (int r = 0; r < nruns; ++r) {
            hcsp_tune_run x;
            long long a = 0, b = 0;
            bool ok = std::fscanf(fp, " %lld %lld", &a, &b) == 2;
            x.nrows = a;
            x.nnz = b;
            for (int i = 0; ok && i < HCSP_TUNE_NSYM; ++i)
                for (int j = 0; ok && j < HCSP_TUNE_NNUM; ++j) ok = std::fscanf(fp, " %lf", &x.plain_ms[i][j]) == 1;
            ok = ok && std::fscanf(fp, " %lf", &x.rcm_ms) == 1;
            for (int i = 0; ok && i < HCSP_TUNE_NMC; ++i)
                for (int j = 0; ok && j < HCSP_TUNE_NCL; ++j) ok = std::fscanf(fp, " %lf", &x.hc_ms[i][j]) == 1;
            if (!ok) return bad("malformed run line");
            runs.push_back(x);
        }
    }
    std::fclose(fp);
    *out = t;
    return HCSP_OK;
}

// ------------------------------------------------------------ learned model
int hcsp_mlp_create(const float *params_h, const float *norm_h, const char *tag, hcsp_mlp **out)
{
    clear_error();
    if (!out) return fail(HCSP_E_INVALID, "mlp_create: null output");
    hcsp_mlp *m = new (std::nothrow) hcsp_mlp();
    if (!m) return fail(HCSP_E_NOMEM, "mlp_create: out of host memory");
    for (int i = 0; i < HCSP_MLP_NPARAMS; ++i) m->params[i] = params_h ? params_h[i] : 0.0f;
    for (int i = 0; i < HCSP_MLP_NIN; ++i) {
        m->norm[i] = norm_h ? norm_h[i] : 0.0f;
        m->norm[HCSP_MLP_NIN + i] = norm_h ? norm_h[HCSP_MLP_NIN + i] : 1.0f;
    }
    m->tag = tag ? tag : "";
    if (m->tag.find('\n') != std::string::npos || m->tag.size() > 4000) {
        delete m;
        return fail(HCSP_E_INVALID, "mlp_create: tag must be one line of at most 4000 bytes");
    }
    *out = m;
    return HCSP_OK;
}

int hcsp_mlp_destroy(hcsp_mlp *m)
{
    clear_error();
    delete m;
    return HCSP_OK;
}

int hcsp_mlp_get(const hcsp_mlp *m, float *params_h, float *norm_h, char *tag, size_t len)
{
    clear_error();
    if (!m) return fail(HCSP_E_INVALID, "mlp_get: null model");
    if (params_h) std::memcpy(params_h, m->params, sizeof m->params);
    if (norm_h) std::memcpy(norm_h, m->norm, sizeof m->norm);
    if (tag) {
        if (len < m->tag.size() + 1) return fail(HCSP_E_CAPACITY, "mlp_get: tag buffer too small");
        std::memcpy(tag, m->tag.c_str(), m->tag.size() + 1);
    }
    return HCSP_OK;
}

int hcsp_mlp_set(hcsp_mlp *m, const float *params_h, const float *norm_h)
{
    clear_error();
    if (!m) return fail(HCSP_E_INVALID, "mlp_set: null model");
    if (params_h) std::memcpy(m->params, params_h, sizeof m->params);
    if (norm_h) std::memcpy(m->norm, norm_h, sizeof m->norm);
    return HCSP_OK;
}

// Text file: header with the layer sizes, the tag line, the normalization
// (mu then sd) and the parameters, %.9g (exact for float32).
int hcsp_mlp_save(const hcsp_mlp *m, const char *path)
{
    clear_error();
    if (!m || !path) return fail(HCSP_E_INVALID, "mlp_save: null argument");
    FILE *fp = std::fopen(path, "w");
    if (!fp) return fail(HCSP_E_INVALID, std::string("mlp_save: cannot open ") + path);
    std::fprintf(fp, "hcsp-mlp 1 %d %d %d\n%s\n", HCSP_MLP_NIN, HCSP_MLP_NH, HCSP_MLP_NOUT, m->tag.c_str());
    for (int i = 0; i < 2 * HCSP_MLP_NIN; ++i) std::fprintf(fp, "%.9g%c", m->norm[i], i + 1 == 2 * HCSP_MLP_NIN ? '\n' : ' ');
    for (int i = 0; i < HCSP_MLP_NPARAMS; ++i) std::fprintf(fp, "%.9g%c", m->params[i], (i + 1) % 16 ? ' ' : '\n');
    std::fprintf(fp, "\n");
    const bool ok = std::fflush(fp) == 0 && !std::ferror(fp);
    std::fclose(fp);
    return ok ? HCSP_OK : fail(HCSP_E_INVALID, std::string("mlp_save: write failed: ") + path);
}

int hcsp_mlp_load(const char *path, hcsp_mlp **out)
{
    clear_error();
    if (!path || !out) return fail(HCSP_E_INVALID, "mlp_load: null argument");
    *out = nullptr;
    FILE *fp = std::fopen(path, "r");
    if (!fp) return fail(HCSP_E_INVALID, std::string("mlp_load: cannot open ") + path);
    hcsp_mlp *m = new (std::nothrow) hcsp_mlp();
    if (!m) {
        std::fclose(fp);
        return fail(HCSP_E_NOMEM, "mlp_load: out of host memory");
    }
    int v = 0, a = 0, b = 0, c = 0;
    bool ok = std::fscanf(fp, "hcsp-mlp %d %d %d %d", &v, &a, &b, &c) == 4 && v == 1 && a == HCSP_MLP_NIN &&
              b == HCSP_MLP_NH && c == HCSP_MLP_NOUT;
    if (ok) {
        int ch = std::fgetc(fp);  // end of the header line
        ok = ch == '\n';
        std::string tag;
        while (ok && (ch = std::fgetc(fp)) != EOF && ch != '\n') tag.push_back((char)ch);
        ok = ok && ch == '\n';
        m->tag = tag;
    }
    for (int i = 0; ok && i < 2 * HCSP_MLP_NIN; ++i) ok = std::fscanf(fp, " %f", &m->norm[i]) == 1;
    for (int i = 0; ok && i < HCSP_MLP_NPARAMS; ++i) ok = std::fscanf(fp, " %f", &m->params[i]) == 1;
    std::fclose(fp);
    if (!ok) {
        delete m;
        return fail(HCSP_E_INVALID, std::string("mlp_load: ") + path + ": not a model of this version and shape");
    }
    *out = m;
    return HCSP_OK;
}

}  // extern "C"

extern "C" int hcsp_mlp_train_step(float *params_d, const float *norm_d, const float *X_d, const int32_t *y_d,
                                   const float *t_d, int32_t B, float lam, float *act_d, float *Z_d, float *delta_d,
                                   float *loss_d, float *grad_d, float *m_d, float *v_d, int32_t step, float lr,
                                   float beta1, float beta2, float eps, void *stream)
{
    clear_error();
    if (!act_d) return fail(HCSP_E_INVALID, "mlp_train_step: the activations array is required");
    int rc = hcsp_mlp_forward(params_d, norm_d, X_d, B, Z_d, act_d, stream);
    if (rc) return rc;
    rc = hcsp_mlp_backward(params_d, act_d, Z_d, y_d, t_d, B, lam, delta_d, loss_d, grad_d, stream);
    if (rc) return rc;
    return hcsp_mlp_adam(params_d, grad_d, m_d, v_d, step, lr, beta1, beta2, eps, stream);
}
