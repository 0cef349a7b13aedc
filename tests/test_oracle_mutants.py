"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of ``oracle/oracle.c`` (a
dropped term, a wrong sign, index or tie order, a transposed layout, the
algorithm listing's own slip), builds it with gcc into a temporary
directory, and runs the oracle's pin tests (``tests/test_oracle.py``)
against that build in a child process; or in the float64 MLP oracle
(``oracle/mlp.py``), whose mutated source replaces the module's functions in
a child process that then runs ``tests/test_oracle_mlp.py``.  Every mistake
must make some pin fail; the unmodified sources must pass.  Nothing here
touches the GPU library.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, text in oracle.c, replacement, which occurrence)
MUTANTS = [
    ("Gustavson: unfused multiply-add",
     "w->acc[j] = fma(a, Bval ? Bval[r] : 1.0, w->acc[j]);",
     "w->acc[j] = a * (Bval ? Bval[r] : 1.0) + w->acc[j];", 0),
    ("Gustavson: last entry of each row of B dropped",
     "for (int64_t r = Brp[k]; r < Brp[k + 1]; ++r) {",
     "for (int64_t r = Brp[k]; r < Brp[k + 1] - 1; ++r) {", 0),
    ("Gustavson: products in descending k",
     "for (int64_t q = Arp[i]; q < Arp[i + 1]; ++q) {",
     "for (int64_t q = Arp[i + 1] - 1; q >= Arp[i]; --q) {", 0),
    ("Gustavson: short rows sorted descending",
     "while (j >= 0 && a[j] > x)", "while (j >= 0 && a[j] < x)", 0),
    ("Jaccard: union without subtracting the overlap",
     "*un = (rp[i + 1] - rp[i]) + (rp[j + 1] - rp[j]) - o;",
     "*un = (rp[i + 1] - rp[i]) + (rp[j + 1] - rp[j]);", 0),
    ("Jaccard: merge advances the wrong row",
     "else if (col[a] < col[b]) ++a;", "else if (col[a] < col[b]) ++b;", 0),
    ("similarity order: cross products transposed",
     "__int128 l = (__int128)ov1 * un2, r = (__int128)ov2 * un1;",
     "__int128 l = (__int128)ov1 * un1, r = (__int128)ov2 * un2;", 0),
    ("threshold: numerator and denominator swapped",
     "__int128 l = (__int128)ov * den, r = (__int128)un * num;",
     "__int128 l = (__int128)ov * num, r = (__int128)un * den;", 0),
    ("fixed-length: blocks of K + 1 rows",
     "if ((p + 1) % K == 0 || p + 1 == n)", "if ((p + 1) % (K + 1) == 0 || p + 1 == n)", 0),
    ("Alg. 2: cluster size never incremented (as printed)",
     "size += 1;", "size += 0;", 0),
    ("Alg. 2: a row at the threshold starts a new cluster",
     "if (jac_cmp(ov, un, num, den) < 0 || size == max_cluster) {",
     "if (jac_cmp(ov, un, num, den) <= 0 || size == max_cluster) {", 0),
    ("Alg. 2: a joining row becomes the representative",
     "size += 1;", "size += 1; rep = r;", 0),
    ("top-k: threshold not strict",
     "if (jac_cmp(ov, un, num, den) <= 0) continue;", "if (jac_cmp(ov, un, num, den) < 0) continue;", 0),
    ("top-k: ties by larger column first",
     "if (s > 0 || (s == 0 && j < nbr[i * topk + pos - 1])) --pos;",
     "if (s > 0 || (s == 0 && j > nbr[i * topk + pos - 1])) --pos;", 0),
    ("Alg. 3 heap: lower similarity first",
     "if (s) return s > 0;", "if (s) return s < 0;", 0),
    ("Alg. 3 heap: ties by larger first id",
     "if (x->i != y->i) return x->i < y->i;", "if (x->i != y->i) return x->i > y->i;", 0),
    ("Alg. 3 union: cap exceeded by one",
     "if (size[i] + size[j] <= max_cluster) {", "if (size[i] + size[j] <= max_cluster + 1) {", 0),
    ("Alg. 3 union: larger id becomes the root",
     "int32_t r = i < j ? i : j, o = i < j ? j : i;", "int32_t r = i < j ? j : i, o = i < j ? i : j;", 0),
    ("Alg. 3 lifted pairs: threshold not strict",
     "if (jac_cmp(ov, un, num, den) > 0) {", "if (jac_cmp(ov, un, num, den) >= 0) {", 0),
    ("Alg. 3 union reading: members other than the root ignored",
     "for (int32_t p = r; p >= 0; p = next[p]) {", "for (int32_t p = r; p >= 0; p = -1) {", 0),
    ("CSR_Cluster: mask bits in reverse member order",
     "mk |= (uint16_t)(1u << l);", "mk |= (uint16_t)(1u << (s - 1 - l));", 0),
    ("CSR_Cluster: values row by row instead of column by column",
     "v[t * s + l] = val[q];", "v[l * m + t] = val[q];", 0),
    ("Alg. 1: mask ignored (placeholders become entries)",
     "if (!((mk >> l) & 1)) continue;", "if (0) continue;", 0),
    ("Alg. 1: unfused multiply-add",
     "acc[x] = fma(a[l], Bval[r], acc[x]);", "acc[x] = a[l] * Bval[r] + acc[x];", 0),
    ("RCM: Cuthill-McKee order not reversed",
     "perm[i] = order[n - 1 - i];", "perm[i] = order[i];", 0),
    ("RCM: no pseudo-peripheral start",
     "if (d2 <= depth) break;", "if (d2 <= depth || 1) break;", 0),
    ("RCM: neighbours visited in id order",
     "for (int64_t i = 0; i < n; ++i) qsort(ga + gp[i], (size_t)deg[i], sizeof(int32_t), cmp_deg_id);",
     ";", 0),
    ("row counts: repeated columns counted again",
     "if (!(seen[c >> 6] & bit)) { seen[c >> 6] |= bit; ++cnt; }", "{ seen[c >> 6] |= bit; ++cnt; }", 0),
    ("row counts: marks not cleared between rows",
     "for (int64_t r = j->Brp[k]; r < j->Brp[k + 1]; ++r) seen[(uint32_t)j->Bcol[r] >> 6] = 0;", ";", 0),
    ("row statistics: value sum skips the last entry",
     "for (int64_t t = 0; t < cnt; ++t) s += w.acc[w.list[t]];",
     "for (int64_t t = 0; t + 1 < cnt; ++t) s += w.acc[w.list[t]];", 0),
    ("degree order: equal lengths by descending id",
     "for (int64_t i = 0; i < n; ++i) perm[start[maxl - (rp[i + 1] - rp[i])]++] = (int32_t)i;",
     "for (int64_t i = n - 1; i >= 0; --i) perm[start[maxl - (rp[i + 1] - rp[i])]++] = (int32_t)i;", 0),
]


def mutate(src, old, new, k):
    pos = -1
    for _ in range(k + 1):
        pos = src.find(old, pos + 1)
        assert pos >= 0, "mutation site not found: %r" % old
    return src[:pos] + new + src[pos + len(old):]


def run_pins(tmp_path, source, tag):
    d = tmp_path / tag
    d.mkdir()
    c = d / "oracle.c"
    c.write_text(source)
    so = d / "liboracle.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so), str(c),
                           "-lm", "-lpthread"])
    env = dict(os.environ, HCSP_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle.py"), "-x", "-q",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    return r.returncode, r.stdout[-2000:] + r.stderr[-2000:]


def test_unmodified_oracle_passes_its_pins(tmp_path):
    rc, out = run_pins(tmp_path, open(SRC).read(), "original")
    assert rc == 0, out


@pytest.mark.parametrize("name,old,new,k", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new, k):
    rc, out = run_pins(tmp_path, mutate(open(SRC).read(), old, new, k), "mutant")
    # 1: some test failed (a crash of the child counts too: negative status)
    assert rc == 1 or rc < 0, "%s: no pin failed (status %d)\n%s" % (name, rc, out)


MLP_SRC = os.path.join(ROOT, "oracle", "mlp.py")

MLP_MUTANTS = [
    ("forward: first-layer ReLU missing", "h1 = np.maximum(a1, 0.0)", "h1 = a1"),
    ("forward: inputs multiplied by the spread", "xn = (np.asarray(X, np.float64) - mu) / sd",
     "xn = (np.asarray(X, np.float64) - mu) * sd"),
    ("loss: regression term not weighted", "ce.mean() + lam * np.mean(", "ce.mean() + np.mean("),
    ("gradient: label not subtracted from the softmax", "dz[np.arange(B), y] -= 1.0", "dz[np.arange(B), y] -= 0.0"),
    ("gradient: regression factor 2 missing", "dz[:, NCLS] = 2.0 * lam *", "dz[:, NCLS] = lam *"),
    ("gradient: second layer masked by the first layer's signs", "da2 = dh2 * (a2 > 0)", "da2 = dh2 * (a1 > 0)"),
    ("gradient: first-layer bias before the ReLU mask", 'g["b1"] = da1.sum(axis=0)', 'g["b1"] = dh1.sum(axis=0)'),
    ("Adam: no bias correction", "mh = m / (1 - b1 ** step)", "mh = m"),
    ("Adam: second moment of |g| instead of g squared", "v = b2 * v + (1 - b2) * g * g",
     "v = b2 * v + (1 - b2) * np.abs(g)"),
]


def run_mlp_pins(source):
    prog = ("import sys; sys.path.insert(0, %r); import oracle.mlp as m; "
            "exec(compile(sys.stdin.read(), 'mlp.py', 'exec'), m.__dict__); import pytest; "
            "sys.exit(pytest.main([%r, '-x', '-q', '-p', 'no:cacheprovider']))"
            % (ROOT, os.path.join(ROOT, "tests", "test_oracle_mlp.py")))
    r = subprocess.run([sys.executable, "-c", prog], cwd=ROOT, input=source, capture_output=True, text=True,
                       timeout=300)
    return r.returncode, r.stdout[-2000:] + r.stderr[-2000:]


def test_unmodified_mlp_oracle_passes_its_pins():
    rc, out = run_mlp_pins(open(MLP_SRC).read())
    assert rc == 0, out


@pytest.mark.parametrize("name,old,new", MLP_MUTANTS, ids=[m[0] for m in MLP_MUTANTS])
def test_planted_mlp_mistake_fails_a_pin(name, old, new):
    rc, out = run_mlp_pins(mutate(open(MLP_SRC).read(), old, new, 0))
    assert rc == 1 or rc < 0, "%s: no pin failed (status %d)\n%s" % (name, rc, out)
