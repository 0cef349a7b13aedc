"""GPU parity of the batched path: many products of uneven sizes in one
launch sequence, each compared bit for bit with the CPU oracle, and the same
launch sequence captured into a graph and replayed."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2507_21253_amd as hc  # noqa: E402


def dev(H):
    return hc.DeviceCSR.from_host(H)


def assert_same(Cg, Cr, where=""):
    np.testing.assert_array_equal(Cg.rp, Cr.rp, err_msg="row_ptr " + where)
    np.testing.assert_array_equal(Cg.col, Cr.col, err_msg="col " + where)
    np.testing.assert_array_equal(Cg.val, Cr.val, err_msg="val " + where)


def problems(seeds, n_lo=100, n_hi=4000):
    return [synth.batch_problem(s, n_lo, n_hi)[1] for s in seeds]


def check_batch(bt, hosts, refs=None):
    torch.cuda.synchronize()
    nnz = bt.status()
    for p, H in enumerate(hosts):
        ref = refs[p] if refs is not None else oracle.spgemm(H, H)
        assert nnz[p] == ref.nnz, "product %d" % p
        assert_same(bt.result(p, int(nnz[p])).to_host(), ref, "product %d" % p)


def test_batch_mixed_generators_bitwise():
    hosts = problems(range(1000, 1024))
    bt = hc.Batch([(d, d) for d in map(dev, hosts)])
    bt.run()
    check_batch(bt, hosts)


def test_batch_degenerate_members():
    # an empty product, one with empty rows, a 1x1 one, and rectangular A*B
    Z = synth.HostCSR(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0), 0, 0)
    E = synth.HostCSR(np.zeros(8, np.int64), np.zeros(0, np.int32), np.zeros(0), 7, 7)
    one = synth.from_dense(np.array([[3.0]]))
    A = synth.uniform(90, 60, 5, 11)
    B = synth.uniform(60, 130, 7, 12)
    pairs = [(Z, Z), (E, E), (one, one), (A, B), (synth.stencil(5, 9, 3), synth.stencil(5, 9, 3))]
    bt = hc.Batch([(dev(a), dev(b)) for a, b in pairs])
    bt.run()
    torch.cuda.synchronize()
    nnz = bt.status()
    for p, (a, b) in enumerate(pairs):
        ref = oracle.spgemm(a, b)
        assert nnz[p] == ref.nnz
        assert_same(bt.result(p, int(nnz[p])).to_host(), ref, "product %d" % p)


def test_batch_forced_dense_path_bitwise():
    # small shared-memory tables push the larger units onto the global-memory path
    hosts = problems(range(1100, 1108), 200, 2000) + [synth.uniform(300, 300, 30, 5)]
    bt = hc.Batch([(d, d) for d in map(dev, hosts)], hc.opts(sym_tmax_log2=7, num_tmax=96))
    bt.run()
    check_batch(bt, hosts)


def test_batch_equals_unbatched_gpu():
    hosts = problems(range(1200, 1210), 500, 6000)
    ds = [dev(H) for H in hosts]
    bt = hc.Batch([(d, d) for d in ds])
    bt.run()
    torch.cuda.synchronize()
    nnz = bt.status()
    for p, d in enumerate(ds):
        C = hc.spgemm(d, d).to_host()
        assert_same(bt.result(p, int(nnz[p])).to_host(), C, "product %d" % p)


def test_batch_of_clustered_operands_bitwise():
    hosts = problems(range(1300, 1310), 200, 3000)
    pairs = []
    for i, H in enumerate(hosts):
        plan = hc.plan_hierarchical(H, (3, 10), [2, 4, 8, 16][i % 4])
        D = dev(H)
        pairs.append((hc.cluster_build(D, plan), D))
    bt = hc.Batch(pairs)
    bt.run()
    check_batch(bt, hosts)


@pytest.mark.parametrize("sym,num", [(100, 70), (70, 50), (70, 70), (100, 50)])
def test_batch_tuned_group_options_bitwise(sym, num):
    # the table fills the autotuner picks for the benchmark's batch groups
    hosts = problems(range(1500, 1512), 200, 6000)
    bt = hc.Batch([(d, d) for d in map(dev, hosts)], hc.opts(sym_load_pct=sym, load_pct=num))
    bt.run()
    check_batch(bt, hosts)


def test_batch_clustered_tuned_options_bitwise():
    # clustered members as the tuner builds them: rows in RCM order, hierarchical clusters of at most 4
    hosts = problems(range(1520, 1528), 500, 6000)
    pairs = []
    for H in hosts:
        D = dev(H)
        plan = hc.plan_hierarchical(H, (3, 10), 4, hc.SIM_ROOT, perm_in=oracle.order_rcm(H))
        pairs.append((hc.cluster_build(D, plan), D))
    bt = hc.Batch(pairs, hc.opts(sym_load_pct=100, load_pct=70))
    bt.run()
    check_batch(bt, hosts)


def test_batch_graph_replays():
    # the whole launch sequence captured once; A's values change between
    # replays (same structure), eager work runs in between, every replay checked
    hosts = problems(range(1400, 1412), 200, 5000)
    ds = [dev(H) for H in hosts]
    bt = hc.Batch([(d, d) for d in ds])
    bt.run()                                  # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bt.run(s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep, scale in enumerate([1.0, -0.5, 2.0]):
        for d in ds:
            d.val.mul_(scale)                 # eager work between replays
        torch.cuda.synchronize()
        cur = []
        for H, d in zip(hosts, ds):
            Hs = synth.HostCSR(H.rp, H.col, d.val.cpu().numpy(), H.nrows, H.ncols)
            cur.append(oracle.spgemm(Hs, Hs))
        bt.C_col.fill_(-1)
        bt.C_val.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check_batch(bt, hosts, cur)


def test_batch_full_size_sampled_rows():
    # the full batch (512 products, seeds 1000..1511, 1e3..2e5 rows each) in the
    # launch configuration the benchmark replays; sampled rows of every product
    # are compared with the oracle row by row, and every row count is checked
    # against the closed upper bound
    hosts = [synth.batch_problem(s)[1] for s in range(1000, 1512)]
    ds = [dev(H) for H in hosts]
    bt = hc.Batch([(d, d) for d in ds])
    g = torch.cuda.CUDAGraph()
    bt.run()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bt.run(s)
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    nnz = bt.status()
    rp_all = bt.C_row_ptr.cpu().numpy()
    rng = np.random.default_rng(7)
    for p, H in enumerate(hosts):
        s0 = int(bt.seg_off[p])
        rp = rp_all[s0:s0 + H.nrows + 1]
        assert rp[0] == 0 and rp[-1] == nnz[p]
        rows = [0, H.nrows - 1] + list(rng.integers(0, H.nrows, 3))
        o0 = int(bt.out_off[p])
        for r in rows:
            ref = oracle.spgemm(H, H, (int(r), int(r) + 1))
            b, e = int(rp[r]), int(rp[r + 1])
            assert e - b == ref.nnz, "product %d row %d" % (p, r)
            np.testing.assert_array_equal(bt.C_col[o0 + b:o0 + e].cpu().numpy(), ref.col)
            np.testing.assert_array_equal(bt.C_val[o0 + b:o0 + e].cpu().numpy(), ref.val)
