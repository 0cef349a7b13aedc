"""GPU parity of the predicted-size product: whatever the predicted
compression ratio, C equals the oracle's bit for bit, and the rows recomputed
through the exact symbolic phase are exactly those whose true count exceeds
their predicted capacity."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2507_21253_amd as hc  # noqa: E402


def inputs():
    yield "stencil27_relabelled", synth.workload_stencil27(12, 2, 3)[0], None
    yield "uniform", synth.uniform(900, 700, 9, 3), synth.uniform(700, 800, 12, 4)
    rng = np.random.default_rng(5)
    dens = rng.choice([0.0, 0.02, 0.1, 0.5], size=300)
    pat = rng.random((300, 300)) < dens[:, None]
    R = synth.from_dense(np.where(pat, rng.uniform(-1, 1, (300, 300)), 0.0), pat)
    yield "ragged", R, None


@pytest.mark.parametrize("ratio", [0.02, 0.15, 0.5, 1.0])
def test_predicted_product_bitwise_and_overflow_count(ratio):
    for name, A, B in inputs():
        B = A if B is None else B
        ref = oracle.spgemm(A, B)
        P = hc.PredictedProduct(hc.DeviceCSR.from_host(A), hc.DeviceCSR.from_host(B), ratio)
        C = P.run().to_host()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(C.rp, ref.rp, err_msg=name)
        np.testing.assert_array_equal(C.col, ref.col, err_msg=name)
        np.testing.assert_array_equal(C.val, ref.val, err_msg=name)
        ub = np.zeros(A.nrows, np.int64)
        bl = np.diff(B.rp)
        np.add.at(ub, np.repeat(np.arange(A.nrows), np.diff(A.rp)), bl[A.col])
        cap = np.minimum(ub, np.ceil(ub.astype(np.float32) * np.float32(ratio)).astype(np.int64))
        cap = np.where(ub > 0, np.maximum(cap, 1), 0)
        # rows whose true count exceeds the capacity, plus rows whose capacity needs a table larger than
        # shared memory holds (8192 slots on a 160 KiB device; the bounds allow 6144 too)
        over = np.diff(ref.rp) > cap
        need = (cap * 100 + 59) // 60
        lo = int(np.sum(over | (need > 8192)))
        hi = int(np.sum(over | (need > 6144)))
        assert lo <= P.n_overflow <= hi, (name, P.n_overflow, lo, hi)
        if not np.any(need > 6144):
            assert P.n_overflow == int(np.sum(over)), name
        assert P.products == int(ub.sum())


def test_predicted_product_with_global_memory_rows():
    # rows too long for shared memory always take the exact path
    R = synth.rmat(11, 16, 0.57, 0.19, 0.19, 4)
    ref = oracle.spgemm(R, R)
    P = hc.PredictedProduct(hc.DeviceCSR.from_host(R), hc.DeviceCSR.from_host(R), 0.6,
                            hc.opts(sym_tmax_log2=8, num_tmax=192))
    C = P.run().to_host()
    np.testing.assert_array_equal(C.rp, ref.rp)
    np.testing.assert_array_equal(C.col, ref.col)
    np.testing.assert_array_equal(C.val, ref.val)
    assert P.n_overflow > 0


def test_predicted_capacity_error_is_reported():
    A = synth.uniform(200, 200, 6, 1)
    P = hc.PredictedProduct(hc.DeviceCSR.from_host(A), hc.DeviceCSR.from_host(A), 0.5, capacity=10)
    with pytest.raises(hc.HcspError) as e:
        P.run()
    assert e.value.status == -5


def test_per_row_capacities_bitwise_and_overflow_rows():
    rng = np.random.default_rng(11)
    for name, A, B in inputs():
        B = A if B is None else B
        ref = oracle.spgemm(A, B)
        counts = np.diff(ref.rp)
        ub = np.zeros(A.nrows, np.int64)
        np.add.at(ub, np.repeat(np.arange(A.nrows), np.diff(A.rp)), np.diff(B.rp)[A.col])
        Ad, Bd = hc.DeviceCSR.from_host(A), hc.DeviceCSR.from_host(B)
        # exact counts: nothing overflows; a seeded third of the rows one short: exactly those overflow
        short = (rng.random(A.nrows) < 1 / 3) & (counts >= 2)
        for caps, expect in ((counts.copy(), np.zeros(A.nrows, bool)),
                             (np.where(short, counts - 1, counts + 3), short),
                             (np.where(short, -5, ub), short & (counts > 1))):
            cap_eff = np.where(ub > 0, np.clip(caps, 1, np.maximum(ub, 1)), 0)
            need = (cap_eff * 100 + 59) // 60
            P = hc.PredictedProduct(Ad, Bd, None, cap_row=caps)
            C = P.run().to_host()
            np.testing.assert_array_equal(C.rp, ref.rp, err_msg=name)
            np.testing.assert_array_equal(C.col, ref.col, err_msg=name)
            np.testing.assert_array_equal(C.val, ref.val, err_msg=name)
            over = counts > cap_eff
            assert np.array_equal(over, expect), name
            if not np.any(need > 6144):
                assert P.n_overflow == int(np.sum(over)), (name, P.n_overflow, int(np.sum(over)))


def test_per_row_capacities_declared_sum_too_small():
    A = synth.uniform(300, 300, 6, 2)
    Ad = hc.DeviceCSR.from_host(A)
    P = hc.PredictedProduct(Ad, Ad, None, cap_row=np.full(A.nrows, 20))
    P.cap_sum = 100          # declares less than the rows ask for (the workspace is larger, so it stays in bounds)
    with pytest.raises(hc.HcspError) as e:
        P.run()
    assert e.value.status == -1
