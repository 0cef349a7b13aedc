"""GPU parity of the hierarchical plan's candidate search (SpGEMM_TopK, Alg. 3): the overlap matrix A A^T
is the library's own product of A's pattern with its transpose (formed on the device), and the per-row
top-k selection runs on the GPU.  The lists must equal the oracle's exactly (partners, their order and overlaps), and the plan built from them must
equal the host plan."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2507_21253_amd as hc  # noqa: E402


def symmetric_inputs():
    yield "stencil27_8", synth.stencil(27, 8, 2)
    yield "stencil27_9_relabelled", synth.workload_stencil27(9, 2, 3)[0]
    yield "rmat10", synth.rmat(10, 16, 0.57, 0.19, 0.19, 4)
    yield "stencil5_30", synth.stencil(5, 30, 1)


@pytest.mark.parametrize("name,A", list(symmetric_inputs()))
def test_topk_candidates_match_oracle(name, A):
    Ad = hc.DeviceCSR.from_host(A)
    for t, topk in (((3, 10), 7), ((1, 5), 3), ((1, 2), 1), ((0, 1), 15)):
        for pi in (None, synth.perm(A.nrows, 14), oracle.order_rcm(A)):
            cnt, nbr, ov = hc.topk_candidates_gpu(Ad, t, topk, pi)
            rc, rn, ro, _ = oracle.topk_candidates(A, t, topk, pi)
            where = "%s t=%s topk=%d perm=%s" % (name, t, topk, pi is not None)
            np.testing.assert_array_equal(cnt, rc, err_msg="cnt " + where)
            np.testing.assert_array_equal(nbr, rn, err_msg="nbr " + where)
            np.testing.assert_array_equal(ov, ro, err_msg="ov " + where)


@pytest.mark.parametrize("name,A", list(symmetric_inputs()))
def test_gpu_assisted_plan_equals_host_plan(name, A):
    Ad = hc.DeviceCSR.from_host(A)
    for maxc in (2, 4, 8):
        for sim in (hc.SIM_ROOT, hc.SIM_UNION):
            pi = oracle.order_rcm(A)
            got = hc.plan_hierarchical_gpu(A, Ad, (3, 10), maxc, sim, perm_in=pi)
            ref = hc.plan_hierarchical(A, (3, 10), maxc, sim, perm_in=pi)
            np.testing.assert_array_equal(got.perm, ref.perm, err_msg="%s %d" % (name, maxc))
            np.testing.assert_array_equal(got.cl_row_ptr, ref.cl_row_ptr, err_msg="%s %d" % (name, maxc))


def nonsymmetric_inputs():
    # patterns whose transpose differs from themselves: A A^T is not A A here
    yield "uniform_300x200", synth.uniform(300, 200, 6, 3)
    yield "uniform_3000_d10", synth.uniform(3000, 3000, 10, 8)
    R = synth.rmat(11, 8, 0.57, 0.19, 0.19, 9)     # keep the upper triangle: a non-symmetric pattern
    rows = np.repeat(np.arange(R.nrows), np.diff(R.rp))
    upper = R.col >= rows
    rp = np.zeros(R.nrows + 1, np.int64)
    np.add.at(rp, rows[upper] + 1, 1)
    yield "rmat11_upper", synth.HostCSR(np.cumsum(rp), R.col[upper].copy(), R.val[upper].copy(), R.nrows, R.ncols)


@pytest.mark.parametrize("name,A", list(nonsymmetric_inputs()))
def test_topk_candidates_nonsymmetric_match_oracle(name, A):
    Ad = hc.DeviceCSR.from_host(A)
    for t, topk in (((3, 10), 7), ((1, 5), 3), ((1, 10), 15)):
        for pi in (None, synth.perm(A.nrows, 15)):
            cnt, nbr, ov = hc.topk_candidates_gpu(Ad, t, topk, pi)
            rc, rn, ro, _ = oracle.topk_candidates(A, t, topk, pi)
            where = "%s t=%s topk=%d perm=%s" % (name, t, topk, pi is not None)
            np.testing.assert_array_equal(cnt, rc, err_msg="cnt " + where)
            np.testing.assert_array_equal(nbr, rn, err_msg="nbr " + where)
            np.testing.assert_array_equal(ov, ro, err_msg="ov " + where)
    plan = hc.plan_hierarchical_gpu(A, Ad, (3, 10), 4, hc.SIM_ROOT)
    ref = hc.plan_hierarchical(A, (3, 10), 4, hc.SIM_ROOT)
    np.testing.assert_array_equal(plan.perm, ref.perm)
    np.testing.assert_array_equal(plan.cl_row_ptr, ref.cl_row_ptr)
