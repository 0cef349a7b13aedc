"""GPU parity for square x tall-skinny products (the paper's second workload, Sec. "SpGEMM Performance on
Square x Tall-skinny matrix"): A a graph, B the multi-source BFS frontier matrix of A at one iteration (one
column per source).  The HIP path through the C ABI must equal the oracle bit for bit, for plain CSR and for
CSR_Cluster operands built once from A (reordered rows, hierarchical and variable-length clusters)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2507_21253_amd as hc  # noqa: E402


def assert_same(Cg, Cr, where):
    np.testing.assert_array_equal(Cg.rp, Cr.rp, err_msg="row_ptr " + where)
    np.testing.assert_array_equal(Cg.col, Cr.col, err_msg="col " + where)
    np.testing.assert_array_equal(Cg.val, Cr.val, err_msg="val " + where)


def graphs():
    yield "stencil27_12_relabelled", synth.workload_stencil27(12, 5, 6)[0]
    yield "rmat10", synth.rmat(10, 16, 0.57, 0.19, 0.19, 8)


@pytest.mark.parametrize("name,A", list(graphs()))
def test_frontier_products_bitwise(name, A):
    Ad = hc.DeviceCSR.from_host(A)
    rcm = oracle.order_rcm(A)
    operands = {"csr": Ad,
                "rcm_hc4": hc.cluster_build(Ad, hc.plan_hierarchical(A, (3, 10), 4, hc.SIM_ROOT, perm_in=rcm)),
                "variable8": hc.cluster_build(Ad, hc.plan_variable(A, (3, 10), 8))}
    for level in (1, 2, 3, 5):
        B = synth.frontiers(A, 64, level, 9)
        ref = oracle.spgemm(A, B)
        Bd = hc.DeviceCSR.from_host(B)
        for op, X in operands.items():
            C = hc.spgemm(X, Bd)
            torch.cuda.synchronize()
            assert_same(C.to_host(), ref, "%s %s level %d" % (name, op, level))


def test_narrow_and_empty_frontiers():
    # frontiers past the graph's eccentricity are empty; a single source gives a one-column B
    A = synth.workload_stencil27(6, 5, 6)[0]
    Ad = hc.DeviceCSR.from_host(A)
    for nsrc, level in ((1, 2), (16, 40), (216, 1)):
        B = synth.frontiers(A, nsrc, level, 3)
        C = hc.spgemm(Ad, hc.DeviceCSR.from_host(B))
        torch.cuda.synchronize()
        assert_same(C.to_host(), oracle.spgemm(A, B), "nsrc %d level %d" % (nsrc, level))
