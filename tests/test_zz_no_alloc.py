"""spgemm_numeric_static (the numeric pass whose scratch is the library's
static device array, for callers that cannot allocate) through the C ABI:
its output equals spgemm_numeric's on the same plan, and the oracle's, on
two calls in a row (the second on a smaller product, so that the array
holds the first call's tables when the second starts); a plan whose
scratch exceeds the array's size is refused."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_bit_exact

pytestmark = pytest.mark.gpu


def _product_both_ways(A, B, sizer, tuning=None):
    import paper_1303_1651_amd as P
    import torch
    dA = P.DeviceCSR.from_host(A)
    dB = dA if B is A else P.DeviceCSR.from_host(B)
    plan = P.Plan(dA, dB, sizer, tuning=tuning)
    dev = dA.row_ptr.device
    if sizer == "exact":
        rp, nnz = plan.symbolic()
        cap = max(nnz, 1)
    else:
        cap = max(int(plan.info["c_capacity_hint"]), 1)
    outs = []
    for static in (False, True):
        rp = torch.full((A.rows + 1,), -7, dtype=torch.int64, device=dev) if sizer != "exact" else rp.clone()
        col = torch.full((cap,), -7, dtype=torch.int32, device=dev)
        val = torch.full((cap,), float("nan"), dtype=torch.float64, device=dev)
        if static:
            code, got = plan.numeric_static(rp, col, val, capacity=cap)
        else:
            code, got = plan.numeric(rp, col, val, capacity=cap)
        P.check(code, "spgemm_numeric_static" if static else "spgemm_numeric")
        outs.append((rp.cpu().numpy(), col[:got].cpu().numpy(), val[:got].cpu().numpy()))
    info = dict(plan.info)
    plan.close()
    return outs, info


@pytest.mark.parametrize("sizer", ["exact", "upper_bound"])
def test_static_scratch_equals_allocating_call_twice(sizer):
    # power-law rows: some reach the workgroup tier, whose device tables
    # live in the scratch; the second product is smaller
    for n, seed in ((1 << 14, 5), (1 << 11, 6)):
        A = synth.zipf_matrix(n, seed)
        (ref, got), info = _product_both_ways(A, A, sizer)
        assert info["rows_global"] > 0, "the product must use the workgroup tier"
        assert_bit_exact(got, ref)
        assert_bit_exact(got, oracle.spgemm(A, A))


def test_static_scratch_refuses_a_plan_that_does_not_fit():
    import paper_1303_1651_amd as P
    import torch
    from paper_1303_1651_amd import _lib
    A = synth.random_fixed(1 << 18, 16, 3)
    B = synth.random_fixed(1 << 18, 16, 4)
    dA, dB = P.DeviceCSR.from_host(A), P.DeviceCSR.from_host(B)
    plan = P.Plan(dA, dB, "upper_bound")
    # the one pass lays rows out in a padded buffer of 12 bytes per bound entry
    assert 12 * plan.info["c_capacity_hint"] > _lib.spgemm_numeric_static_limit()
    dev = dA.row_ptr.device
    rp = torch.empty(A.rows + 1, dtype=torch.int64, device=dev)
    col = torch.empty(16, dtype=torch.int32, device=dev)
    val = torch.empty(16, dtype=torch.float64, device=dev)
    code, _ = plan.numeric_static(rp, col, val, capacity=16)
    assert code == 5   # SPGEMM_E_WORKSPACE
    plan.close()
