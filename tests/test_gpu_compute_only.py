"""The pure computation kernel (Section IV-A) on the GPU through the C ABI:
every row of C accumulated as the numeric pass does, nothing stored; the
per-row entry counts and largest magnitudes must equal those of the
oracle's product bit for bit.  Products whose rows do not all take the
register merge are refused."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import bits

pytestmark = pytest.mark.gpu


def _row_stats(want):
    rp, _, val = want
    cnt = np.diff(rp).astype(np.int32)
    mx = np.zeros(len(cnt))
    nz = cnt > 0
    if nz.any():
        mx[nz] = np.maximum.reduceat(np.abs(val), rp[:-1][nz])
    return cnt, mx


CASES = {
    "stencil5_64": lambda: (synth.stencil(64),) * 2,
    "stencil9_40": lambda: (synth.stencil(40, 2, 9),) * 2,
    "random5_8192": lambda: (synth.random_fixed(8192, 5, 3), synth.random_fixed(8192, 5, 4)),
    "empty_rows": lambda: (synth.random_rows(3000, 3000, np.where(np.arange(3000) % 4 == 0, 0, 3), 5),
                           synth.random_uniform_lengths(3000, 0, 7, 6)),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("sizer", ["exact", "upper_bound"])
def test_compute_only_row_stats_equal_oracle(case, sizer):
    import paper_1303_1651_amd as P
    A, B = CASES[case]()
    dA = P.DeviceCSR.from_host(A)
    dB = dA if B is A else P.DeviceCSR.from_host(B)
    plan = P.Plan(dA, dB, sizer)
    cnt, mx = plan.compute_only()
    plan.close()
    want_cnt, want_mx = _row_stats(oracle.spgemm(A, B))
    np.testing.assert_array_equal(cnt.cpu().numpy(), want_cnt)
    np.testing.assert_array_equal(bits(mx.cpu().numpy()), bits(want_mx))


def test_compute_only_full_size_stencil():
    import paper_1303_1651_amd as P
    A = synth.stencil(2048)
    dA = P.DeviceCSR.from_host(A)
    plan = P.Plan(dA, dA, "exact")
    cnt, mx = plan.compute_only()
    plan.close()
    want_cnt, want_mx = _row_stats(oracle.spgemm(A, A))
    assert int(cnt.sum()) == 54484996
    np.testing.assert_array_equal(cnt.cpu().numpy(), want_cnt)
    np.testing.assert_array_equal(bits(mx.cpu().numpy()), bits(want_mx))


def test_compute_only_refuses_tiled_products():
    import paper_1303_1651_amd as P
    A = synth.random_fixed(4096, 24, 1)
    dA = P.DeviceCSR.from_host(A)
    plan = P.Plan(dA, dA, "exact")
    with pytest.raises(P.SpgemmError) as e:
        plan.compute_only()
    assert e.value.code == 10
    plan.close()
