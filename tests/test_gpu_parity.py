"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Structure (row_ptr, col) must match bit-exactly.  Values must match
bit-exactly in the default (ordered) mode, which accumulates every entry in
A's column order with separate multiply and add, exactly like the oracle;
the FAST flag is held to 1e-13 relative per entry.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import golden_io
from tests.gpu_util import (assert_bit_exact, assert_close, assert_fast_close, bits, check_row_blocks,
                            gpu_product, magnitudes, sample_blocks)

pytestmark = pytest.mark.gpu

SIZERS = ["exact", "upper_bound"]

# tier forcing through the tuning block
TIERS = {
    "default": None,
    "hash_only": {"merge_max_nnz": -1},
    "global_only": {"merge_max_nnz": -1, "table_slots": -1},
    "hash_dense": {"merge_max_nnz": -1, "dense_ratio": 1e9},
    "hash_sparse": {"merge_max_nnz": -1, "dense_ratio": 1e-9},
    "small_table": {"merge_max_nnz": -1, "table_slots": 256, "stage_slots": 256},
    "big_table": {"merge_max_nnz": -1, "table_slots": 4096, "stage_slots": 4096},
    "merge4": {"merge_lists": 4, "merge_max_nnz": 128},
}


@pytest.mark.parametrize("name", ["hand_product.txt", "cancellation.txt"])
@pytest.mark.parametrize("sizer", SIZERS)
def test_hand_examples(name, sizer):
    d = golden_io.load(name)
    A, B, C = golden_io.csr(d, "A"), golden_io.csr(d, "B"), golden_io.csr(d, "C")
    got = gpu_product(A, B, sizer)
    assert_bit_exact(got, (C.row_ptr, C.col, C.val))


@pytest.mark.parametrize("sizer", SIZERS)
@pytest.mark.parametrize("tier", list(TIERS))
def test_stencil64_all_tiers(sizer, tier):
    # the 64x64 five-point matrix squared (the small configuration)
    A = synth.stencil(64)
    got = gpu_product(A, A, sizer, tuning=TIERS[tier])
    assert_bit_exact(got, oracle.spgemm(A, A))
    assert got[3]["multiplications"] == 25 * 64 * 64 - 36 * 64 + 8


@pytest.mark.parametrize("tier", list(TIERS))
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_rows_all_tiers(tier, seed):
    A = synth.random_uniform_lengths(3001, 1, 24, seed)
    B = synth.random_uniform_lengths(3001, 0, 30, seed + 100)
    want = oracle.spgemm(A, B)
    for sizer in SIZERS:
        assert_bit_exact(gpu_product(A, B, sizer, tuning=TIERS[tier]), want)


@pytest.mark.parametrize("seed", range(12))
def test_tiny_random_rectangular(seed):
    m = 1 + (seed * 7) % 37
    k = 1 + (seed * 5) % 29
    n = 1 + (seed * 3) % 41
    A = synth.random_sparse(m, k, [0.05, 0.2, 0.5][seed % 3], 2 * seed + 1)
    B = synth.random_sparse(k, n, [0.1, 0.3, 0.6][seed % 3], 2 * seed + 2)
    want = oracle.spgemm(A, B)
    for sizer in SIZERS:
        for tier in ["default", "hash_only", "global_only"]:
            assert_bit_exact(gpu_product(A, B, sizer, tuning=TIERS[tier]), want)


@pytest.mark.parametrize("n,dim,points", [(40, 2, 9), (12, 3, 27)])
def test_wider_stencils(n, dim, points):
    A = synth.stencil(n, dim, points)
    want = oracle.spgemm(A, A)
    for sizer in SIZERS:
        for tier in ["default", "small_table", "global_only", "hash_sparse"]:
            assert_bit_exact(gpu_product(A, A, sizer, tuning=TIERS[tier]), want)


def test_power_law_rows():
    A = synth.zipf_matrix(30000, 11)
    want = oracle.spgemm(A, A)
    for sizer in SIZERS:
        for tier in ["default", "small_table", "big_table"]:
            assert_bit_exact(gpu_product(A, A, sizer, tuning=TIERS[tier]), want)


def test_fast_mode_within_tolerance():
    # every row in the workgroup tier, whose FAST mode adds unordered: each
    # entry within 1e-13 of the oracle's value (relative), or of the sum of
    # its products' magnitudes where the sum cancels
    A = synth.zipf_matrix(20000, 12)
    want = oracle.spgemm(A, A)
    for sizer in SIZERS:
        got = gpu_product(A, A, sizer, fast=True, tuning=TIERS["global_only"])
        assert_fast_close(got, want, magnitudes(A, A), 1e-13)


def test_ordered_accumulation_on_gpu():
    # 1e16 + 1 - 1e16: only A's column order gives 0
    A = synth.CSR(1, 3, np.array([0, 3]), np.array([0, 1, 2], np.int32), np.array([1e16, 1.0, -1e16]))
    B = synth.CSR(3, 1, np.array([0, 1, 2, 3]), np.array([0, 0, 0], np.int32), np.ones(3))
    for sizer in SIZERS:
        for tier in TIERS:
            got = gpu_product(A, B, sizer, tuning=TIERS[tier])
            assert got[2][0] == 0.0


def test_no_fma_on_gpu():
    a = 1.0 + 2.0 ** -30
    c = -(1.0 + 2.0 ** -29)
    A = synth.CSR(1, 2, np.array([0, 2]), np.array([0, 1], np.int32), np.array([1.0, a]))
    B = synth.CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([c, a]))
    for sizer in SIZERS:
        for tier in TIERS:
            got = gpu_product(A, B, sizer, tuning=TIERS[tier])
            assert got[2][0] == 0.0


def test_negative_zero_becomes_positive_zero():
    A = synth.CSR(1, 1, np.array([0, 1]), np.array([0], np.int32), np.array([-0.0]))
    B = synth.CSR(1, 1, np.array([0, 1]), np.array([0], np.int32), np.array([5.0]))
    for sizer in SIZERS:
        for tier in TIERS:
            got = gpu_product(A, B, sizer, tuning=TIERS[tier])
            assert bits(got[2])[0] == bits(0.0)


def _signed_zero_rows(seed):
    # rows of 12 entries whose B rows draw their columns from a pool of 1,000
    # scattered columns: a few products per row share a column, the column
    # region is wide (hashed, not dense), and the values make signed zeros
    # and order-sensitive sums (the numeric pass sorts such rows' products)
    rng = np.random.default_rng(seed)
    m, k, n, per = 200, 4096, 100000, 12
    pool = np.sort(rng.choice(n, 1000, replace=False)).astype(np.int32)

    def mat(rows, cols, choose, vals):
        rp = np.arange(rows + 1, dtype=np.int64) * per
        col = np.concatenate([np.sort(choose()) for _ in range(rows)]).astype(np.int32)
        return synth.CSR(rows, cols, rp, col, rng.choice(vals, rows * per))
    A = mat(m, k, lambda: rng.choice(k, per, replace=False), np.array([-0.0, 1.0, -1.0, 1e16, -1e16, 3.0]))
    B = mat(k, n, lambda: rng.choice(pool, per, replace=False), np.array([0.0, 2.0, -0.5, 1.0, -0.0]))
    return A, B


@pytest.mark.parametrize("tier", ["default", "hash_only", "small_table"])
def test_signed_zeros_and_order_in_sorted_product_rows(tier):
    A, B = _signed_zero_rows(7)
    want = oracle.spgemm(A, B)
    got = gpu_product(A, B, "exact", tuning=TIERS[tier])
    assert_bit_exact(got, want)
    assert np.any(np.signbit(A.val)) and not np.any(np.signbit(want[2][want[2] == 0.0]))


@pytest.mark.parametrize("sizer", SIZERS)
def test_workgroup_tier_row_with_a_long_run(sizer):
    # one row of 2,000 columns, 500 of them consecutive in the middle of a
    # wide region: in the workgroup tier's order-preserving table they share
    # a few home slots, so one run of occupied slots crosses the boundary of
    # the LDS chunks of the sorted write-out by more than their pad
    rng = np.random.default_rng(3)
    n = 1_000_000
    spread = rng.choice(np.setdiff1d(np.arange(n), np.arange(500_000, 500_500)), 1500, replace=False)
    cols = np.sort(np.concatenate([spread, np.arange(500_000, 500_500)])).astype(np.int32)
    B = synth.CSR(2, n, np.array([0, cols.size, cols.size + 1]), np.concatenate([cols, [7]]).astype(np.int32),
                  rng.uniform(-1, 1, cols.size + 1))
    A = synth.CSR(3, 2, np.array([0, 2, 3, 3]), np.array([0, 1, 0], np.int32), np.array([1.5, -2.0, 0.25]))
    want = oracle.spgemm(A, B)
    got = gpu_product(A, B, sizer, tuning=TIERS["global_only"])
    assert_bit_exact(got, want)
    assert got[3]["rows_global"] >= 2


@pytest.mark.parametrize("sizer", SIZERS)
@pytest.mark.parametrize("bcols", [10, 100_000])
def test_split_huge_rows(sizer, bcols):
    # every fourth row of A has 1,500-3,000 entries (narrow B: 7,500-9,000)
    # and every fourth, offset by two, 400-1,000 (narrow B: 1,000-3,000), over
    # B rows of 8-10 (narrow B, 10 columns) or 10-40 entries: rows of 32,768
    # or more products are computed by the workgroup tier in 16 column
    # ranges (with 10 columns most ranges are empty); the other huge rows
    # (8,192 or more) take one range
    rng = np.random.default_rng(bcols)
    k = 12000 if bcols == 10 else 4000
    lens_b = rng.integers(8, 11, k) if bcols == 10 else rng.integers(10, 41, k)
    bptr = np.zeros(k + 1, np.int64)
    bptr[1:] = np.cumsum(lens_b)
    bcol = np.concatenate([np.sort(rng.choice(bcols, l, replace=False)) for l in lens_b]).astype(np.int32)
    B = synth.CSR(k, bcols, bptr, bcol, rng.uniform(-1, 1, bcol.size))
    big = (7500, 9001) if bcols == 10 else (1500, 3001)
    mid = (1000, 3001) if bcols == 10 else (400, 1001)
    sel = np.arange(40) % 4
    lens_a = np.where(sel == 0, rng.integers(*big, 40), np.where(sel == 2, rng.integers(*mid, 40), rng.integers(1, 30, 40)))
    aptr = np.zeros(41, np.int64)
    aptr[1:] = np.cumsum(lens_a)
    acol = np.concatenate([np.sort(rng.choice(k, l, replace=False)) for l in lens_a]).astype(np.int32)
    A = synth.CSR(40, k, aptr, acol, rng.uniform(-1, 1, acol.size))
    want = oracle.spgemm(A, B)
    for tier in ("default", "global_only", "small_table"):
        got = gpu_product(A, B, sizer, tuning=TIERS[tier])
        assert_bit_exact(got, want)
    # fast mode reorders each sum: within 2 n u of the sum of the products'
    # magnitudes (n <= 9,000 terms per entry), values of either sign.  Sums of
    # thousands of terms are not held to 1e-13 relative: a reordered sum of n
    # terms can move by about n u times the magnitude sum, which for random
    # signs is ~sqrt(n) times |c|
    got = gpu_product(A, B, sizer, fast=True)
    mag = oracle.spgemm(synth.CSR(A.rows, A.cols, A.row_ptr, A.col, np.abs(A.val)),
                        synth.CSR(B.rows, B.cols, B.row_ptr, B.col, np.abs(B.val)))
    np.testing.assert_array_equal(got[0], want[0])
    np.testing.assert_array_equal(got[1], want[1])
    assert np.all(np.abs(got[2] - want[2]) <= 2 * 9000 * 2.0 ** -53 * mag[2])


def _banded(n, half, seed):
    # row k holds columns k - half .. k + half (clipped): B rows longer than a
    # wave whose products fall in a narrow window
    rng = np.random.default_rng(seed)
    rows = [np.arange(max(0, k - half), min(n, k + half + 1), dtype=np.int32) for k in range(n)]
    ptr = np.zeros(n + 1, np.int64)
    ptr[1:] = np.cumsum([r.size for r in rows])
    col = np.concatenate(rows)
    return synth.CSR(n, n, ptr, col, rng.uniform(-1, 1, col.size))


@pytest.mark.parametrize("half", [20, 50, 90])
def test_counting_bitmap_rows(half):
    # exact sizing counts rows whose columns lie in a narrow window with one
    # bit per column; with B rows of up to 181 entries the rows longer than
    # a wave take the bitmap's second loop; A rows of 1..24 entries
    n = 3000
    B = _banded(n, half, 5)
    A = synth.random_uniform_lengths(n, 1, 24, 9)
    # A's columns near the row index, so the window stays narrow
    rng = np.random.default_rng(11)
    col = np.empty_like(A.col)
    for i in range(n):
        s, e = A.row_ptr[i], A.row_ptr[i + 1]
        lo, hi = max(0, i - 100), min(n, i + 100)
        col[s:e] = np.sort(rng.choice(np.arange(lo, hi), e - s, replace=False))
    A = synth.CSR(n, n, A.row_ptr, col.astype(np.int32), A.val)
    want = oracle.spgemm(A, B)
    for tier in ("default", "hash_only", "small_table"):
        assert_bit_exact(gpu_product(A, B, "exact", tuning=TIERS[tier]), want)


@pytest.mark.parametrize("m,k,n", [(0, 0, 0), (0, 5, 3), (4, 0, 3), (4, 5, 0), (5, 4, 3)])
def test_empty_operands(m, k, n):
    A = synth.CSR(m, k, np.zeros(m + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    B = synth.random_sparse(k, n, 0.5, 1)
    for sizer in SIZERS:
        got = gpu_product(A, B, sizer)
        assert got[0].shape == (m + 1,) and got[0][-1] == 0 and got[1].size == 0


def test_empty_rows_between_full_rows():
    lengths = np.where(np.arange(5000) % 3 == 0, 0, 7)
    A = synth.random_rows(5000, 5000, lengths, 3)
    B = synth.random_uniform_lengths(5000, 0, 9, 4)
    want = oracle.spgemm(A, B)
    for sizer in SIZERS:
        assert_bit_exact(gpu_product(A, B, sizer), want)


def test_identity_products():
    A = synth.random_uniform_lengths(4000, 0, 20, 8)
    I = synth.identity(4000)
    for sizer in SIZERS:
        assert_bit_exact(gpu_product(A, I, sizer), (A.row_ptr, A.col, A.val))
        assert_bit_exact(gpu_product(I, A, sizer), (A.row_ptr, A.col, A.val))


def test_dense_row_hits_every_column():
    # one row of A selects every row of B: the output row is dense
    n = 3000
    A = synth.CSR(1, n, np.array([0, n]), np.arange(n, dtype=np.int32), np.ones(n))
    B = synth.random_uniform_lengths(n, 1, 6, 9)
    want = oracle.spgemm(A, B)
    for sizer in SIZERS:
        for tier in ["default", "global_only", "hash_sparse"]:
            assert_bit_exact(gpu_product(A, B, sizer, tuning=TIERS[tier]), want)


def test_capacity_error_reports_required_size():
    import paper_1303_1651_amd as P
    import torch
    A = synth.stencil(32)
    dA = P.DeviceCSR.from_host(A)
    want = oracle.spgemm(A, A)
    nnz = int(want[0][-1])
    plan = P.Plan(dA, dA, "upper_bound")
    rp = torch.empty(A.rows + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(nnz - 1, dtype=torch.int32, device="cuda")
    val = torch.empty(nnz - 1, dtype=torch.float64, device="cuda")
    code, got = plan.numeric(rp, col, val)
    assert code == 6 and got == nnz
    col = torch.empty(nnz, dtype=torch.int32, device="cuda")
    val = torch.empty(nnz, dtype=torch.float64, device="cuda")
    code, got = plan.numeric(rp, col, val)
    assert code == 0 and got == nnz
    assert_bit_exact((rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()), want)
    plan.close()


@pytest.mark.parametrize("which", ["A", "B"])
def test_plan_rejects_nnz_that_disagrees_with_row_ptr(which):
    # the plan keeps arrays sized by the descriptors' nnz; a descriptor whose
    # nnz is not row_ptr[rows] is refused before any pass
    import ctypes
    import torch
    import paper_1303_1651_amd as P
    from paper_1303_1651_amd import _lib as L
    A = synth.random_uniform_lengths(300, 20, 30, 3)
    dA = P.DeviceCSR.from_host(A)
    for nnz in (int(A.row_ptr[-1]) - 1, int(A.row_ptr[-1]) + 5):
        da, db = dA.descriptor(), dA.descriptor()
        (da if which == "A" else db).nnz = nnz
        opts = L.spgemm_options(L.SIZER_EXACT, 0, None, None)
        need = ctypes.c_size_t()
        L.check(L.spgemm_plan_workspace_size(ctypes.byref(da), ctypes.byref(db), ctypes.byref(opts),
                                             ctypes.byref(need)), "workspace")
        ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
        plan = ctypes.c_void_p()
        code = L.spgemm_plan_create(ctypes.byref(da), ctypes.byref(db), ctypes.byref(opts), ws.data_ptr(),
                                    need.value, None, ctypes.byref(plan), None)
        torch.cuda.synchronize()
        assert code == 2, code


def test_validate_rejects_unsorted_columns():
    import paper_1303_1651_amd as P
    A = synth.CSR(2, 3, np.array([0, 2, 3]), np.array([2, 1, 0], np.int32), np.ones(3))
    B = synth.random_sparse(3, 3, 0.6, 1)
    with pytest.raises(P.SpgemmError) as e:
        gpu_product(A, B, "exact", validate=True)
    assert e.value.code == 3
    # canonical input passes validation
    A2 = synth.CSR(2, 3, np.array([0, 2, 3]), np.array([1, 2, 0], np.int32), np.ones(3))
    assert_bit_exact(gpu_product(A2, B, "exact", validate=True), oracle.spgemm(A2, B))


def test_repeated_runs_identical():
    A = synth.zipf_matrix(20000, 5)
    first = gpu_product(A, A, "upper_bound")
    for _ in range(3):
        again = gpu_product(A, A, "upper_bound")
        assert_bit_exact(again, first[:3])


# ----------------------------------------------------------- full sizes
def test_stencil2048_full_size():
    A = synth.stencil(2048)
    want = oracle.spgemm(A, A)
    for sizer in SIZERS:
        got = gpu_product(A, A, sizer)
        assert got[3]["multiplications"] == 104783880
        assert int(got[0][-1]) == 54484996
        assert_bit_exact(got, want)


def test_random_2pow21_sampled_blocks():
    n = 1 << 21
    A = synth.random_fixed(n, 16, 1)
    B = synth.random_fixed(n, 16, 2)
    for sizer in SIZERS:
        got = gpu_product(A, B, sizer)
        assert got[3]["multiplications"] == n * 256
        blocks = sample_blocks(n, 24, 512, 7)
        check_row_blocks(got, A, B, blocks, exact=True)
        # every row has between 16 and 256 entries
        lens = np.diff(got[0])
        assert lens.min() >= 16 and lens.max() <= 256


def test_autotuner_picks_a_valid_tuning(tmp_path):
    import json
    import paper_1303_1651_amd as P
    from paper_1303_1651_amd.autotune import autotune
    A = synth.zipf_matrix(20000, 31)
    dA = P.DeviceCSR.from_host(A)
    grid = {"table_slots": [256, 1024], "stage_slots": [512, 1024], "merge_max_nnz": [32, 64]}
    cache = str(tmp_path / "tune.json")
    best = autotune(dA, dA, "exact", grid=grid, reps=1, cache=cache)
    assert set(best) == set(grid)
    assert json.load(open(cache))
    # cached on the second call, and the tuned product is still exact
    assert autotune(dA, dA, "exact", grid=grid, reps=1, cache=cache) == best
    assert_bit_exact(gpu_product(A, A, "exact", tuning=best), oracle.spgemm(A, A))


@pytest.mark.parametrize("n", [8192, 40960])
def test_fill01_random_dense_window_and_sorted_table(n):
    # the storing-strategy study's random matrices (0.1 % fill, Section IV-B):
    # product rows of about (0.001 n)^2 entries over all n columns; the
    # workgroup tier with a dense window (MinMax) for every row, with a
    # hashed, sorted table (Sort) for every row, and the default choice
    A = synth.random_fill(n, 0.001, 5)
    B = synth.random_fill(n, 0.001, 6)
    want = oracle.spgemm(A, B)
    dense = {"merge_max_nnz": -1, "table_slots": -1, "dense_ratio": 1e9}
    hashed = {"merge_max_nnz": -1, "table_slots": -1, "dense_ratio": 1e-9}
    for sizer in SIZERS:
        for tuning in (None, dense, hashed):
            got = gpu_product(A, B, sizer, tuning=tuning)
            assert_bit_exact(got, want)


@pytest.mark.skip(reason="the LDS bitmap path of the workgroup tier (tuning bitmap_cols > 0) is off: its first "
                         "GPU run, a batched learned one pass, ended in a memory violation whose cause has not "
                         "been found; it stays off the GPU until one is shown")
@pytest.mark.parametrize("sizer", SIZERS)
def test_workgroup_bitmap_window(sizer):
    # every row in the workgroup tier, its column region as an LDS bitmap
    A = synth.random_fill(8192, 0.001, 5)
    B = synth.random_fill(8192, 0.001, 6)
    want = oracle.spgemm(A, B)
    got = gpu_product(A, B, sizer, tuning={"merge_max_nnz": -1, "table_slots": -1, "bitmap_cols": 1 << 20})
    assert_bit_exact(got, want)


@pytest.mark.parametrize("k", [16, 24, 32])
def test_expand_sort_rows_up_to_1024_products(k):
    # rows of k x k products over a million columns (few shared): in the
    # numeric pass expand-sort rows, those above 512 products sorted 16 keys
    # per lane; the one pass takes them through its table
    A = synth.random_fixed(1500, k, 41 + k, cols=1 << 16)
    B = synth.random_fixed(1 << 16, k, 97 + k, cols=1 << 20)
    want = oracle.spgemm(A, B)
    for sizer in SIZERS:
        assert_bit_exact(gpu_product(A, B, sizer), want)
