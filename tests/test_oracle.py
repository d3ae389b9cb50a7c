"""Pins for the CPU oracle against what the paper and the mathematics fix.

None of these tests needs a GPU.  Each pin is chosen so that a plausible slip
in the oracle (a dropped term, a wrong index, a transposed operand, a wrong
accumulation order, a dropped cancelled entry) fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from tests import golden_io


def brute_force(A, B):
    """Dense triple loop written independently of the oracle: c_ij is the sum
    over k ascending of a_ik * b_kj over structurally present pairs, starting
    from +0.0, one rounding per multiply and per add (Python floats)."""
    Ad = A.to_dense()
    Bd = B.to_dense()
    Am = np.zeros((A.rows, A.cols), dtype=bool)
    Bm = np.zeros((B.rows, B.cols), dtype=bool)
    Am[np.repeat(np.arange(A.rows), np.diff(A.row_ptr)), A.col] = True
    Bm[np.repeat(np.arange(B.rows), np.diff(B.row_ptr)), B.col] = True
    ptr, cols, vals = [0], [], []
    for i in range(A.rows):
        for j in range(B.cols):
            present = False
            acc = 0.0
            for k in range(A.cols):
                if Am[i, k] and Bm[k, j]:
                    present = True
                    acc = acc + float(Ad[i, k]) * float(Bd[k, j])
            if present:
                cols.append(j)
                vals.append(acc)
        ptr.append(len(cols))
    return np.array(ptr, np.int64), np.array(cols, np.int32), np.array(vals, np.float64)


def bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


def assert_same(got, want):
    gp, gc, gv = got
    wp, wc, wv = want
    np.testing.assert_array_equal(gp, wp)
    np.testing.assert_array_equal(gc, wc)
    np.testing.assert_array_equal(bits(gv), bits(wv))


# ----------------------------------------------------------- hand examples
@pytest.mark.parametrize("name", ["hand_product.txt", "cancellation.txt"])
def test_hand_worked_examples(name):
    d = golden_io.load(name)
    A, B, C = golden_io.csr(d, "A"), golden_io.csr(d, "B"), golden_io.csr(d, "C")
    assert_same(oracle.spgemm(A, B), (C.row_ptr, C.col, C.val))
    assert oracle.multiplications(A, B) == int(d["mults"][0])
    f1, ub, mx = oracle.features(A, B)
    assert list(ub) == [int(x) for x in d["row_mults"]]
    if "row_maxb" in d:
        assert list(f1) == [int(x) for x in d["row_nnz_a"]]
        assert list(mx) == [int(x) for x in d["row_maxb"]]


def test_longest_selected_row_of_the_five_point_stencil():
    # Closed form: row i of the n x n five-point matrix selects the rows of
    # its in-grid neighbours and itself; a row of the matrix has 1 + deg
    # entries (deg = in-grid neighbours: 2 at a corner, 3 on an edge, 4
    # inside).  The longest selected row is 5 wherever some selected point
    # is interior, 4 at the corners of grids with n >= 3 (the corner selects
    # itself (3) and two edge points (4)); every row selects five rows
    # except corners (3) and edges (4).
    n = 7
    A = synth.stencil(n)
    f1, ub, mx = oracle.features(A, A)
    deg = lambda x, y: (x > 0) + (x < n - 1) + (y > 0) + (y < n - 1)
    for y in range(n):
        for x in range(n):
            i = x + n * y
            sel = [(x, y)] + [(x + dx, y + dy) for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1))
                              if 0 <= x + dx < n and 0 <= y + dy < n]
            assert f1[i] == len(sel) == 1 + deg(x, y)
            corner = x in (0, n - 1) and y in (0, n - 1)
            touches_interior = any(0 < a < n - 1 and 0 < b < n - 1 for a, b in sel)
            assert touches_interior == (not corner)
            assert mx[i] == (4 if corner else 5), (x, y)
            assert ub[i] == sum(1 + deg(a, b) for a, b in sel)


def test_longest_selected_row_equals_count_for_single_entry_rows():
    # A row of A with one stored entry selects one row of B, so nnz(C_i), the
    # bound and the longest selected row all equal that row's length
    A = synth.random_uniform_lengths(400, 0, 1, 21)
    B = synth.random_uniform_lengths(400, 0, 30, 22)
    f1, ub, mx = oracle.features(A, B)
    counts = oracle.row_counts(A, B)
    one = f1 == 1
    assert one.sum() > 100
    np.testing.assert_array_equal(mx[one], counts[one])
    np.testing.assert_array_equal(ub[one], counts[one])
    assert np.all(mx[f1 == 0] == 0)


def test_longest_selected_row_of_nested_rows():
    # B rows 0..3 hold 1, 4, 2 and 3 entries; a row of A selecting {0, 2, 3}
    # has longest selected row 3, one selecting {1} has 4, {0} has 1
    B = synth.CSR(4, 5, np.array([0, 1, 5, 7, 10]),
                  np.array([2, 0, 1, 2, 3, 1, 4, 0, 2, 4], np.int32), np.ones(10))
    A = synth.CSR(3, 4, np.array([0, 3, 4, 5]), np.array([0, 2, 3, 1, 0], np.int32), np.ones(5))
    f1, ub, mx = oracle.features(A, B)
    assert list(f1) == [3, 1, 1] and list(ub) == [6, 4, 1] and list(mx) == [3, 4, 1]


def test_cancelled_entry_is_kept_as_positive_zero():
    d = golden_io.load("cancellation.txt")
    ptr, col, val = oracle.spgemm(golden_io.csr(d, "A"), golden_io.csr(d, "B"))
    assert ptr[-1] == 1 and col[0] == 0
    assert bits(val)[0] == bits(0.0)   # +0.0, not -0.0


def test_negative_zero_product_accumulates_from_positive_zero():
    # temp starts at +0.0 (Section IV-A listing); +0.0 + (-0.0) = +0.0
    A = synth.CSR(1, 1, np.array([0, 1]), np.array([0], np.int32), np.array([-0.0]))
    B = synth.CSR(1, 1, np.array([0, 1]), np.array([0], np.int32), np.array([5.0]))
    ptr, col, val = oracle.spgemm(A, B)
    assert bits(val)[0] == bits(0.0)


# --------------------------------------------------------------- brute force
CASES = []
for seed in range(60):
    m = 1 + (seed * 7) % 23
    k = 1 + (seed * 5) % 19
    n = 1 + (seed * 3) % 29
    dens = [0.0, 0.05, 0.2, 0.4, 0.6][seed % 5]
    CASES.append((seed, m, k, n, dens))


@pytest.mark.parametrize("seed,m,k,n,dens", CASES)
def test_oracle_equals_brute_force_bit_exact(seed, m, k, n, dens):
    A = synth.random_sparse(m, k, dens, 2 * seed + 1)
    B = synth.random_sparse(k, n, min(1.0, dens * 1.5), 2 * seed + 2)
    assert_same(oracle.spgemm(A, B), brute_force(A, B))


def test_oracle_equals_brute_force_with_repeated_terms():
    # integers with many terms per output: exact in any order, so this pins
    # structure and values through long accumulation chains
    A = synth.random_sparse(17, 31, 0.7, 101, integer=True)
    B = synth.random_sparse(31, 13, 0.7, 102, integer=True)
    assert_same(oracle.spgemm(A, B), brute_force(A, B))


def test_accumulation_order_is_ascending_k():
    # 1e16 + 1 - 1e16 differs by order: ((0 + 1e16) + 1) + (-1e16) = 0,
    # while any order that adds the 1 last gives 1.  A's stored order is
    # ascending column, so the products arrive as k = 0, 1, 2.
    A = synth.CSR(1, 3, np.array([0, 3]), np.array([0, 1, 2], np.int32), np.array([1e16, 1.0, -1e16]))
    B = synth.CSR(3, 1, np.array([0, 1, 2, 3]), np.array([0, 0, 0], np.int32), np.ones(3))
    _, _, val = oracle.spgemm(A, B)
    assert val[0] == 0.0
    A2 = synth.CSR(1, 3, np.array([0, 3]), np.array([0, 1, 2], np.int32), np.array([1e16, -1e16, 1.0]))
    _, _, val2 = oracle.spgemm(A2, B)
    assert val2[0] == 1.0


def test_no_fused_multiply_add():
    # temp = c first, then temp + a*a.  a*a = 1 + 2^-29 + 2^-60 is inexact in
    # FP64; a separate multiply rounds it to 1 + 2^-29 and the add gives 0,
    # a fused multiply-add would keep 2^-60.
    a = 1.0 + 2.0 ** -30
    c = -(1.0 + 2.0 ** -29)
    assert a * a == -c                  # the rounded product
    A = synth.CSR(1, 2, np.array([0, 2]), np.array([0, 1], np.int32), np.array([1.0, a]))
    B = synth.CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([c, a]))
    _, _, val = oracle.spgemm(A, B)
    assert val[0] == 0.0
    assert val[0] != 2.0 ** -60


# ------------------------------------------------------- closed-form stencils
def stencil5_square_entry(n, i, j):
    """Closed form of (A*A)_ij for the 5-point matrix, diagonal 4, off -1."""
    xi, yi = i % n, i // n
    xj, yj = j % n, j // n
    dx, dy = xj - xi, yj - yi
    if dx == 0 and dy == 0:
        deg = (xi > 0) + (xi < n - 1) + (yi > 0) + (yi < n - 1)
        return 16.0 + deg
    if abs(dx) + abs(dy) == 1:
        return -8.0
    if (abs(dx), abs(dy)) in ((2, 0), (0, 2)):
        return 1.0
    if abs(dx) == 1 and abs(dy) == 1:
        return 2.0
    return None


@pytest.mark.parametrize("n", [2, 3, 4, 7, 16, 33])
def test_stencil5_square_closed_form(n):
    A = synth.stencil(n)
    ptr, col, val = oracle.spgemm(A, A)
    N = n * n
    assert A.nnz == 5 * n * n - 4 * n
    assert ptr[-1] == 13 * n * n - 20 * n + 4
    assert oracle.multiplications(A, A) == 25 * n * n - 36 * n + 8
    for i in range(N):
        cols = col[ptr[i]:ptr[i + 1]]
        vals = val[ptr[i]:ptr[i + 1]]
        want = [(j, stencil5_square_entry(n, i, j)) for j in range(N)]
        want = [(j, v) for j, v in want if v is not None]
        assert list(cols) == [j for j, _ in want]
        assert list(vals) == [v for _, v in want]


@pytest.mark.parametrize("n,dim,points", [(2, 2, 9), (5, 2, 9), (9, 2, 9), (2, 3, 27), (4, 3, 27), (6, 3, 27)])
def test_chebyshev_stencil_square_closed_form(n, dim, points):
    """A = dI - S (S the 0/1 adjacency of Chebyshev distance 1):
    (A^2)_ii = d^2 + deg(i); (A^2)_ij = -2d [i~j] + common(i, j);
    pattern = all grid points within Chebyshev distance 2."""
    A = synth.stencil(n, dim, points)
    d = float(points - 1)
    ptr, col, val = oracle.spgemm(A, A)
    assert A.nnz == (3 * n - 2) ** dim
    assert ptr[-1] == (5 * n - 6) ** dim
    assert oracle.multiplications(A, A) == (9 * n - 10) ** dim
    N = n ** dim
    coords = np.stack([(np.arange(N) // n ** a) % n for a in range(dim)], axis=1)
    for i in range(0, N, max(1, N // 40)):
        ci = coords[i]
        nb = np.all(np.abs(coords - ci) <= 1, axis=1)
        nb[i] = False
        cols = col[ptr[i]:ptr[i + 1]]
        vals = val[ptr[i]:ptr[i + 1]]
        want_cols = np.nonzero(np.all(np.abs(coords - ci) <= 2, axis=1))[0]
        np.testing.assert_array_equal(cols, want_cols)
        for j, v in zip(cols, vals):
            if j == i:
                expect = d * d + nb.sum()
            else:
                nbj = np.all(np.abs(coords - coords[j]) <= 1, axis=1)
                nbj[j] = False
                expect = (-2.0 * d if nb[j] else 0.0) + float(np.sum(nb & nbj))
            assert v == expect


# ----------------------------------------------------------------- invariants
@pytest.mark.parametrize("seed", range(8))
def test_row_bounds_and_multiplication_count(seed):
    A = synth.random_uniform_lengths(300, 1, 12, seed)
    B = synth.random_uniform_lengths(300, 0, 9, seed + 50)
    f1, ub, mx = oracle.features(A, B)
    counts = oracle.row_counts(A, B)
    assert np.all(mx <= counts) and np.all(counts <= ub)
    # sum of per-row bounds equals the column-count formula of Section III
    assert int(ub.sum()) == oracle.multiplications(A, B)
    assert oracle.flops(A, B) == 2 * int(ub.sum())
    np.testing.assert_array_equal(f1, np.diff(A.row_ptr))


def test_upper_bound_tight_iff_selected_rows_disjoint():
    # rows of B with pairwise disjoint columns reach the bound exactly
    B = synth.CSR(3, 6, np.array([0, 2, 4, 6]), np.array([0, 1, 2, 3, 4, 5], np.int32), np.ones(6))
    A = synth.CSR(1, 3, np.array([0, 3]), np.array([0, 1, 2], np.int32), np.ones(3))
    assert oracle.row_counts(A, B)[0] == oracle.features(A, B)[1][0] == 6
    B2 = synth.CSR(3, 6, np.array([0, 2, 4, 6]), np.array([0, 1, 1, 3, 4, 5], np.int32), np.ones(6))
    assert oracle.row_counts(A, B2)[0] == 5


def test_identity_and_permutation_products():
    A = synth.random_uniform_lengths(200, 0, 10, 7)
    I = synth.identity(200)
    assert_same(oracle.spgemm(A, I), (A.row_ptr, A.col, A.val))
    assert_same(oracle.spgemm(I, A), (A.row_ptr, A.col, A.val))
    perm = np.random.default_rng(3).permutation(200)
    P = synth.permutation(perm)
    ptr, col, val = oracle.spgemm(P, A)          # rows of A permuted
    for i in range(200):
        c, v = A.row(int(perm[i]))
        np.testing.assert_array_equal(col[ptr[i]:ptr[i + 1]], c)
        np.testing.assert_array_equal(val[ptr[i]:ptr[i + 1]], v)


def transpose(M):
    order = np.lexsort((np.repeat(np.arange(M.rows), np.diff(M.row_ptr)), M.col))
    r = np.repeat(np.arange(M.rows), np.diff(M.row_ptr))[order]
    c = M.col[order]
    ptr = np.zeros(M.cols + 1, np.int64)
    np.cumsum(np.bincount(c, minlength=M.cols), out=ptr[1:])
    return synth.CSR(M.cols, M.rows, ptr, r.astype(np.int32), M.val[order])


@pytest.mark.parametrize("seed", range(4))
def test_transpose_identity_bit_exact(seed):
    # (AB)^T = B^T A^T, and both sides accumulate entry (i, j) over k ascending
    A = synth.random_sparse(40, 30, 0.15, seed + 10)
    B = synth.random_sparse(30, 50, 0.15, seed + 20)
    C = oracle.spgemm_csr(A, B)
    CT = transpose(synth.CSR(C.rows, C.cols, C.row_ptr, C.col, C.val))
    D = oracle.spgemm(transpose(B), transpose(A))
    assert_same(D, (CT.row_ptr, CT.col, CT.val))


@pytest.mark.parametrize("seed,m,n,dens", [(1, 40, 30, 0.15), (2, 1, 50, 0.5), (3, 60, 1, 0.5), (4, 25, 25, 0.0),
                                            (5, 120, 70, 0.05)])
def test_oracle_transpose_pins(seed, m, n, dens):
    # the oracle's transpose (a stable sort by column) against the dense
    # transpose, the lexsort formulation above, and T(T(M)) == M
    M = synth.random_sparse(m, n, dens, seed + 50)
    T = oracle.transpose(M)
    dense = np.zeros((n, m))
    r = np.repeat(np.arange(T.rows), np.diff(T.row_ptr))
    dense[r, T.col] = T.val
    np.testing.assert_array_equal(dense, M.to_dense().T)
    L = transpose(M)
    np.testing.assert_array_equal(T.row_ptr, L.row_ptr)
    np.testing.assert_array_equal(T.col, L.col)
    np.testing.assert_array_equal(bits(T.val), bits(L.val))
    for i in range(T.rows):
        assert np.all(np.diff(T.col[T.row_ptr[i]:T.row_ptr[i + 1]]) > 0)
    TT = oracle.transpose(T)
    np.testing.assert_array_equal(TT.row_ptr, M.row_ptr)
    np.testing.assert_array_equal(TT.col, M.col)
    np.testing.assert_array_equal(bits(TT.val), bits(M.val))


def test_oracle_transpose_product_identity():
    # (AB)^T = B^T A^T bit for bit, with the oracle's own transpose
    A = synth.random_sparse(50, 40, 0.12, 71)
    B = synth.random_sparse(40, 60, 0.12, 72)
    C = oracle.spgemm_csr(A, B)
    CT = oracle.transpose(C)
    D = oracle.spgemm(oracle.transpose(B), oracle.transpose(A))
    assert_same(D, (CT.row_ptr, CT.col, CT.val))


@pytest.mark.parametrize("seed", range(4))
def test_freivalds_exact_on_integers(seed):
    A = synth.random_sparse(80, 60, 0.2, seed + 30, integer=True)
    B = synth.random_sparse(60, 70, 0.2, seed + 40, integer=True)
    C = oracle.spgemm_csr(A, B)
    x = (np.arange(B.cols) % 7 - 3).astype(np.float64)
    Cs = synth.CSR(C.rows, C.cols, C.row_ptr, C.col, C.val)
    np.testing.assert_array_equal(Cs.to_dense() @ x, A.to_dense() @ (B.to_dense() @ x))


def test_matches_scipy_where_nothing_cancels():
    sp = pytest.importorskip("scipy.sparse")
    A = synth.random_uniform_lengths(3000, 1, 20, 5)
    B = synth.random_uniform_lengths(3000, 1, 20, 6)
    ptr, col, val = oracle.spgemm(A, B)
    sa = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.rows, A.cols))
    sb = sp.csr_matrix((B.val, B.col, B.row_ptr), shape=(B.rows, B.cols))
    sc = (sa @ sb).tocsr()
    sc.sort_indices()
    np.testing.assert_array_equal(ptr, sc.indptr)
    np.testing.assert_array_equal(col, sc.indices)
    np.testing.assert_allclose(val, sc.data, rtol=1e-13, atol=0)


def test_row_range_variant_is_a_slice():
    A = synth.random_uniform_lengths(500, 0, 15, 9)
    B = synth.random_uniform_lengths(500, 0, 15, 10)
    fp, fc, fv = oracle.spgemm(A, B)
    for r0, r1 in [(0, 1), (17, 123), (499, 500), (250, 250)]:
        p, c, v = oracle.spgemm(A, B, r0, r1)
        np.testing.assert_array_equal(p, fp[r0:r1 + 1] - fp[r0])
        np.testing.assert_array_equal(c, fc[fp[r0]:fp[r1]])
        np.testing.assert_array_equal(bits(v), bits(fv[fp[r0]:fp[r1]]))


@pytest.mark.parametrize("m,k,n", [(0, 0, 0), (0, 5, 3), (4, 0, 3), (4, 5, 0), (3, 3, 3)])
def test_empty_shapes(m, k, n):
    A = synth.CSR(m, k, np.zeros(m + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    B = synth.random_sparse(k, n, 0.5, 1)
    ptr, col, val = oracle.spgemm(A, B)
    assert ptr.shape == (m + 1,) and ptr[-1] == 0 and col.size == 0


def test_generators_match_paper_workload_shapes():
    # five-band structure of the FD matrix (Section III)
    A = synth.stencil(10)
    assert np.diff(A.row_ptr).max() == 5
    R = synth.random_fixed(1000, 5, 1)
    assert np.all(np.diff(R.row_ptr) == 5)
    for i in range(1000):
        c, _ = R.row(i)
        assert np.all(np.diff(c) > 0)
    assert np.all((R.val > -1) & (R.val < 1))


def test_fill_generator_rows():
    # 0.1 % fill: ceil(0.001 n) distinct columns per row, sorted, in range
    for n, k in ((5000, 5), (38912, 39), (1000, 1)):
        A = synth.random_fill(n, 0.001, 3)
        assert A.rows == n and A.cols == n
        lens = np.diff(A.row_ptr)
        assert np.all(lens == k)
        for i in range(0, n, max(1, n // 50)):
            c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
            assert np.all(np.diff(c) > 0) and c.min() >= 0 and c.max() < n
        assert np.all(np.abs(A.val) < 1.0)
