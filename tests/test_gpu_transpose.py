"""GPU parity of the transpose (the conversion of an operand stored by
columns to rows, Section IV-A) and of the product with a CSC right-hand
side, against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_bit_exact, bits, gpu_product

pytestmark = pytest.mark.gpu


def _dense_column(n_rows, n_cols, heavy, seed):
    # random rows plus one column present in every row: its row of the
    # transpose has n_rows entries (ranked 64 at a time)
    M = synth.random_uniform_lengths(n_rows, 0, 12, seed)
    rows = []
    for i in range(n_rows):
        c = M.col[M.row_ptr[i]:M.row_ptr[i + 1]].astype(np.int64) % n_cols
        rows.append(np.unique(np.append(c, heavy)))
    ptr = np.zeros(n_rows + 1, np.int64)
    ptr[1:] = np.cumsum([r.size for r in rows])
    col = np.concatenate(rows).astype(np.int32)
    return synth.CSR(n_rows, n_cols, ptr, col, np.random.default_rng(seed).uniform(-1, 1, col.size))


def _by_columns(M):
    # the CSR of M^T: transposing it gives rows as long as M's
    T = oracle.transpose(M)
    return synth.CSR(T.rows, T.cols, T.row_ptr, T.col, T.val)


def _long_columns(n_rows, n_cols, seed):
    # random rows, one column in every row, another in every third row: rows
    # of the transpose of n_rows and n_rows / 3 entries (sorted in chunks)
    M = synth.random_uniform_lengths(n_rows, 0, 6, seed)
    rows = []
    for i in range(n_rows):
        c = M.col[M.row_ptr[i]:M.row_ptr[i + 1]].astype(np.int64) % n_cols
        extra = [5] + ([n_cols - 2] if i % 3 == 0 else [])
        rows.append(np.unique(np.append(c, extra)))
    ptr = np.zeros(n_rows + 1, np.int64)
    ptr[1:] = np.cumsum([r.size for r in rows])
    col = np.concatenate(rows).astype(np.int32)
    return synth.CSR(n_rows, n_cols, ptr, col, np.random.default_rng(seed).uniform(-1, 1, col.size))


CASES = {
    # rows of the transpose of up to a few thousand entries (sorted in LDS)
    "zipf_by_columns": lambda: _by_columns(synth.zipf_matrix(20000, 5)),
    "random_rect": lambda: synth.random_sparse(700, 300, 0.02, 3),
    "stencil27": lambda: synth.stencil(12, 3, 27),
    "zipf": lambda: synth.zipf_matrix(20000, 5),
    "dense_column": lambda: _dense_column(5000, 900, 17, 8),
    "one_row": lambda: synth.random_sparse(1, 5000, 0.3, 9),
    # rows of the transpose of 120,000 and 40,000 entries
    "long_columns": lambda: _long_columns(120000, 2000, 12),
    "empty": lambda: synth.random_sparse(30, 20, 0.0, 1),
    "no_rows": lambda: synth.CSR(0, 7, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0)),
    "no_cols": lambda: synth.CSR(5, 0, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_transpose_equals_oracle(case):
    import paper_1303_1651_amd as P
    M = CASES[case]()
    want = oracle.transpose(M)
    T = P.transpose(P.DeviceCSR.from_host(M))
    assert (T.rows, T.cols) == (M.cols, M.rows)
    np.testing.assert_array_equal(T.row_ptr.cpu().numpy(), want.row_ptr)
    np.testing.assert_array_equal(T.col.cpu().numpy(), want.col)
    np.testing.assert_array_equal(bits(T.val.cpu().numpy()), bits(want.val))
    # structure only: the same pattern
    S = P.transpose(P.DeviceCSR.from_host(M), values=False)
    np.testing.assert_array_equal(S.col.cpu().numpy(), want.col)


@pytest.mark.parametrize("sizer", ["exact", "upper_bound"])
def test_product_with_csc_operand(sizer):
    # B given by columns: its CSC arrays are the CSR of B^T
    import paper_1303_1651_amd as P
    A = synth.random_uniform_lengths(3000, 1, 20, 21)
    B = synth.random_uniform_lengths(3000, 0, 25, 22)
    BT = oracle.transpose(B)
    B_csc = synth.CSR(BT.rows, BT.cols, BT.row_ptr, BT.col, BT.val)
    res = P.spgemm_csc(P.DeviceCSR.from_host(A), P.DeviceCSR.from_host(B_csc), sizer=sizer)
    got = (res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), res.val.cpu().numpy())
    assert_bit_exact(got, oracle.spgemm(A, B))


def test_transpose_twice_is_identity_on_full_size_stencil():
    import paper_1303_1651_amd as P
    M = synth.stencil(1024)
    d = P.DeviceCSR.from_host(M)
    TT = P.transpose(P.transpose(d))
    np.testing.assert_array_equal(TT.row_ptr.cpu().numpy(), M.row_ptr)
    np.testing.assert_array_equal(TT.col.cpu().numpy(), M.col)
    np.testing.assert_array_equal(bits(TT.val.cpu().numpy()), bits(M.val))


def test_transpose_rejects_bad_descriptors():
    import ctypes

    import torch

    import paper_1303_1651_amd as P
    from paper_1303_1651_amd import _lib as L
    M = synth.random_sparse(50, 40, 0.1, 4)
    d = P.DeviceCSR.from_host(M)
    t_rp = torch.empty(M.cols + 1, dtype=torch.int64, device="cuda")
    t_col = torch.empty(max(M.nnz, 1), dtype=torch.int32, device="cuda")
    t_val = torch.empty(max(M.nnz, 1), dtype=torch.float64, device="cuda")

    def run(desc):
        scratch = torch.empty(max(L.spgemm_transpose_scratch(ctypes.byref(desc)), 1), dtype=torch.uint8,
                              device="cuda")
        code = L.spgemm_transpose(ctypes.byref(desc), t_rp.data_ptr(), t_col.data_ptr(), t_val.data_ptr(),
                                  scratch.data_ptr(), scratch.numel(), None)
        torch.cuda.synchronize()
        return code

    # a column index outside [0, cols): skipped, reported
    bad = d.col.clone()
    bad[3] = M.cols + 5
    desc = L.spgemm_csr(M.rows, M.cols, M.nnz, d.row_ptr.data_ptr(), bad.data_ptr(), d.val.data_ptr())
    assert run(desc) == 3
    # nnz that disagrees with row_ptr[rows]: refused before any row is walked
    desc = L.spgemm_csr(M.rows, M.cols, M.nnz - 1, d.row_ptr.data_ptr(), d.col.data_ptr(), d.val.data_ptr())
    assert run(desc) == 2
    # and the good descriptor still works afterwards
    assert run(d.descriptor()) == 0
