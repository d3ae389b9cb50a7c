"""CPU oracle for the sparse matrix-matrix product C = A * B (CSR, FP64).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
bench's CPU-baseline leg may import this package.  It shares no code with the
GPU library (``paper_1303_1651_amd``), and the GPU library never imports it.

Contents
--------
``spgemm``         plain single-threaded Gustavson product (``spgemm_ref.c``),
                   paper Section IV-A (row-major algorithm and its listing) with
                   the "Sort" storing strategy of Section IV-B.
``row_counts``     nnz of every output row (same C file, structure only).
``features``       per-row nnz(A_i), the number of multiplications of row i and
                   the longest selected B row: plain definitions.  The per-row
                   multiplication count is the paper's size estimate
                   (Section IV-B) taken row by row.
``multiplications`` the paper's multiplication count (Section III):
                   sum over k of nnz(column k of A) * nnz(row k of B).
``transpose``      the CSR of M^T: the conversion of an operand stored by
                   columns (CSC) to rows, which Section IV-A applies before the
                   row-major product.
``mlp_ref``        FP64 reference of the row-size network, its loss, backward
                   pass and Adam step (not part of the paper; parity for the
                   project's own learned sizer).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spgemm_ref.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc: strict IEEE FP64, no contraction."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        lib.oracle_row_counts.argtypes = [I, I, P, P, I, P, P, P]
        lib.oracle_row_counts.restype = ctypes.c_int
        lib.oracle_rows.argtypes = [I, I, P, P, P, I, P, P, P, P, P, P]
        lib.oracle_rows.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _canon(M):
    return (np.ascontiguousarray(M.row_ptr, dtype=np.int64),
            np.ascontiguousarray(M.col, dtype=np.int32),
            np.ascontiguousarray(M.val, dtype=np.float64))


def row_counts(A, B, r0: int = 0, r1: int | None = None) -> np.ndarray:
    if A.cols != B.rows:
        raise ValueError("A.cols != B.rows")
    r1 = A.rows if r1 is None else r1
    ap, ac, _ = _canon(A)
    bp, bc, _ = _canon(B)
    counts = np.zeros(max(r1 - r0, 0), dtype=np.int64)
    if r1 > r0 and _load().oracle_row_counts(r0, r1, _p(ap), _p(ac), B.cols, _p(bp), _p(bc), _p(counts)) != 0:
        raise MemoryError("oracle scratch")
    return counts


def spgemm(A, B, r0: int = 0, r1: int | None = None):
    """Rows r0..r1-1 of C = A * B as (row_ptr int64, col int32, val float64);
    row_ptr starts at 0 for row r0."""
    r1 = A.rows if r1 is None else r1
    counts = row_counts(A, B, r0, r1)
    c_ptr = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=c_ptr[1:])
    nnz = int(c_ptr[-1])
    c_col = np.zeros(max(nnz, 1), dtype=np.int32)
    c_val = np.zeros(max(nnz, 1), dtype=np.float64)
    ap, ac, av = _canon(A)
    bp, bc, bv = _canon(B)
    if r1 > r0 and _load().oracle_rows(r0, r1, _p(ap), _p(ac), _p(av), B.cols, _p(bp), _p(bc), _p(bv),
                                       _p(c_ptr), _p(c_col), _p(c_val)) != 0:
        raise MemoryError("oracle scratch")
    return c_ptr, c_col[:nnz], c_val[:nnz]


def spgemm_csr(A, B):
    """Whole product as a ``synth.CSR``-shaped object (duck-typed)."""
    from types import SimpleNamespace
    ptr, col, val = spgemm(A, B)
    return SimpleNamespace(rows=A.rows, cols=B.cols, row_ptr=ptr, col=col, val=val, nnz=int(ptr[-1]))


def features(A, B):
    """Per row i of A: (nnz(A_i), sum_k nnz(B_k), max_k nnz(B_k)) over the
    columns k stored in row i.  The middle one is the number of
    multiplications of row i, an upper bound of nnz(C_i) (Section IV-B)."""
    a_len = np.diff(A.row_ptr).astype(np.int64)
    b_len = np.diff(B.row_ptr).astype(np.int64)
    owner = np.repeat(np.arange(A.rows), a_len)
    sel = b_len[A.col.astype(np.int64)] if A.nnz else np.zeros(0, dtype=np.int64)
    ub = np.bincount(owner, weights=sel, minlength=A.rows).astype(np.int64) if A.nnz else np.zeros(A.rows, np.int64)
    mx = np.zeros(A.rows, dtype=np.int64)
    if A.nnz:
        np.maximum.at(mx, owner, sel)
    return a_len, ub, mx


def multiplications(A, B) -> int:
    """Section III: sum_k abar_k * bbar_k, abar_k = nnz of column k of A,
    bbar_k = nnz of row k of B."""
    abar = np.bincount(A.col.astype(np.int64), minlength=A.cols).astype(np.int64)
    bbar = np.diff(B.row_ptr).astype(np.int64)
    return int(np.dot(abar, bbar))


def transpose(M):
    """The CSR of M^T (a CSC matrix's arrays are the CSR of its transpose;
    Section IV-A converts a right-hand operand stored by columns to rows).
    Plain definition: M's entries (r, c, v) in row order, stably sorted by c,
    so every row of the transpose lists its columns r in increasing order."""
    from types import SimpleNamespace
    rows = np.repeat(np.arange(M.rows, dtype=np.int64), np.diff(M.row_ptr).astype(np.int64))
    col = np.asarray(M.col, dtype=np.int64)
    order = np.argsort(col, kind="stable")
    ptr = np.zeros(M.cols + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(np.bincount(col, minlength=M.cols))
    return SimpleNamespace(rows=M.cols, cols=M.rows, row_ptr=ptr, col=rows[order].astype(np.int32),
                           val=np.asarray(M.val, dtype=np.float64)[order], nnz=int(ptr[-1]))


def flops(A, B) -> int:
    """Section III: the worst-case flop count, twice the multiplications."""
    return 2 * multiplications(A, B)
