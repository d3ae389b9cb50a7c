"""Seeded synthetic CSR inputs shared by the oracle, the tests and the bench.

This module holds no part of the product's arithmetic: it only builds input
matrices (structure plus values) from seeds.  Every random number comes from
SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) used in counter mode: draw ``i`` of stream ``s`` is
the SplitMix64 finaliser applied to ``s + (i + 1) * 0x9E3779B97F4A7C15``,
which is exactly the ``i``-th output of a SplitMix64 generator seeded with
``s``.

Workloads follow the paper's test cases (Section III): the five-point
finite-difference stencil of a Dirichlet problem on a square ("FD"), and square
random matrices with a fixed number of entries at random places in every row
("random").  The 9-point and 27-point stencils, the random matrix with exactly
``k`` distinct columns, the power-law row lengths and the batched mix extend
those recipes to the sizes this project measures.

CSR convention: ``row_ptr`` int64 (rows + 1), ``col`` int32 strictly
increasing inside each row, ``val`` float64.
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


@dataclass
class CSR:
    rows: int
    cols: int
    row_ptr: np.ndarray  # int64, rows + 1
    col: np.ndarray      # int32, nnz
    val: np.ndarray      # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row(self, i: int):
        s, e = int(self.row_ptr[i]), int(self.row_ptr[i + 1])
        return self.col[s:e], self.val[s:e]

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.rows, self.cols))
        r = np.repeat(np.arange(self.rows), np.diff(self.row_ptr))
        d[r, self.col] = self.val
        return d


# ---------------------------------------------------------------- random bits
def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 output number ``counters`` of the stream seeded with ``seed``."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (counters.astype(np.uint64) + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _sub_seed(seed: int, tag: int) -> int:
    """Independent stream for a (seed, purpose) pair: one SplitMix64 draw."""
    return int(splitmix64(seed, np.array([tag], dtype=np.uint64))[0])


def uniform_pm1(bits: np.ndarray) -> np.ndarray:
    """U(-1, 1) from the top 53 bits: 2 * (b >> 11) * 2^-53 - 1."""
    return 2.0 * ((bits >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)) - 1.0


def uniform_index(bits: np.ndarray, n: int) -> np.ndarray:
    """Index in [0, n) from the top 32 bits: (b >> 32) * n >> 32."""
    return (((bits >> np.uint64(32)) * np.uint64(n)) >> np.uint64(32)).astype(np.int64)


# ------------------------------------------------------------------ stencils
def _from_coo_sorted(rows: int, cols: int, r: np.ndarray, c: np.ndarray, v: np.ndarray) -> CSR:
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    row_ptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=rows), out=row_ptr[1:])
    return CSR(rows, cols, row_ptr, c.astype(np.int32), v.astype(np.float64))


def stencil(n: int, dim: int = 2, points: int = 5, diag: float | None = None, off: float = -1.0) -> CSR:
    """Finite-difference stencil matrix on an n^dim grid, Dirichlet boundary.

    Grid point (x, y[, z]) has index x + n*y (+ n*n*z).  Neighbours outside the
    grid are dropped (truncated stencil).  ``points`` = 5 (2-D, axis
    neighbours), 9 (2-D, all neighbours within Chebyshev distance 1) or 27
    (3-D, likewise).  ``diag`` defaults to the number of neighbours of an
    interior point (4, 8 or 26) and ``off`` to -1.
    """
    if (dim, points) not in ((2, 5), (2, 9), (3, 27)):
        raise ValueError("supported stencils: 2-D 5-point, 2-D 9-point, 3-D 27-point")
    if diag is None:
        diag = float(points - 1)
    if points == 5:
        offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
        offs = [o + (0,) for o in offs]
    elif points == 9:
        offs = [(dx, dy, 0) for dx in (-1, 0, 1) for dy in (-1, 0, 1)]
    else:
        offs = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)]
    N = n ** dim
    idx = np.arange(N, dtype=np.int64)
    x = idx % n
    y = (idx // n) % n
    z = idx // (n * n) if dim == 3 else np.zeros_like(idx)
    rs, cs, vs = [], [], []
    for dx, dy, dz in offs:
        xx, yy, zz = x + dx, y + dy, z + dz
        ok = (xx >= 0) & (xx < n) & (yy >= 0) & (yy < n)
        if dim == 3:
            ok &= (zz >= 0) & (zz < n)
        j = xx + n * yy + n * n * zz
        rs.append(idx[ok])
        cs.append(j[ok])
        vs.append(np.full(int(ok.sum()), diag if (dx, dy, dz) == (0, 0, 0) else off))
    return _from_coo_sorted(N, N, np.concatenate(rs), np.concatenate(cs), np.concatenate(vs))


# --------------------------------------------------------------- random rows
def random_rows(rows: int, cols: int, lengths: np.ndarray, seed: int) -> CSR:
    """Row i gets ``lengths[i]`` distinct uniform-random columns, values U(-1, 1).

    Columns are drawn in rounds: every row draws its missing entries, the row
    is sorted and de-duplicated, and rows still short draw again from fresh
    counters.  Values are assigned after the columns are fixed, one draw per
    stored entry, so they do not depend on the number of rounds.
    """
    lengths = np.asarray(lengths, dtype=np.int64)
    if rows and lengths.max(initial=0) > cols:
        raise ValueError("row length exceeds the number of columns")
    row_ptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col_seed = _sub_seed(seed, 1)
    val_seed = _sub_seed(seed, 2)
    owner = np.repeat(np.arange(rows, dtype=np.int64), lengths)
    have_r = np.empty(0, dtype=np.int64)
    have_c = np.empty(0, dtype=np.int64)
    need = lengths.copy()
    counter = 0
    while True:
        tot = int(need.sum())
        if tot == 0:
            break
        r = np.repeat(np.arange(rows, dtype=np.int64), need)
        bits = splitmix64(col_seed, np.arange(counter, counter + tot, dtype=np.uint64))
        counter += tot
        c = uniform_index(bits, cols)
        allr = np.concatenate([have_r, r])
        allc = np.concatenate([have_c, c])
        key = allr * cols + allc
        key = np.unique(key)                     # sorted, distinct
        have_r, have_c = key // cols, key % cols
        got = np.bincount(have_r, minlength=rows)
        # a row may have drawn more distinct columns than needed only if it had
        # duplicates in an earlier round; keep the first `lengths` by draw order
        # is unnecessary: unique() only removes, so got <= lengths always.
        need = lengths - got
    assert have_r.shape[0] == nnz and np.array_equal(have_r, owner)
    val = uniform_pm1(splitmix64(val_seed, np.arange(nnz, dtype=np.uint64)))
    return CSR(rows, cols, row_ptr, have_c.astype(np.int32), val)


def random_fixed(n: int, k: int, seed: int, cols: int | None = None) -> CSR:
    """n x cols matrix with exactly k distinct random columns per row."""
    cols = n if cols is None else cols
    return random_rows(n, cols, np.full(n, k, dtype=np.int64), seed)


def random_fill(n: int, fill: float, seed: int) -> CSR:
    """n x n matrix with ceil(fill * n) distinct uniform-random columns per
    row, values U(-1, 1): the random test case at a fixed fill (0.1 % in the
    storing-strategy study of Section IV-B, whose product rows then hold
    about (0.001 n)^2 entries spread over all n columns)."""
    return random_fixed(n, max(1, int(math.ceil(fill * n - 1e-9))), seed)


def random_uniform_lengths(n: int, lo: int, hi: int, seed: int) -> CSR:
    """Square n x n matrix, row lengths uniform in {lo..hi} (capped at n)."""
    bits = splitmix64(_sub_seed(seed, 3), np.arange(n, dtype=np.uint64))
    lengths = np.minimum(lo + uniform_index(bits, hi - lo + 1), n)
    return random_rows(n, n, lengths, seed)


def zipf_lengths(n: int, s: float, lmax: int, seed: int) -> np.ndarray:
    """Row lengths L >= 1 with P(L = l) = l^-s / zeta(s) for l < lmax and the
    whole tail mass P(L >= lmax) put on lmax (clipping, not renormalising)."""
    ls = np.arange(1, lmax, dtype=np.float64)
    zeta = math.pi ** 2 / 6.0 if s == 2.0 else float(np.sum(np.arange(1, 10**7, dtype=np.float64) ** -s))
    p = ls ** -s / zeta
    cdf = np.cumsum(p)
    u = (splitmix64(_sub_seed(seed, 4), np.arange(n, dtype=np.uint64)) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    lengths = np.searchsorted(cdf, u, side="right") + 1    # u >= cdf[-1] -> lmax
    return np.minimum(lengths, lmax).astype(np.int64)


def zipf_matrix(n: int, seed: int, s: float = 2.0, lmax: int = 4096) -> CSR:
    lengths = np.minimum(zipf_lengths(n, s, lmax, seed), n)
    return random_rows(n, n, lengths, seed)


def identity(n: int) -> CSR:
    return CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.ones(n))


def permutation(perm: np.ndarray, values: np.ndarray | None = None) -> CSR:
    n = perm.shape[0]
    v = np.ones(n) if values is None else values.astype(np.float64)
    return CSR(n, n, np.arange(n + 1, dtype=np.int64), perm.astype(np.int32), v)


def random_sparse(m: int, k: int, density: float, seed: int, integer: bool = False) -> CSR:
    """m x k matrix, each entry present with probability ``density``;
    values U(-1, 1) or small integers in [-3, 3] when ``integer``."""
    tot = m * k
    bits = splitmix64(_sub_seed(seed, 5), np.arange(tot, dtype=np.uint64))
    present = ((bits >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)) < density
    idx = np.nonzero(present)[0]
    r, c = idx // max(k, 1), idx % max(k, 1)
    vb = splitmix64(_sub_seed(seed, 6), np.arange(idx.shape[0], dtype=np.uint64))
    if integer:
        v = (uniform_index(vb, 7) - 3).astype(np.float64)
    else:
        v = uniform_pm1(vb)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=m), out=row_ptr[1:])
    return CSR(m, k, row_ptr, c.astype(np.int32), v)


# ------------------------------------------------------------------- batched
@dataclass
class BatchInstance:
    kind: str        # "stencil5" or "random"
    A: CSR
    B: CSR


def batch_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Sizes log-uniform in [lo, hi]."""
    u = (splitmix64(_sub_seed(seed, 7), np.arange(count, dtype=np.uint64)) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def batch_mix(count: int, seed: int, lo: int = 256, hi: int = 65536, rmin: int = 4, rmax: int = 32):
    """Independent products C_i = A_i * B_i: even i a 5-point stencil squared on
    a round(sqrt(N_i))^2 grid (B_i = A_i), odd i random with U{rmin..rmax}
    entries per row and an independent B_i."""
    sizes = batch_sizes(count, lo, hi, seed)
    out = []
    for i, n in enumerate(sizes):
        if i % 2 == 0:
            g = max(2, int(round(math.sqrt(int(n)))))
            A = stencil(g, 2, 5, 4.0, -1.0)
            out.append(BatchInstance("stencil5", A, A))
        else:
            n = int(n)
            A = random_uniform_lengths(n, rmin, rmax, _sub_seed(seed, 1000 + 2 * i))
            B = random_uniform_lengths(n, rmin, rmax, _sub_seed(seed, 1001 + 2 * i))
            out.append(BatchInstance("random", A, B))
    return out


# ------------------------------------------------ row-size network start
def mlp_init(seed: int, hidden: int = 32) -> np.ndarray:
    """Starting parameters of the 3-32-32-1 row-size network, flat in the
    order W1 (32x3), b1, W2 (32x32), b2, w3, b3: weights uniform in
    +-sqrt(6 / fan_in) (He et al., 2015, uniform form), biases zero."""
    u = uniform_pm1(splitmix64(_sub_seed(seed, 8), np.arange(hidden * 3 + hidden * hidden + hidden, dtype=np.uint64)))
    w1 = u[:hidden * 3] * math.sqrt(6.0 / 3.0)
    w2 = u[hidden * 3:hidden * 3 + hidden * hidden] * math.sqrt(6.0 / hidden)
    w3 = u[hidden * 3 + hidden * hidden:] * math.sqrt(6.0 / hidden)
    z = np.zeros(hidden)
    return np.concatenate([w1, z, w2, z, w3, [0.0]])
