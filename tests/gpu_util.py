"""Helpers shared by the GPU tests: run the HIP path, compare with the oracle."""
import numpy as np

import oracle


def bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


def gpu_product(A, B, sizer="exact", model=None, fast=False, tuning=None, validate=False):
    import paper_1303_1651_amd as P
    dA = P.DeviceCSR.from_host(A)
    dB = dA if B is A else P.DeviceCSR.from_host(B)
    res = P.spgemm(dA, dB, sizer=sizer, model=model, fast=fast, tuning=tuning, validate=validate)
    return (res.row_ptr.cpu().numpy(), res.col.cpu().numpy(), res.val.cpu().numpy(), res.info)


def assert_structure_equal(got_ptr, got_col, want_ptr, want_col):
    np.testing.assert_array_equal(got_ptr, want_ptr)
    np.testing.assert_array_equal(got_col, want_col)


def assert_bit_exact(got, want):
    gp, gc, gv = got[:3]
    wp, wc, wv = want
    assert_structure_equal(gp, gc, wp, wc)
    np.testing.assert_array_equal(bits(gv), bits(wv))


def assert_close(got, want, rtol=1e-13):
    """Structure bit-exact; values |d| <= rtol * |ref| per entry."""
    gp, gc, gv = got[:3]
    wp, wc, wv = want
    assert_structure_equal(gp, gc, wp, wc)
    d = np.abs(gv - wv)
    bad = d > rtol * np.abs(wv)
    assert not np.any(bad), "values differ at %d entries, e.g. %s vs %s" % (
        int(bad.sum()), gv[bad][:3], wv[bad][:3])


def oracle_rows(A, B, r0, r1):
    return oracle.spgemm(A, B, r0, r1)


def check_row_blocks(got, A, B, blocks, exact=True):
    """Compare row blocks [r0, r1) of a GPU product with the oracle's row-range product."""
    gp, gc, gv = got[:3]
    for r0, r1 in blocks:
        wp, wc, wv = oracle.spgemm(A, B, r0, r1)
        s, e = int(gp[r0]), int(gp[r1])
        np.testing.assert_array_equal(gp[r0:r1 + 1] - gp[r0], wp)
        np.testing.assert_array_equal(gc[s:e], wc)
        if exact:
            np.testing.assert_array_equal(bits(gv[s:e]), bits(wv))
        else:
            assert np.all(np.abs(gv[s:e] - wv) <= 1e-13 * np.abs(wv))


def sample_blocks(rows, nblocks, width, seed):
    rng = np.random.default_rng(seed)
    starts = {0, max(0, rows - width)}
    starts |= set(int(x) for x in rng.integers(0, max(1, rows - width), nblocks))
    return sorted((s, min(rows, s + width)) for s in starts)


def magnitudes(A, B, r0=0, r1=None):
    """Per entry of C (rows r0..r1), the sum of |a_ik * b_kj| over its
    products: the oracle's product of |A| and |B|."""
    from types import SimpleNamespace
    absA = SimpleNamespace(rows=A.rows, cols=A.cols, row_ptr=A.row_ptr, col=A.col, val=np.abs(A.val))
    absB = SimpleNamespace(rows=B.rows, cols=B.cols, row_ptr=B.row_ptr, col=B.col, val=np.abs(B.val))
    return oracle.spgemm(absA, absB, r0, r1)[2]


def assert_fast_close(got, want, mag, rtol=1e-13):
    """Structure bit-exact; each value within rtol * |c| of the oracle's,
    except where the sum cancels heavily (|c| < 2^-20 * sum |a b|), where it
    is held to rtol * sum |a b| instead.  Returns the number of such entries."""
    gp, gc, gv = got[:3]
    wp, wc, wv = want
    assert_structure_equal(gp, gc, wp, wc)
    d = np.abs(np.asarray(gv) - np.asarray(wv))
    cancel = np.abs(wv) < 2.0 ** -20 * mag
    bound = np.where(cancel, rtol * mag, rtol * np.abs(wv))
    bad = d > bound
    assert not np.any(bad), "values differ at %d entries, e.g. %s vs %s" % (
        int(bad.sum()), np.asarray(gv)[bad][:3], np.asarray(wv)[bad][:3])
    return int(cancel.sum())


def check_device_blocks(rp_dev, col_dev, val_dev, A, B, blocks, base=0):
    """Row blocks [r0, r1) of a product held on the device (row pointers
    relative to `base` in the column and value arrays) against the oracle's
    row-range product, bit for bit; only the blocks are copied to the host."""
    for r0, r1 in blocks:
        rp = rp_dev[r0:r1 + 1].cpu().numpy()
        s, e = base + int(rp[0]), base + int(rp[-1])
        col = col_dev[s:e].cpu().numpy()
        val = val_dev[s:e].cpu().numpy()
        wp, wc, wv = oracle.spgemm(A, B, r0, r1)
        np.testing.assert_array_equal(rp - rp[0], wp)
        np.testing.assert_array_equal(col, wc)
        np.testing.assert_array_equal(bits(val), bits(wv))
