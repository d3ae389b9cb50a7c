"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function that include/spgemm.h declares, and rejects bad descriptors
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spgemm.h")
LIB = os.path.join(ROOT, "paper_1303_1651_amd", "libspgemm.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(spgemm_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for n in ["spgemm_plan_create", "spgemm_symbolic", "spgemm_numeric", "spgemm_batched"]:
        assert n in names


def test_library_exports_every_declared_function(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    lib.spgemm_status_string.restype = ctypes.c_char_p
    assert lib.spgemm_status_string(0) == b"ok"
    assert lib.spgemm_status_string(6) == b"output capacity too small"
    assert lib.spgemm_status_string(99) == b"unknown status"


def test_descriptor_errors_before_any_device_call():
    from paper_1303_1651_amd import _lib as L
    A = L.spgemm_csr(10, 5, 0, 1, None, None)
    B = L.spgemm_csr(6, 5, 0, 1, None, None)    # A.cols != B.rows
    opts = L.spgemm_options(0, 0, None, None)
    nb = L.SZ()
    assert L.spgemm_plan_workspace_size(ctypes.byref(A), ctypes.byref(B), ctypes.byref(opts), ctypes.byref(nb)) == 2
    B.rows = 5
    assert L.spgemm_plan_workspace_size(ctypes.byref(A), ctypes.byref(B), ctypes.byref(opts), ctypes.byref(nb)) == 0
    assert nb.value > 0
    A.nnz = 3                                     # nnz > 0 but no column array
    assert L.spgemm_plan_workspace_size(ctypes.byref(A), ctypes.byref(B), ctypes.byref(opts), ctypes.byref(nb)) == 1
    A.nnz = 0
    A.cols = B.rows = 1 << 31                     # columns beyond int32
    assert L.spgemm_plan_workspace_size(ctypes.byref(A), ctypes.byref(B), ctypes.byref(opts), ctypes.byref(nb)) == 4
    A.rows = -1
    assert L.spgemm_plan_workspace_size(ctypes.byref(A), ctypes.byref(B), ctypes.byref(opts), ctypes.byref(nb)) == 2


def test_learned_sizer_without_model_is_rejected():
    from paper_1303_1651_amd import _lib as L
    A = L.spgemm_csr(4, 4, 0, 1, None, None)
    opts = L.spgemm_options(2, 0, None, None)
    plan = ctypes.c_void_p()
    code = L.spgemm_plan_create(ctypes.byref(A), ctypes.byref(A), ctypes.byref(opts), 1, 1 << 20, None,
                                ctypes.byref(plan), None)
    assert code == 7 and not plan.value


def test_invalid_tuning_is_rejected():
    from paper_1303_1651_amd import _lib as L
    A = L.spgemm_csr(4, 4, 0, 1, None, None)
    for bad in (dict(table_slots=300), dict(stage_slots=100), dict(stage_slots=9000),
                dict(merge_lists=6), dict(spill_ratio=5.0)):
        t = L.spgemm_tuning(**bad)
        opts = L.spgemm_options(0, 0, None, ctypes.pointer(t))
        plan = ctypes.c_void_p()
        code = L.spgemm_plan_create(ctypes.byref(A), ctypes.byref(A), ctypes.byref(opts), 256, 1 << 20, None,
                                    ctypes.byref(plan), None)
        assert code == 10, bad


def test_unaligned_workspace_is_rejected():
    # checked before any device work: the workspace holds 16-byte records
    from paper_1303_1651_amd import _lib as L
    A = L.spgemm_csr(4, 4, 0, 1, None, None)
    opts = L.spgemm_options(0, 0, None, None)
    plan = ctypes.c_void_p()
    for ws in (8, 16, 272):
        code = L.spgemm_plan_create(ctypes.byref(A), ctypes.byref(A), ctypes.byref(opts), ws, 1 << 20, None,
                                    ctypes.byref(plan), None)
        assert code == 5 and not plan.value, ws


def test_model_file_round_trip(tmp_path):
    import numpy as np
    from paper_1303_1651_amd import Model
    th = np.linspace(-1, 1, 1217).astype(np.float32)
    m = Model.create(th, [1, 2, 3], [4, 5, 6])
    p = str(tmp_path / "m.bin")
    m.save(p)
    m2 = Model.load(p)
    th2, mu2, sd2 = m2.params()
    np.testing.assert_array_equal(th2, th)
    np.testing.assert_array_equal(mu2, [1, 2, 3])
    np.testing.assert_array_equal(sd2, [4, 5, 6])
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"not a model")
    with pytest.raises(Exception):
        Model.load(str(bad))


def test_model_with_non_finite_or_bad_scale_is_rejected(tmp_path):
    import numpy as np
    from paper_1303_1651_amd import Model
    from paper_1303_1651_amd._lib import SpgemmError
    th = np.zeros(1217, np.float32)
    for bad_th, mu, sd in [(np.nan, [0, 0, 0], [1, 1, 1]), (np.inf, [0, 0, 0], [1, 1, 1]),
                           (0.0, [0, np.nan, 0], [1, 1, 1]), (0.0, [0, 0, 0], [1, 0, 1]),
                           (0.0, [0, 0, 0], [1, 1, -2]), (0.0, [0, 0, 0], [1, np.inf, 1])]:
        t = th.copy()
        t[5] = bad_th
        with pytest.raises(SpgemmError) as e:
            Model.create(t, mu, sd)
        assert e.value.code == 10          # SPGEMM_E_INVALID
    # a file holding a NaN weight is refused by the loader the same way
    good = Model.create(th, [0, 0, 0], [1, 1, 1])
    p = str(tmp_path / "m.bin")
    good.save(p)
    raw = bytearray(open(p, "rb").read())
    raw[12 + 4 * 7:12 + 4 * 8] = np.array([np.nan], np.float32).tobytes()
    open(p, "wb").write(bytes(raw))
    with pytest.raises(SpgemmError) as e:
        Model.load(p)
    assert e.value.code == 10


def test_batched_plan_checks_descriptors_without_a_device():
    from paper_1303_1651_amd import _lib as L
    opts = L.spgemm_options(1, 0, None, None)
    A = (L.spgemm_csr * 2)(L.spgemm_csr(4, 3, 0, 1, None, None), L.spgemm_csr(2, 5, 0, 1, None, None))
    B = (L.spgemm_csr * 2)(L.spgemm_csr(3, 4, 0, 1, None, None), L.spgemm_csr(4, 2, 0, 1, None, None))
    rb = (ctypes.c_int64 * 3)()
    ws = L.SZ()
    h = ctypes.c_void_p()
    # instance 1: A.cols (5) != B.rows (4)
    assert L.spgemm_batched_plan(2, A, B, ctypes.byref(opts), rb, ctypes.byref(ws), ctypes.byref(h)) == 2
    assert not h.value
    # learned sizing without a model
    lo = L.spgemm_options(2, 0, None, None)
    assert L.spgemm_batched_plan(1, A, B, ctypes.byref(lo), rb, ctypes.byref(ws), ctypes.byref(h)) == 7


def test_transpose_host_checks():
    # refused before any device work
    from paper_1303_1651_amd import _lib as L
    M = L.spgemm_csr(4, 3, 0, 256, None, None)
    assert L.spgemm_transpose_scratch(ctypes.byref(M)) > 0
    assert L.spgemm_transpose(None, 256, 256, None, 256, 1 << 20, None) == 1
    assert L.spgemm_transpose(ctypes.byref(M), None, 256, None, 256, 1 << 20, None) == 1
    bad = L.spgemm_csr(-1, 3, 0, 256, None, None)
    assert L.spgemm_transpose(ctypes.byref(bad), 256, 256, None, 256, 1 << 20, None) == 2
    big = L.spgemm_csr(1 << 31, 3, 0, 256, None, None)
    assert L.spgemm_transpose(ctypes.byref(big), 256, 256, None, 256, 1 << 20, None) == 4
    assert L.spgemm_transpose(ctypes.byref(M), 256, 256, None, 264, 1 << 20, None) == 5   # unaligned
    assert L.spgemm_transpose(ctypes.byref(M), 256, 256, None, 256, 16, None) == 5       # too small
    withnnz = L.spgemm_csr(4, 3, 5, 256, None, None)                                     # no columns
    assert L.spgemm_transpose(ctypes.byref(withnnz), 256, 256, None, 256, 1 << 20, None) == 1
