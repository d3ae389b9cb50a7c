"""GPU parity at the shapes of the measured workloads (through the C ABI):
the power-law product N = 2^20 in full with every sizer, the learned one
trained on 2^22 rows of symbolic-pass output; the 9-point 2048 x 2048 and
27-point 160^3 squares, plain and learned, alone and together in one batch,
on sampled 4,096-row blocks plus their closed-form sizes; a batch of
instances with sizes log-uniform in [256, 65536] on sampled instances.
Structure and values must equal the oracle's bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import (assert_bit_exact, assert_fast_close, check_device_blocks, gpu_product, magnitudes,
                            sample_blocks)

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[configs] " + msg, flush=True)


def _dev(M):
    import paper_1303_1651_amd as P
    return P.DeviceCSR.from_host(M)


# ---------------------------------------------------------- power law 2^20
@pytest.fixture(scope="module")
def zipf():
    A = synth.zipf_matrix(1 << 20, 3)
    return A, oracle.spgemm(A, A)


@pytest.fixture(scope="module")
def zipf_model():
    # four matrices of 2^20 rows with seeds disjoint from the evaluation
    # seed: 2^22 rows of (features, exact size) pairs
    import paper_1303_1651_amd as P
    pairs = []
    for s in range(1001, 1005):
        d = _dev(synth.zipf_matrix(1 << 20, s))
        pairs.append((d, d))
    model, facts = P.fit_model(pairs, seed=1001, epochs=10, batch_size=16384)
    assert facts["train_rows"] == 1 << 22
    return model


@pytest.mark.parametrize("sizer", ["exact", "upper_bound"])
def test_zipf_2pow20_full(zipf, sizer):
    A, want = zipf
    _say("zipf 2^20 " + sizer)
    got = gpu_product(A, A, sizer)
    assert got[3]["multiplications"] == oracle.multiplications(A, A)
    assert got[3]["rows_global"] > 0
    assert_bit_exact(got, want)


def test_zipf_2pow20_learned_full(zipf, zipf_model):
    A, want = zipf
    _say("zipf 2^20 learned")
    got = gpu_product(A, A, "learned", model=zipf_model)
    assert_bit_exact(got, want)
    # the capacities stay within a few percent of nnz(C)
    assert got[3]["c_capacity_hint"] <= 1.1 * int(want[0][-1])


def test_zipf_2pow20_fast_mode(zipf):
    # FAST reorders the adds of workgroup-tier rows (every row here): each
    # entry within 1e-13 of the oracle's value, or of its magnitude sum where
    # the sum cancels
    A, want = zipf
    _say("zipf 2^20 fast")
    got = gpu_product(A, A, "exact", fast=True, tuning={"merge_max_nnz": -1, "table_slots": -1})
    n_cancel = assert_fast_close(got, want, magnitudes(A, A), 1e-13)
    _say("fast mode: %d entries under the cancellation rule" % n_cancel)


# -------------------------------------------------- 9- and 27-point squares
WIDE = {"st9": (2048, 2, 9), "st27": (160, 3, 27)}


@pytest.fixture(scope="module")
def wide():
    return {k: synth.stencil(n, d, p) for k, (n, d, p) in WIDE.items()}


@pytest.fixture(scope="module")
def stencil_model():
    # smaller grids of the same stencils (disjoint sizes stand in for
    # disjoint seeds: stencils are deterministic)
    import paper_1303_1651_amd as P
    srcs = [synth.stencil(g) for g in (64, 96, 128)]
    srcs += [synth.stencil(g, d, p) for p, d, g in ((9, 2, 64), (9, 2, 96), (27, 3, 16), (27, 3, 24))]
    pairs = [(d, d) for d in map(_dev, srcs)]
    model, _ = P.fit_model(pairs, seed=1002, per_source=1 << 16, epochs=30)
    return model


def _closed_form(key):
    n, d, _ = WIDE[key]
    return (5 * n - 6) ** d, (9 * n - 10) ** d


@pytest.mark.parametrize("key", list(WIDE))
@pytest.mark.parametrize("sizer", ["exact", "learned"])
def test_wide_stencil_full_shape_sampled_blocks(wide, stencil_model, key, sizer):
    import paper_1303_1651_amd as P
    A = wide[key]
    _say("%s %s" % (key, sizer))
    dA = _dev(A)
    res = P.spgemm(dA, dA, sizer=sizer, model=stencil_model if sizer == "learned" else None)
    nnz, mults = _closed_form(key)
    assert res.info["multiplications"] == mults
    assert int(res.row_ptr[-1]) == nnz and res.nnz == nnz
    assert bool((res.row_ptr[1:] >= res.row_ptr[:-1]).all())
    check_device_blocks(res.row_ptr, res.col, res.val, A, A, sample_blocks(A.rows, 16, 4096, 5))


def test_wide_stencils_in_one_learned_batch(wide, stencil_model):
    # the learned sizer and the batched launch together: both squares as one
    # batch, checked on sampled blocks of each product, on the first run and
    # on a graph replay
    import paper_1303_1651_amd as P
    _say("st9 + st27 learned batch")
    mats = [wide["st9"], wide["st27"]]
    ds = [_dev(M) for M in mats]
    batch = P.Batch(ds, ds, "learned", model=stencil_model)
    for run in range(2):
        base, nnz = batch.run()
        for i, key in enumerate(("st9", "st27")):
            want_nnz, _ = _closed_form(key)
            assert nnz[i] == want_nnz
            rb = int(batch.row_base[i])
            rp = batch.row_pool[rb:rb + mats[i].rows + 1]
            check_device_blocks(rp, batch.col_pool, batch.val_pool, mats[i], mats[i],
                                sample_blocks(mats[i].rows, 8, 4096, 10 + run), base=int(base[i]))
    assert batch.uses_graph()
    batch.close()


# -------------------------------------------- batch with sizes to 65,536
@pytest.fixture(scope="module")
def big_batch():
    insts = synth.batch_mix(256, 4, lo=256, hi=65536)
    sizes = np.array([it.A.rows for it in insts])
    assert sizes.max() > 30000 and sizes.min() < 1000
    return insts


@pytest.mark.parametrize("sizer", ["exact", "upper_bound", "learned"])
def test_batch_sizes_to_65536_sampled_instances(big_batch, sizer):
    import paper_1303_1651_amd as P
    _say("batch 256 " + sizer)
    insts = big_batch
    As, Bs = [], []
    for it in insts:
        dA = _dev(it.A)
        As.append(dA)
        Bs.append(dA if it.B is it.A else _dev(it.B))
    model = None
    if sizer == "learned":
        train = synth.batch_mix(48, 1004, lo=256, hi=8192)
        pairs = []
        for it in train:
            dA = _dev(it.A)
            pairs.append((dA, dA if it.B is it.A else _dev(it.B)))
        model, _ = P.fit_model(pairs, seed=1004, epochs=20)
    batch = P.Batch(As, Bs, sizer, model=model)
    base, nnz = batch.run()
    # every instance's size from the oracle's row counts
    want_nnz = np.array([int(oracle.row_counts(it.A, it.B).sum()) for it in insts])
    np.testing.assert_array_equal(nnz, want_nnz)
    rng = np.random.default_rng(9)
    picks = sorted(set(rng.choice(len(insts), 12, replace=False).tolist()) | {0, len(insts) - 1,
                                                                             int(np.argmax([it.A.rows for it in insts]))})
    for i in picks:
        assert_bit_exact(batch.product(i), oracle.spgemm(insts[i].A, insts[i].B))
    batch.close()
