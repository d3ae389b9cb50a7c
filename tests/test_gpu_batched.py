"""Batched products on the GPU: every product of the batch equals the CPU
oracle bit for bit, on the checked first run and on graph replays (with the
program's own GPU work between replays and new values), for every sizer."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_bit_exact

pytestmark = pytest.mark.gpu


def _batch(count, seed, lo=16, hi=600):
    return synth.batch_mix(count, seed, lo=lo, hi=hi)


def _dev(insts):
    import paper_1303_1651_amd as P
    As, Bs = [], []
    for it in insts:
        dA = P.DeviceCSR.from_host(it.A)
        As.append(dA)
        Bs.append(dA if it.B is it.A else P.DeviceCSR.from_host(it.B))
    return As, Bs


def _check_all(batch, insts, wants):
    base, nnz = batch.nnz_base, batch.nnz
    assert base[0] == 0 and np.all(np.diff(base) == nnz)
    for i, want in enumerate(wants):
        rp, col, val = batch.product(i)
        assert_bit_exact((rp, col, val), want)


@pytest.mark.parametrize("sizer", ["upper_bound", "exact"])
def test_batch_equals_oracle_and_replays(sizer):
    import paper_1303_1651_amd as P
    import torch
    insts = _batch(40, 11)
    wants = [oracle.spgemm(it.A, it.B) for it in insts]
    As, Bs = _dev(insts)
    batch = P.Batch(As, Bs, sizer)
    batch.run()
    _check_all(batch, insts, wants)
    assert batch.uses_graph()
    for rep in range(3):
        # other GPU work between replays
        x = torch.randn(1 << 16, device="cuda").cumsum(0)
        one = P.spgemm(As[1], Bs[1], "exact")
        assert_bit_exact((one.row_ptr.cpu().numpy(), one.col.cpu().numpy(), one.val.cpu().numpy()), wants[1])
        batch.col_pool.fill_(-7)
        batch.val_pool.fill_(float("nan"))
        batch.run()
        _check_all(batch, insts, wants)
        del x


def test_replay_sees_new_values():
    import paper_1303_1651_amd as P
    insts = _batch(12, 5)
    As, Bs = _dev(insts)
    batch = P.Batch(As, Bs, "upper_bound")
    batch.run()
    for scale in (2.0, -0.5):
        for i, it in enumerate(insts):
            As[i].val.mul_(scale)
            if Bs[i] is not As[i]:
                Bs[i].val.mul_(scale)
        new = []
        for i, it in enumerate(insts):
            A = synth.CSR(it.A.rows, it.A.cols, it.A.row_ptr, it.A.col, As[i].val.cpu().numpy())
            B = A if it.B is it.A else synth.CSR(it.B.rows, it.B.cols, it.B.row_ptr, it.B.col, Bs[i].val.cpu().numpy())
            new.append(oracle.spgemm(A, B))
        assert batch.uses_graph()
        batch.run()
        _check_all(batch, insts, new)


def test_batch_with_empty_instances_and_learned_sizer():
    import paper_1303_1651_amd as P
    insts = _batch(10, 3)
    empty = synth.CSR(0, 7, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    no_entries = synth.CSR(5, 4, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0))
    b4 = synth.random_sparse(4, 9, 0.5, 2)
    b7 = synth.random_sparse(7, 3, 0.5, 4)
    insts.insert(3, synth.BatchInstance("empty", empty, b7))
    insts.insert(6, synth.BatchInstance("zero", no_entries, b4))
    wants = [oracle.spgemm(it.A, it.B) for it in insts]
    As, Bs = _dev(insts)
    # a network that predicts the smallest size for every row: capacities
    # fall short, rows spill or are computed again with their exact size,
    # and the pools grow once
    theta = np.zeros(1217, np.float32)
    theta[-1] = -30.0
    model = P.Model.create(theta, [0, 0, 0], [1, 1, 1])
    batch = P.Batch(As, Bs, "learned", model=model)
    batch.run()
    _check_all(batch, insts, wants)
    batch.run()
    _check_all(batch, insts, wants)


def test_batch_matches_per_instance_products():
    import paper_1303_1651_amd as P
    insts = _batch(16, 21, lo=256, hi=4096)
    As, Bs = _dev(insts)
    batch = P.Batch(As, Bs, "upper_bound")
    batch.run()
    for i, it in enumerate(insts):
        want = oracle.spgemm(it.A, it.B)
        one = P.spgemm(As[i], Bs[i], "exact")
        assert_bit_exact(batch.product(i), want)
        assert_bit_exact((one.row_ptr.cpu().numpy(), one.col.cpu().numpy(), one.val.cpu().numpy()), want)


def test_batch_autotuner_picks_a_valid_tuning_and_stays_exact():
    import paper_1303_1651_amd as P
    from paper_1303_1651_amd.autotune import autotune_batch
    insts = _batch(24, 41, lo=64, hi=2048)
    wants = [oracle.spgemm(it.A, it.B) for it in insts]
    As, Bs = _dev(insts)
    grid = {"table_slots": [512, 1024], "dense_ratio": [1.0, 2.0]}
    best, cands = autotune_batch(As, Bs, "exact", grid=grid, reps=1)
    assert len(cands) == 4 and best in [t for _, t in cands]
    batch = P.Batch(As, Bs, "exact", tuning=best)
    batch.run()
    batch.run()
    _check_all(batch, insts, wants)
