"""The learned row-size network on the GPU: gradients and predictions against
the FP64 oracle, training, and the one-pass product it sizes (which must
still equal the oracle bit for bit, whatever the network predicts)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp_ref
from tests.gpu_util import assert_bit_exact, gpu_product

pytestmark = pytest.mark.gpu


def _features_labels(A, B):
    f1, ub, mx = oracle.features(A, B)
    n = oracle.row_counts(A, B)
    return f1, np.minimum(ub, B.cols), mx, n


def _to_dev(*arrs):
    import torch
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).cuda() for a in arrs]


def _model(seed=3):
    import paper_1303_1651_amd as P
    theta = synth.mlp_init(seed).astype(np.float32)
    mu = np.array([2.0, 5.0, 3.0], np.float32)
    sd = np.array([1.5, 2.5, 1.7], np.float32)
    return P.Model.create(theta, mu, sd), theta.astype(np.float64), mu.astype(np.float64), sd.astype(np.float64)


def test_device_features_match_oracle():
    import paper_1303_1651_amd as P
    A = synth.zipf_matrix(20000, 21)
    dA = P.DeviceCSR.from_host(A)
    f1, f2, f3 = P.row_features(dA, dA)
    o1, o2, o3 = oracle.features(A, A)
    np.testing.assert_array_equal(f1.cpu().numpy(), o1)
    np.testing.assert_array_equal(f2.cpu().numpy(), np.minimum(o2, A.cols))
    np.testing.assert_array_equal(f3.cpu().numpy(), o3)


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_fp64_oracle(seed):
    A = synth.zipf_matrix(3000, 30 + seed)
    f1, f2, f3, n = _features_labels(A, A)
    model, theta, mu, sd = _model(seed)
    d1, d2, d3, dn = _to_dev(f1, f2, f3, n)
    loss, grad = model.loss_grad(d1, d2, d3, dn)
    X = mlp_ref.inputs(f1, f2, f3, mu, sd)
    t, w = mlp_ref.targets(n, f2, f3)
    L, g = mlp_ref.loss_and_grad(theta, X, t, w)
    assert abs(loss - L) <= 1e-4 * abs(L) + 1e-7
    gg = grad.cpu().numpy().astype(np.float64)
    scale = np.max(np.abs(g))
    np.testing.assert_allclose(gg, g, rtol=1e-4, atol=1e-5 * scale)


def test_prediction_matches_fp64_oracle():
    A = synth.zipf_matrix(50000, 40)
    f1, f2, f3, n = _features_labels(A, A)
    model, theta, mu, sd = _model(5)
    d1, d2, d3 = _to_dev(f1, f2, f3)
    p = model.predict(d1, d2, d3).cpu().numpy().astype(np.float64)
    want = mlp_ref.predict(theta, mu, sd, f1, f2, f3)
    np.testing.assert_allclose(p, want, rtol=1e-4, atol=1e-3)
    assert np.all(p >= f3 - 1e-3) and np.all(p <= f2 + 1e-3)


def test_training_lowers_loss_and_tracks_oracle_step():
    import paper_1303_1651_amd as P
    A = synth.zipf_matrix(1 << 15, 50)
    f1, f2, f3, n = _features_labels(A, A)
    d1, d2, d3, dn = _to_dev(f1, f2, f3, n)
    mu, sd = P.feature_stats(d1, d2, d3)
    want_mu = np.log2(1.0 + np.stack([f1, f2, f3], 1)).mean(0)
    np.testing.assert_allclose(mu, want_mu, rtol=1e-5)
    theta0 = synth.mlp_init(7)
    # one full-batch Adam step on the GPU equals the oracle's step
    m1, curve = P.train_model(theta0, mu, sd, d1, d2, d3, dn, epochs=1, batch_size=1 << 15, lr=1e-3)
    th1 = m1.params()[0].astype(np.float64)
    X = mlp_ref.inputs(f1, f2, f3, mu.astype(np.float64), sd.astype(np.float64))
    t, w = mlp_ref.targets(n, f2, f3)
    th0 = theta0.astype(np.float32).astype(np.float64)
    _, g = mlp_ref.loss_and_grad(th0, X, t, w)
    want, _, _ = mlp_ref.adam_step(th0, g, np.zeros_like(th0), np.zeros_like(th0), 1, 1e-3)
    # Adam's first step moves every parameter by ~lr * sign(g); compare where |g| is not tiny
    big = np.abs(g) > 1e-3 * np.max(np.abs(g))
    np.testing.assert_allclose(th1[big], want[big], rtol=0, atol=2e-5)
    # many epochs lower the loss
    m2, curve2 = P.train_model(theta0, mu, sd, d1, d2, d3, dn, epochs=30, batch_size=4096, lr=3e-3)
    L0 = mlp_ref.loss(th0, X, t, w)
    L1 = mlp_ref.loss(m2.params()[0].astype(np.float64), X, t, w)
    assert L1 < 0.5 * L0


def _trained_model():
    import paper_1303_1651_amd as P
    import torch
    mats = [synth.zipf_matrix(1 << 15, 60 + i) for i in range(2)] + [synth.stencil(48), synth.random_fixed(4096, 8, 9)]
    fs, ls = [], []
    for M in mats:
        f1, f2, f3, n = _features_labels(M, M)
        fs.append(np.stack([f1, f2, f3]))
        ls.append(n)
    F = np.concatenate(fs, axis=1)
    L = np.concatenate(ls)
    perm = np.random.default_rng(0).permutation(F.shape[1])
    d1, d2, d3, dn = _to_dev(F[0][perm], F[1][perm], F[2][perm], L[perm])
    mu, sd = P.feature_stats(d1, d2, d3)
    model, _ = P.train_model(synth.mlp_init(11), mu, sd, d1, d2, d3, dn, epochs=15, batch_size=4096, lr=3e-3)
    return model


@pytest.fixture(scope="module")
def trained():
    return _trained_model()


@pytest.mark.parametrize("case", ["stencil64", "zipf", "random", "stencil27"])
def test_learned_product_equals_oracle(trained, case):
    if case == "stencil64":
        A = B = synth.stencil(64)
    elif case == "zipf":
        A = B = synth.zipf_matrix(40000, 3)
    elif case == "random":
        A = synth.random_uniform_lengths(6000, 4, 32, 5)
        B = synth.random_uniform_lengths(6000, 4, 32, 6)
    else:
        A = B = synth.stencil(14, 3, 27)
    want = oracle.spgemm(A, B)
    for tier in [None, {"merge_max_nnz": -1}, {"merge_max_nnz": -1, "table_slots": 256, "stage_slots": 256}]:
        got = gpu_product(A, B, "learned", model=trained, tuning=tier)
        assert_bit_exact(got, want)


def test_bad_model_still_gives_exact_product():
    # a network that predicts the smallest size for every row, with no spill
    # arena, sends the rows their tiles have no room for to the exact path;
    # the product must not change
    import paper_1303_1651_amd as P
    theta = np.zeros(1217, np.float32)
    theta[-1] = -30.0                   # rho ~ 0: predict the longest B row
    model = P.Model.create(theta, [0, 0, 0], [1, 1, 1])
    A = synth.zipf_matrix(30000, 8)
    want = oracle.spgemm(A, A)
    for tuning in ({"merge_max_nnz": -1, "spill_ratio": -1}, {"spill_ratio": -1}):
        got = gpu_product(A, A, "learned", model=model, tuning=tuning)
        assert_bit_exact(got, want)
        assert got[3]["overflow_rows"] > 0 and got[3]["spilled_rows"] == 0


@pytest.mark.parametrize("case", ["zipf", "stencil"])
def test_network_that_overflows_to_nan_sizes_rows_by_their_bound(case):
    # every weight is finite (the model is accepted), but in FP32 the output
    # layer adds two products that each overflow to opposite infinities:
    # z = 1e30 * h - 1e30 * h with h = 1e30 * relu(x0) is NaN (or, fused,
    # infinite) on the device, 0 in exact arithmetic.  A prediction that is
    # not a number inside [longest B row, bound] sizes the row by its bound;
    # the product must still equal the oracle bit for bit.
    import paper_1303_1651_amd as P
    W1 = np.zeros((32, 3)); W1[0, 0] = 1.0; W1[1, 0] = 1.0
    W2 = np.zeros((32, 32)); W2[0, 0] = 1e30; W2[1, 1] = 1e30
    w3 = np.zeros(32); w3[0] = 1e30; w3[1] = -1e30
    theta = mlp_ref.pack(W1, np.zeros(32), W2, np.zeros(32), w3, 0.0).astype(np.float32)
    assert np.all(np.isfinite(theta))
    model = P.Model.create(theta, [0, 0, 0], [1, 1, 1])
    A = synth.zipf_matrix(30000, 8) if case == "zipf" else synth.stencil(64)
    want = oracle.spgemm(A, A)
    for tuning in (None, {"spill_ratio": -1}):
        got = gpu_product(A, A, "learned", model=model, tuning=tuning)
        assert_bit_exact(got, want)
        assert got[3]["overflow_rows"] == 0


@pytest.mark.parametrize("tuning", [None, {"merge_max_nnz": -1}])
def test_short_capacities_spill_into_the_arena(tuning):
    # capacities of the longest selected B row for rows of several times
    # that: the rows a tile has no room for take places in the spill arena
    # (at least 4096 entries, more than this whole product), merge rows are
    # merged again into it, and no row is computed a second time
    import paper_1303_1651_amd as P
    theta = np.zeros(1217, np.float32)
    theta[-1] = -30.0
    model = P.Model.create(theta, [0, 0, 0], [1, 1, 1])
    A = synth.random_uniform_lengths(60, 2, 20, 17)
    assert np.diff(A.row_ptr).max() > 16      # not the merge-only path
    want = oracle.spgemm(A, A)
    assert want[0][-1] < 4096
    got = gpu_product(A, A, "learned", model=model, tuning=tuning)
    assert_bit_exact(got, want)
    assert got[3]["overflow_rows"] == 0
    assert got[3]["spilled_rows"] > 0
    if tuning is None:
        assert got[3]["rows_merge"] > 0


def test_trained_network_gains_over_the_bound():
    # what the network buys: on wide stencils the multiplication count
    # overestimates nnz(C_i) several times; the learned capacities stay close
    # to it, so C is allocated and staged at about its real size, while the
    # product stays exact
    import paper_1303_1651_amd as P
    import torch
    train = [synth.stencil(40, 2, 9), synth.stencil(10, 3, 27), synth.stencil(48), synth.zipf_matrix(1 << 14, 70)]
    fs, ls = [], []
    for M in train:
        f1, f2, f3, n = _features_labels(M, M)
        fs.append(np.stack([f1, f2, f3]))
        ls.append(n)
    F = np.concatenate(fs, axis=1)
    L = np.concatenate(ls)
    perm = np.random.default_rng(1).permutation(F.shape[1])
    d1, d2, d3, dn = _to_dev(F[0][perm], F[1][perm], F[2][perm], L[perm])
    mu, sd = P.feature_stats(d1, d2, d3)
    model, _ = P.train_model(synth.mlp_init(12), mu, sd, d1, d2, d3, dn, epochs=40, batch_size=2048, lr=3e-3)
    for A in (synth.stencil(64, 2, 9), synth.stencil(14, 3, 27)):
        want = oracle.spgemm(A, A)
        nnz = int(want[0][-1])
        dA = P.DeviceCSR.from_host(A)
        ub_plan = P.Plan(dA, dA, "upper_bound")
        lr_plan = P.Plan(dA, dA, "learned", model)
        ub_cap, lr_cap = ub_plan.info["c_capacity_hint"], lr_plan.info["c_capacity_hint"]
        ub_plan.close()
        lr_plan.close()
        assert ub_cap >= 2.5 * nnz
        assert 0.9 * nnz <= lr_cap <= 1.3 * nnz, (lr_cap, nnz)
        got = gpu_product(A, A, "learned", model=model)
        assert_bit_exact(got, want)
        assert got[3]["overflow_rows"] <= 0.05 * A.rows
