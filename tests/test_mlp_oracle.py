"""Pins for the FP64 reference of the learned row-size network."""
import math

import numpy as np
import pytest

from oracle import mlp_ref
import synth


def _rand_theta(seed, scale=0.5):
    return scale * synth.uniform_pm1(synth.splitmix64(seed, np.arange(mlp_ref.NPARAM, dtype=np.uint64)))


def _batch(seed, n=37):
    X = synth.uniform_pm1(synth.splitmix64(seed, np.arange(3 * n, dtype=np.uint64))).reshape(n, 3) * 2.0
    t = 0.5 + 0.5 * synth.uniform_pm1(synth.splitmix64(seed + 1, np.arange(n, dtype=np.uint64)))
    w = (np.arange(n) % 5 != 0).astype(np.float64)
    return X, t, w


def test_parameter_count():
    assert mlp_ref.NPARAM == 32 * 3 + 32 + 32 * 32 + 32 + 32 + 1 == 1217


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradient_matches_central_differences(seed):
    theta = _rand_theta(seed)
    X, t, w = _batch(seed + 100)
    _, g = mlp_ref.loss_and_grad(theta, X, t, w)
    h = 1e-6
    idx = np.arange(0, mlp_ref.NPARAM, 7)
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp_ref.loss(tp, X, t, w) - mlp_ref.loss(tm, X, t, w)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_zero_weights_give_logistic_of_output_bias():
    theta = np.zeros(mlp_ref.NPARAM)
    theta[-1] = 0.7
    X, _, _ = _batch(5)
    rho, _ = mlp_ref.forward(theta, X)
    np.testing.assert_allclose(rho, 1.0 / (1.0 + math.exp(-0.7)), rtol=0, atol=1e-15)


def test_one_hidden_path_by_hand():
    # only W1[0,1] = 2, b1[0] = 0.5, W2[3,0] = 1.5, w3[3] = -1, b3 = 0.25 are set
    W1 = np.zeros((32, 3)); W1[0, 1] = 2.0
    b1 = np.zeros(32); b1[0] = 0.5
    W2 = np.zeros((32, 32)); W2[3, 0] = 1.5
    b2 = np.zeros(32)
    w3 = np.zeros(32); w3[3] = -1.0
    theta = mlp_ref.pack(W1, b1, W2, b2, w3, 0.25)
    X = np.array([[9.0, 0.75, -4.0], [0.0, -1.0, 0.0]])
    rho, _ = mlp_ref.forward(theta, X)
    # x1 = 0.75: h1_0 = relu(1.5 + 0.5) = 2, h2_3 = 3, z = -3 + 0.25
    # x1 = -1:   h1_0 = relu(-2 + 0.5) = 0, h2_3 = 0, z = 0.25
    np.testing.assert_allclose(rho, [1 / (1 + math.exp(2.75)), 1 / (1 + math.exp(-0.25))], rtol=1e-15)


def test_adam_first_step_is_signed_learning_rate():
    theta = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 0.0])
    th, m, v = mlp_ref.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0 + 1e-30)
    # step 1: mhat = g, vhat = g^2, update = lr * g / |g|
    np.testing.assert_allclose(th, [0.99, -1.99, 3.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_targets_and_weights():
    t, w = mlp_ref.targets(n=[5, 7, 3, 0], f2=[10, 7, 3, 0], f3=[4, 3, 3, 0])
    np.testing.assert_allclose(t, [1 / 6, 1.0, 0.0, 0.0])
    np.testing.assert_array_equal(w, [1, 1, 0, 0])


def test_inputs_by_hand():
    # x = (log2(1 + f) - mu) / sd, feature by feature:
    # f = (1, 3, 7): log2 = (1, 2, 3); mu = (0, 1, 1), sd = (1, 0.5, 4)
    # -> x = (1, 2, 0.5); f = (0, 15, 0): log2 = (0, 4, 0) -> (0, 6, -0.25)
    X = mlp_ref.inputs([1, 0], [3, 15], [7, 0], mu=[0.0, 1.0, 1.0], sd=[1.0, 0.5, 4.0])
    np.testing.assert_array_equal(X, [[1.0, 2.0, 0.5], [0.0, 6.0, -0.25]])


def test_prediction_maps_rho_onto_the_interval_from_the_longest_row():
    # zero weights and b3 = ln 3: rho = 1 / (1 + 1/3) = 3/4 for every row,
    # so the prediction is maxB + 3/4 (UB - maxB): (f3, f2) = (4, 12) -> 10,
    # (2, 2) -> 2, (0, 8) -> 6
    theta = np.zeros(mlp_ref.NPARAM)
    theta[-1] = math.log(3.0)
    p = mlp_ref.predict(theta, [0, 0, 0], [1, 1, 1], [3, 1, 4], [12, 2, 8], [4, 2, 0])
    np.testing.assert_allclose(p, [10.0, 2.0, 6.0], rtol=1e-15)


def test_prediction_through_the_standardised_input_by_hand():
    # W1[0, 0] = 1, W2[0, 0] = 1, w3[0] = 1, everything else 0: z = relu(x0).
    # f1 = 1 gives log2(2) = 1; mu0 = 0, sd0 = 1 / ln 3 -> x0 = ln 3,
    # rho = 3/4, prediction = 4 + 0.75 * 8 = 10.  f1 = 0 gives x0 = 0 -> z = 0,
    # rho = 1/2, prediction = 8.  mu0 = 2 with f1 = 1 gives x0 < 0: ReLU -> 8.
    W1 = np.zeros((32, 3)); W1[0, 0] = 1.0
    W2 = np.zeros((32, 32)); W2[0, 0] = 1.0
    w3 = np.zeros(32); w3[0] = 1.0
    theta = mlp_ref.pack(W1, np.zeros(32), W2, np.zeros(32), w3, 0.0)
    sd = [1.0 / math.log(3.0), 1.0, 1.0]
    p = mlp_ref.predict(theta, [0, 0, 0], sd, [1, 0], [12, 12], [4, 4])
    np.testing.assert_allclose(p, [10.0, 8.0], rtol=1e-14)
    p = mlp_ref.predict(theta, [2, 0, 0], sd, [1], [12], [4])
    np.testing.assert_allclose(p, [8.0], rtol=1e-15)


def test_prediction_stays_inside_bounds():
    theta = _rand_theta(9, scale=3.0)
    f3 = np.array([1, 5, 16, 0])
    f2 = np.array([1, 25, 256, 0])
    f1 = np.array([1, 5, 16, 0])
    p = mlp_ref.predict(theta, [0, 0, 0], [1, 1, 1], f1, f2, f3)
    assert np.all(p >= f3) and np.all(p <= f2)


def test_gradient_descent_lowers_loss():
    theta = _rand_theta(11, 0.3)
    X, t, w = _batch(12, 200)
    L0 = mlp_ref.loss(theta, X, t, w)
    m = np.zeros_like(theta); v = np.zeros_like(theta)
    for s in range(1, 201):
        _, g = mlp_ref.loss_and_grad(theta, X, t, w)
        theta, m, v = mlp_ref.adam_step(theta, g, m, v, s, lr=1e-2)
    assert mlp_ref.loss(theta, X, t, w) < 0.5 * L0
