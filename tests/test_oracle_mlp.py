"""Pins of the learned-preconditioner oracle (CPU only).

Each check compares oracle.mlp with something other than itself: closed
forms of the network on special parameters, central finite differences of
the loss, the closed form of the first Adam step and hand-evaluated features
and targets.
"""

import numpy as np
import pytest

from oracle import mlp as om

F, H = om.N_FEATURES, om.HIDDEN


def _params(seed, scale=0.3):
    return np.random.default_rng(seed).standard_normal(om.n_params()) * scale


def test_parameter_count():
    assert om.n_params() == 64 * 12 + 64 + 64 * 64 + 64 + 64 + 1 == 5057


def test_forward_zero_second_layer_is_constant():
    p = _params(1)
    W1, b1, W2, b2, w3, b3 = om.unpack(p)
    W2[:] = 0.0
    X = np.random.default_rng(2).standard_normal((7, F))
    g, _ = om.forward(p, X)
    expect = float(np.tanh(b2) @ w3 + b3)
    assert np.allclose(g, expect, rtol=0, atol=1e-14)


def test_forward_single_active_unit():
    p = np.zeros(om.n_params())
    W1, b1, W2, b2, w3, b3 = om.unpack(p)
    a = np.linspace(-0.5, 0.6, F)
    W1[0] = a
    W2[0, 0] = 1.7
    w3[0] = -0.8
    p[-1] = 0.25
    X = np.random.default_rng(3).standard_normal((5, F))
    g, _ = om.forward(p, X)
    expect = -0.8 * np.tanh(1.7 * np.tanh(X @ a)) + 0.25
    assert np.allclose(g, expect, rtol=0, atol=1e-14)


def test_gradient_matches_central_differences():
    p = _params(4)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((9, F))
    y = rng.standard_normal(9)
    loss, grad = om.loss_and_grad(p, X, y)
    g0, _ = om.forward(p, X)
    assert abs(loss - np.mean((g0 - y) ** 2)) < 1e-15
    h = 1e-6
    idx = rng.choice(om.n_params(), 60, replace=False)
    idx = np.concatenate([idx, [0, 64 * F, 64 * F + 64, om.n_params() - 65, om.n_params() - 1]])
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (om.loss_and_grad(pp, X, y)[0] - om.loss_and_grad(pm, X, y)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_first_adam_step_closed_form():
    p = _params(6)
    g = np.random.default_rng(7).standard_normal(om.n_params())
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    p1, m1, v1 = om.adam_step(p, m, v, 1, g, lr=1e-3)
    # m_hat = g and v_hat = g^2 at step 1
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_features_by_hand():
    theta = -2.0
    diag = np.array([-1.0, -2.0 + 1e-14, 3.0])
    r = np.array([0.3, -0.4, 0.0])
    u = np.array([0.6, 0.0, 0.8])
    static = np.arange(24, dtype=float).reshape(3, 8)
    X = om.features(theta, diag, r, u, static)
    s3 = np.sqrt(3.0)
    assert np.allclose(X[:, 0], [-1.0 / 2, -1e-14 / 2, -5.0 / 2])
    assert np.allclose(X[:, 1], [0.0, np.log(1e-12) / 10, np.log(5.0) / 10])
    assert np.allclose(X[:, 2], [0.6 * s3, -0.8 * s3, 0.0])
    assert np.allclose(X[:, 3], [0.6 * s3, 0.0, 0.8 * s3])
    assert np.array_equal(X[:, 4:], static)
    st = om.static_features([2, 4], [0, -2], [1, 2], [0, 1], [1, 0], [0, -1], [0, 7], 3, 8, 8)
    assert np.allclose(st, [[0.25, 0.0, 0.5, 0.0, 1.0, 0.0, 0.0, 3.5 / 8],
                            [0.5, -0.25, 1.0, 0.5, 0.0, -1.0, np.log(8.0) / 8, 3.5 / 8]])


def test_correction_reduces_to_diagonal_at_zero_output():
    theta = 1.5
    diag = np.array([0.5, 1.5, 4.0])
    r = np.array([1.0, 2.0, -3.0])
    t = om.correction(theta, diag, r, np.zeros(3))
    assert np.allclose(t, [1.0, 2.0 / 1e-12, -3.0 / -2.5])
    t = om.correction(theta, diag, r, np.array([10.0, -10.0, np.log(2.0)]))
    assert np.allclose(t, [np.exp(3.0), 2e12 * np.exp(-3.0), 2.4])


def test_targets_by_hand():
    rng = np.random.default_rng(8)
    dr = rng.standard_normal(50)
    u = rng.standard_normal(50)
    # psi - c u proportional to dr: every ratio is the same positive number
    c = 0.3
    psi = 2.5 * dr + c * u
    out = om.targets(psi, u, c, dr)
    assert np.allclose(out, 0.0, atol=1e-12)
    # a second scale of psi changes nothing (alpha absorbs it)
    assert np.allclose(om.targets(7.0 * psi, u, 7.0 * c, dr), out, atol=1e-12)
    # two elements with doubled / opposite entries
    ts = dr.copy()
    ts[3] *= 2.0
    ts[4] *= -1.0
    alpha = (ts @ dr) / (ts @ ts)
    out = om.targets(ts + c * u, u, c, dr)
    with np.errstate(invalid="ignore"):
        expect = np.log(alpha * ts / dr)
    expect[4] = -3.0
    assert np.allclose(out[[0, 1, 2, 3, 5]], np.clip(expect[[0, 1, 2, 3, 5]], -3, 3), atol=1e-12)
    assert out[4] == -3.0
    dr2 = dr.copy()
    dr2[7] = 0.0
    assert om.targets(ts + c * u, u, c, dr2)[7] == 0.0


@pytest.mark.parametrize("lr", [1e-2, 1e-3])
def test_training_reduces_loss_on_a_learnable_map(lr):
    rng = np.random.default_rng(9)
    X = rng.standard_normal((256, F))
    y = np.tanh(X[:, 0] - 0.5 * X[:, 3])
    p = _params(10, 0.1)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = om.loss_and_grad(p, X, y)[0]
    for t in range(1, 201):
        loss, g = om.loss_and_grad(p, X, y)
        p, m, v = om.adam_step(p, m, v, t, g, lr)
    assert om.loss_and_grad(p, X, y)[0] < 0.3 * l0
