"""Pins of the FP64 network reference: central finite differences of the loss,
and one Adam step against its definition worked by hand."""
import numpy as np
import pytest

from oracle import mlp


def _params(sizes, seed):
    rng = np.random.default_rng(seed)
    ps = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        ps.append(rng.uniform(-1, 1, (fo, fi)) / np.sqrt(fi))
        ps.append(rng.uniform(-0.1, 0.1, fo))
    return ps


def test_gradients_match_finite_differences():
    sizes = [7, 9, 8, 5]
    ps = _params(sizes, 0)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((6, 7))
    y = rng.standard_normal((6, 5))
    loss, grads = mlp.loss_and_grads(ps, x, y)
    h = 1e-6
    for k, p in enumerate(ps):
        flat = p.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 13)):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss_and_grads(ps, x, y)[0]
            flat[idx] = old - h
            lm = mlp.loss_and_grads(ps, x, y)[0]
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            g = grads[k].reshape(-1)[idx]
            assert g == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_single_adam_step_by_hand():
    # From zero moments, step 1: mhat = g, vhat = g^2, so the update is lr*g/(|g|+eps).
    p = [np.array([[1.0, -2.0]]), np.array([0.5])]
    g = [np.array([[0.25, -4.0]]), np.array([0.0])]
    m = [np.zeros_like(x) for x in p]
    v = [np.zeros_like(x) for x in p]
    out, m, v = mlp.adam_step(p, g, m, v, 1, lr=0.1)
    np.testing.assert_allclose(out[0], [[1.0 - 0.1 * 0.25 / (0.25 + 1e-8),
                                         -2.0 + 0.1 * 4.0 / (4.0 + 1e-8)]], rtol=1e-15)
    np.testing.assert_allclose(out[1], [0.5])
    np.testing.assert_allclose(m[0], 0.1 * np.array([[0.25, -4.0]]))
    np.testing.assert_allclose(v[0], 0.001 * np.array([[0.0625, 16.0]]))


def test_training_reduces_loss():
    sizes = [4, 16, 16, 3]
    ps = _params(sizes, 2)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((64, 4))
    y = np.tanh(x[:, :3]) + 0.1 * x[:, 1:4]
    _, hist = mlp.train(ps, x, y, 200, lr=1e-2)
    assert hist[-1] < 0.2 * hist[0]


def test_train_linear_model_reaches_least_squares():
    """A network with no hidden layer is a linear model, so full-batch Adam on
    its MSE converges to the least-squares solution (numpy lstsq on [x, 1])."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((40, 3))
    y = x @ np.array([[0.5, -1.0], [2.0, 0.3], [-0.7, 1.1]]) + np.array([0.2, -0.4]) \
        + 0.05 * rng.standard_normal((40, 2))
    ps = [np.zeros((2, 3)), np.zeros(2)]
    out, hist = mlp.train(ps, x, y, 3000, lr=2e-2)
    coef, *_ = np.linalg.lstsq(np.hstack([x, np.ones((40, 1))]), y, rcond=None)
    np.testing.assert_allclose(out[0], coef[:3].T, atol=2e-4)
    np.testing.assert_allclose(out[1], coef[3], atol=2e-4)
    assert hist[-1] == pytest.approx(np.mean((np.hstack([x, np.ones((40, 1))]) @ coef - y) ** 2),
                                     rel=1e-5)


def test_two_adam_steps_by_hand():
    """Two steps on a scalar with gradients 2 then -1 (lr 0.1): the bias-
    corrected moments give updates -0.1 and then
    -0.1 (0.18 - 0.1)/0.19 / (sqrt((0.003996 + 0.000999)/0.001999) + 1e-8)."""
    p = [np.array([1.0])]
    m = [np.zeros(1)]
    v = [np.zeros(1)]
    p, m, v = mlp.adam_step(p, [np.array([2.0])], m, v, 1, lr=0.1)
    np.testing.assert_allclose(p[0], [1.0 - 0.1 * 2.0 / (2.0 + 1e-8)], rtol=1e-15)
    p, m, v = mlp.adam_step(p, [np.array([-1.0])], m, v, 2, lr=0.1)
    m2 = 0.9 * 0.2 + 0.1 * (-1.0)           # 0.08
    v2 = 0.999 * 0.004 + 0.001 * 1.0         # 0.004996
    mhat, vhat = m2 / (1 - 0.81), v2 / (1 - 0.998001)
    np.testing.assert_allclose(p[0], [1.0 - 0.1 * 2.0 / (2.0 + 1e-8) - 0.1 * mhat / (np.sqrt(vhat) + 1e-8)],
                               rtol=1e-14)


def test_minibatches_in_order():
    """batch = n / 2: two Adam steps per epoch on the two halves in order
    equal two explicit calls of adam_step with those halves' gradients."""
    sizes = [3, 5, 2]
    ps = _params(sizes, 5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((8, 3))
    y = rng.standard_normal((8, 2))
    out, _ = mlp.train(ps, x, y, 1, lr=1e-2, batch=4)
    q = [p.copy() for p in ps]
    m = [np.zeros_like(p) for p in q]
    v = [np.zeros_like(p) for p in q]
    for step, sl in enumerate((slice(0, 4), slice(4, 8)), start=1):
        _, g = mlp.loss_and_grads(q, x[sl], y[sl])
        q, m, v = mlp.adam_step(q, g, m, v, step, lr=1e-2)
    for a, b in zip(out, q):
        np.testing.assert_allclose(a, b, rtol=1e-14, atol=0)
