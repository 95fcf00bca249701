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
