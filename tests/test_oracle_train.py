"""Pins of the oracle's training step: Adam, the activation chain and the
clone / split / prune refinement."""
import math

import numpy as np
import pytest

import oracle


def random_state(n, deg, seed):
    rng = np.random.default_rng(seed)
    R = oracle.train_rows(deg)
    raw = rng.normal(0, 1, (R, n))
    raw[3:6] = rng.uniform(-4, -1, (3, n))
    raw[10] = rng.uniform(-3, 3, n)
    return raw


def grads_of(rng, raw):
    n = raw.shape[1]
    return dict(mean=rng.normal(size=(3, n)), scale=rng.normal(size=(3, n)), quat=rng.normal(size=(4, n)),
                opacity=rng.normal(size=n), sh=rng.normal(size=(raw.shape[0] - 11, n)))


def test_activation_chain_by_finite_differences():
    """raw_gradients is d(sum g * act(raw)) / d raw for the activations
    s = exp(log s), sigma = sigmoid(logit) (central differences)."""
    rng = np.random.default_rng(1)
    raw = random_state(5, 1, 1)
    g = grads_of(rng, raw)

    def loss(r):
        s, o = oracle.activate(r)
        return (g["mean"] * r[0:3]).sum() + (g["scale"] * s).sum() + (g["quat"] * r[6:10]).sum() + \
            (g["opacity"] * o).sum() + (g["sh"] * r[11:]).sum()

    gr = oracle.raw_gradients(raw, g)
    h = 1e-6
    for idx in [(0, 2), (3, 1), (5, 4), (7, 0), (10, 3), (12, 2)]:
        e = np.zeros_like(raw)
        e[idx] = h
        fd = (loss(raw + e) - loss(raw - e)) / (2 * h)
        assert gr[idx] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_adam_constant_gradient_closed_form():
    """With a constant raw gradient g, m_hat = g and v_hat = g^2 at every
    step, so each step moves a parameter by lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    raw0 = random_state(7, 0, 2)
    g = grads_of(rng, raw0)
    # constant in raw space: gradients w.r.t. mean / quat / SH are raw ones;
    # keep the scale and opacity rows at zero so their chain is constant too
    g["scale"][:] = 0.0
    g["opacity"][:] = 0.0
    lr = (1e-3, 2e-3, 3e-3, 4e-3, 5e-3)
    raw, m, v = raw0, np.zeros_like(raw0), np.zeros_like(raw0)
    for t in range(1, 6):
        o = oracle.adam_step(raw, m, v, g, t, lr, eps=1e-12)
        raw, m, v = o["raw"], o["m"], o["v"]
    gr = oracle.raw_gradients(raw0, g)
    step = np.where(gr != 0, gr / (np.abs(gr) + 1e-12), 0.0)
    np.testing.assert_allclose(raw[0:3], raw0[0:3] - 5 * lr[0] * step[0:3], atol=1e-12)
    np.testing.assert_allclose(raw[6:10], raw0[6:10] - 5 * lr[2] * step[6:10], atol=1e-12)
    np.testing.assert_allclose(raw[11:], raw0[11:] - 5 * lr[4] * step[11:], atol=1e-12)
    np.testing.assert_allclose(raw[3:6], raw0[3:6], atol=0)


def test_densify_hand_cases():
    """Four Gaussians: low opacity (pruned), hot and small (cloned), hot and
    large (split into two), cold (kept)."""
    deg = 0
    R = oracle.train_rows(deg)
    raw = np.zeros((R, 4))
    raw[6] = 1.0  # identity rotation
    raw[3:6] = math.log(0.01)
    raw[3:6, 2] = [math.log(0.5), math.log(0.02), math.log(0.02)]
    raw[10] = [math.log(0.001 / 0.999), 2.0, 2.0, 2.0]
    raw[0:3, 2] = [1.0, 2.0, 3.0]
    accum = np.array([5.0, 5.0, 5.0, 1e-6])
    count = np.array([10.0, 10.0, 10.0, 10.0])
    noise = np.zeros((6, 4))
    noise[0:3, 2] = [1.0, 0.0, 0.0]
    noise[3:6, 2] = [0.0, -2.0, 0.0]
    m = np.ones((R, 4))
    out = oracle.densify(raw, m, m, accum, count, noise, grad_threshold=0.2, split_scale=0.1, min_opacity=0.005)
    assert list(out["kinds"]) == [0, 2, 3, 1]
    assert out["raw"].shape == (R, 5)
    np.testing.assert_array_equal(out["raw"][:, 0], raw[:, 1])
    np.testing.assert_array_equal(out["raw"][:, 1], raw[:, 1])
    assert (out["m"][:, 0] == 1).all() and (out["m"][:, 1] == 0).all()
    np.testing.assert_allclose(out["raw"][0:3, 2], [1.5, 2.0, 3.0], atol=1e-12)   # mean + 0.5 * 1 along x
    np.testing.assert_allclose(out["raw"][0:3, 3], [1.0, 1.96, 3.0], atol=1e-12)  # mean - 0.02 * 2 along y
    np.testing.assert_allclose(out["scale"][:, 2], np.array([0.5, 0.02, 0.02]) / 1.6, rtol=1e-12)
    np.testing.assert_array_equal(out["raw"][:, 4], raw[:, 3])
    assert (out["accum"] == 0).all() and (out["count"] == 0).all()
