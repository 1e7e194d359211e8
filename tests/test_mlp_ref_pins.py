"""Pins of the FP64 network reference (CPU): gradients against central
finite differences of its own loss, a hand-computed forward pass, and the
closed form of the first Adam step."""
import numpy as np

from oracle import mlp_ref as R


def _params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, R.NPARAM)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    flat = _params(2)
    X = rng.normal(size=(7, R.IN))
    Y = rng.normal(size=7)
    _, g = R.loss_and_grad(flat, X, Y)
    idx = rng.choice(R.NPARAM, size=60, replace=False)
    idx = np.concatenate([idx, [0, R.NPARAM - 1, R.IN * R.H + 3]])   # a W1, b3 and a b1 entry
    h = 1e-6
    for i in idx:
        e = np.zeros(R.NPARAM)
        e[i] = h
        fd = (R.loss_and_grad(flat + e, X, Y)[0] - R.loss_and_grad(flat - e, X, Y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_by_hand_on_a_tiny_net():
    parts = {n: np.zeros(s) for n, s in R.SIZES}
    parts["W1"][0, 0], parts["W1"][1, 1], parts["b1"][1] = 2.0, -1.0, 0.5
    parts["W2"][0, 0], parts["W2"][1, 0], parts["W2"][1, 1] = 1.0, 3.0, -4.0
    parts["W3"][0], parts["W3"][1], parts["b3"][0] = 0.5, 1.0, 0.25
    x = np.zeros((1, R.IN))
    x[0, 0], x[0, 1] = 1.5, 0.2
    # h1 = relu([3, 0.3]); h2 = relu([3 + 0.9, -1.2]) = [3.9, 0]; y = 1.95 + 0.25
    out, _ = R.forward(R.pack(parts), x)
    assert abs(out[0] - 2.2) <= 1e-12


def test_first_adam_step_is_signed_learning_rate():
    rng = np.random.default_rng(3)
    flat, g = rng.normal(size=R.NPARAM), rng.normal(size=R.NPARAM)
    new, m, v = R.adam(flat, g, np.zeros_like(g), np.zeros_like(g), 1, 0.01)
    # bias-corrected moments equal g and g^2 after one step
    np.testing.assert_allclose(new, flat - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)


def _constant_gradient_run(adam, steps, lr=0.01, seed=4):
    rng = np.random.default_rng(seed)
    flat, g = rng.normal(size=R.NPARAM), rng.normal(size=R.NPARAM)
    m, v = np.zeros_like(g), np.zeros_like(g)
    cur = flat.copy()
    for t in range(1, steps + 1):
        cur, m, v = adam(cur, g, m, v, t, lr)
    return flat, g, cur


def test_adam_constant_gradient_moves_by_signed_learning_rate_every_step():
    # With the same gradient g at every step the moments are m_t = (1-b1^t) g
    # and v_t = (1-b2^t) g^2, so the bias-corrected moments are exactly g and
    # g^2 at every step and each step moves every parameter by -lr g/(|g|+eps).
    for steps in (2, 3, 7, 25):
        flat, g, cur = _constant_gradient_run(R.adam, steps)
        np.testing.assert_allclose(cur, flat - steps * 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_adam_pin_catches_wrong_bias_correction():
    # plausible mistakes in the bias correction pass the first-step pin but
    # not the constant-gradient pin above
    def no_step_exponent(flat, grad, m, v, step, lr):
        b1, b2, eps = 0.9, 0.999, 1e-8
        m = b1 * m + (1 - b1) * grad
        v = b2 * v + (1 - b2) * grad * grad
        return flat - lr * (m / (1 - b1)) / (np.sqrt(v / (1 - b2)) + eps), m, v

    def swapped_betas(flat, grad, m, v, step, lr):
        b1, b2, eps = 0.9, 0.999, 1e-8
        m = b1 * m + (1 - b1) * grad
        v = b2 * v + (1 - b2) * grad * grad
        return flat - lr * (m / (1 - b2 ** step)) / (np.sqrt(v / (1 - b1 ** step)) + eps), m, v

    for bad in (no_step_exponent, swapped_betas):
        flat, g, cur = _constant_gradient_run(bad, 3)
        assert np.max(np.abs(cur - (flat - 3 * 0.01 * g / (np.abs(g) + 1e-8)))) > 1e-4
