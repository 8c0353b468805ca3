"""Pins for the FP64 surrogate-network reference (CPU only)."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_special_cases():
    ulp = 2.0 ** -7  # bfloat16 spacing at 1
    cases = {
        1.0: 1.0,
        1.0 + ulp / 2: 1.0,                     # tie -> even (1.0)
        1.0 + 1.5 * ulp: 1.0 + 2 * ulp,          # tie -> even
        1.0 + ulp / 2 + 2.0 ** -20: 1.0 + ulp,   # just above the tie
        -(1.0 + ulp / 2 + 2.0 ** -20): -(1.0 + ulp),
        3.0e-3: 3.0e-3,
    }
    for x, want in cases.items():
        got = mlp.round_bf16(np.array([x]))[0]
        if x == 3.0e-3:
            assert abs(got - x) <= 2.0 ** -8 * abs(x) and got != x  # half of the 2^-7 relative spacing
        else:
            assert got == want, (x, got, want)
    # every bf16 value is a fixed point
    vals = np.array([0.5, 0.75, 1.0078125, -2.0, 65280.0])
    assert np.array_equal(mlp.round_bf16(vals), vals)


def test_linear_layer_closed_form():
    rng = np.random.default_rng(0)
    W = rng.normal(size=(4, 3))
    b = rng.normal(size=4)
    x = rng.normal(size=(5, 3))
    y, _ = mlp.forward(np.concatenate([W.reshape(-1), b]), [3, 4], x, bf16=False)
    assert np.allclose(y, x @ W.T + b, rtol=0, atol=1e-13)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    widths = [3, 16, 12, 5]
    p = mlp.init_params(widths, rng) + rng.normal(scale=0.1, size=sum(
        widths[l] * widths[l + 1] + widths[l + 1] for l in range(3)))
    x = rng.normal(size=(7, 3))
    t = rng.normal(size=(7, 5))
    w = rng.uniform(0.2, 1.0, size=(7, 5))
    _, g = mlp.loss_grad(p, widths, x, t, w, bf16=False)
    idx = rng.choice(p.size, size=40, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss_grad(p + e, widths, x, t, w, bf16=False)[0]
              - mlp.loss_grad(p - e, widths, x, t, w, bf16=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_closed_form():
    # first step: m_hat = g, v_hat = g^2, so p moves by lr g / (|g| + eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = mlp.adam(p, g, np.zeros(3), np.zeros(3), 1, 0.01, 0.9, 0.999, 1e-8)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
