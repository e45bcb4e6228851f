"""Pins of the Adan oracle by closed forms of its recurrences."""
import numpy as np
import pytest

from oracle import adan


def run(theta0, grads, lrs, **hp):
    th = np.array(theta0, dtype=np.float64)
    st = adan.init_state(th.shape)
    out = []
    for k, (g, lr) in enumerate(zip(grads, lrs)):
        th = adan.step(th, g, st, k, lr, **hp)
        out.append((th.copy(), {k2: v.copy() for k2, v in st.items()}))
    return out


def test_constant_gradient_moves_by_a_normalised_step():
    """g_k = g: m = g, v = 0, n = g^2 every step, so each step moves by
    lr_k g / sqrt(g^2 + eps); with lr_k = lr0 gamma^k the total is a geometric sum."""
    g = np.array([0.3, -2.0, 1e-3])
    K, lr0, gamma = 50, 0.01, 0.99995
    lrs = [lr0 * gamma ** k for k in range(K)]
    out = run(np.zeros(3), [g] * K, lrs)
    th, st = out[-1]
    np.testing.assert_allclose(st["m"], g, rtol=1e-14)
    np.testing.assert_allclose(st["v"], 0.0, atol=1e-18)
    np.testing.assert_allclose(st["n"], g * g, rtol=1e-13)
    total = lr0 * (1 - gamma ** K) / (1 - gamma)
    np.testing.assert_allclose(th, -total * g / np.sqrt(g * g + 1e-8), rtol=1e-11)


def test_linear_gradient_sequence_closed_forms():
    """g_k = a + b k: v_k = b for k >= 1 (v_1 = g_1 - g_0, then a fixed point),
    m_k = a + b k - (1 - b1) b / b1 (1 - (1 - b1)^k)."""
    a, b = np.array([1.0, -0.5]), np.array([0.2, 0.05])
    K = 30
    out = run(np.zeros(2), [a + b * k for k in range(K)], [0.01] * K)
    b1 = adan.DEFAULTS["b1"]
    for k in range(1, K):
        st = out[k][1]
        np.testing.assert_allclose(st["v"], b, rtol=1e-12)
        m_ref = a + b * k - (1 - b1) * b / b1 * (1 - (1 - b1) ** k)
        np.testing.assert_allclose(st["m"], m_ref, rtol=1e-11)


def test_zero_gradient_is_pure_weight_decay():
    th0 = np.array([1.0, -3.0])
    K, lr, wd = 20, 0.05, 0.1
    th = run(th0, [np.zeros(2)] * K, [lr] * K, weight_decay=wd)[-1][0]
    np.testing.assert_allclose(th, th0 * (1 + wd * lr) ** (-K), rtol=1e-13)


def test_first_step_uses_the_initialisation():
    g = np.array([0.5, -1.5])
    th = run(np.array([2.0, 2.0]), [g], [0.1])[0][0]
    # m0 = g0, v0 = 0, n0 = g0^2
    np.testing.assert_allclose(th, 2.0 - 0.1 * g / np.sqrt(g * g + 1e-8), rtol=1e-14)


def test_minimises_a_convex_quadratic():
    rng = np.random.default_rng(0)
    Q = rng.normal(size=(6, 6))
    A = Q @ Q.T + 0.5 * np.eye(6)
    x_star = rng.normal(size=6)
    th = np.zeros(6)
    st = adan.init_state(6)
    f0 = 0.5 * (th - x_star) @ A @ (th - x_star)
    for k in range(3000):
        g = A @ (th - x_star)
        th = adan.step(th, g, st, k, 0.01 * 0.999 ** k)
    f = 0.5 * (th - x_star) @ A @ (th - x_star)
    assert f < 1e-6 * f0
