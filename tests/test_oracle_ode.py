"""Pins of the camera-ODE oracle (Eq. 1 with RK4, and its discrete adjoint).

RK4 on a linear field reproduces the 4th-order Taylor polynomial of exp(hM);
a constant field (zero first-layer weights) gives an exactly linear
trajectory; the global error falls as h^4; the adjoint matches central
differences and torch float64 autograd through an independently written RK4.
"""
import math

import numpy as np
import pytest
import torch

import gv_synth
from oracle import camera_ode as co


def test_rk4_step_on_linear_field_is_taylor_polynomial():
    rng = np.random.default_rng(0)
    M = rng.normal(0, 1, (7, 7))
    z = rng.normal(0, 1, 7)
    h = 0.07
    got = co.rk4_step(lambda y, t: M @ y, z, 0.3, h)
    P = np.eye(7)
    acc = np.eye(7)
    for k in range(1, 5):
        P = P @ (h * M) / k
        acc = acc + P
    np.testing.assert_allclose(got, acc @ z, rtol=1e-13, atol=1e-14)


def test_constant_field_gives_linear_trajectory():
    rng = np.random.default_rng(1)
    W1, b1, W2, b2, W3, b3 = co.unpack(gv_synth.init_mlp_theta(rng))
    W1 = np.zeros_like(W1)
    W2 = np.zeros_like(W2)  # f = W3 tanh(b2) + b3, independent of z and t
    theta = co.pack(W1, b1, W2, b2, W3, b3)
    const = W3 @ np.tanh(b2) + b3
    z0 = np.array([1.0, 0.1, -0.2, 0.05, 0.3, -0.1, 0.2])
    F = 9
    states = co.integrate(co.MLPField(theta), z0, F, 4)
    for f in range(F):
        np.testing.assert_allclose(states[f], z0 + const * f / (F - 1), rtol=1e-13, atol=1e-14)
    poses = co.camera_ode_fwd(theta, z0, F, 4)
    np.testing.assert_allclose(np.linalg.norm(poses[:, :4], axis=1), 1.0, rtol=1e-14)


def test_fourth_order_convergence():
    rng = np.random.default_rng(2)
    theta = gv_synth.init_mlp_theta(rng, last_layer_scale=3.0)
    z0 = rng.normal(0, 1, 7)
    ref = co.integrate(co.MLPField(theta), z0, 2, 512)[-1]
    errs = [np.linalg.norm(co.integrate(co.MLPField(theta), z0, 2, s)[-1] - ref) for s in (4, 8, 16)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


def test_adjoint_matches_central_differences():
    rng = np.random.default_rng(3)
    theta = gv_synth.init_mlp_theta(rng, last_layer_scale=1.0)
    z0 = np.array([0.95, 0.1, -0.2, 0.05, 0.3, -0.1, 0.2])
    F, S = 5, 2
    dp = rng.normal(0, 1, (F, 7))
    dth, dz0 = co.camera_ode_bwd(theta, z0, F, S, dp)

    def L(th, z):
        return float(np.sum(co.camera_ode_fwd(th, z, F, S) * dp))

    for i in rng.choice(co.N_THETA, 60, replace=False):
        e = np.zeros(co.N_THETA)
        e[i] = 1e-6
        fd = (L(theta + e, z0) - L(theta - e, z0)) / 2e-6
        assert dth[i] == pytest.approx(fd, rel=1e-5, abs=1e-8), i
    for i in range(7):
        e = np.zeros(7)
        e[i] = 1e-6
        fd = (L(theta, z0 + e) - L(theta, z0 - e)) / 2e-6
        assert dz0[i] == pytest.approx(fd, rel=1e-5, abs=1e-8), i


def test_adjoint_matches_torch_autograd():
    rng = np.random.default_rng(4)
    theta = gv_synth.init_mlp_theta(rng, last_layer_scale=0.5)
    z0 = np.array([0.9, -0.1, 0.3, 0.1, -0.2, 0.1, 0.4])
    F, S = 7, 4
    dp = rng.normal(0, 1, (F, 7))
    dth, dz0 = co.camera_ode_bwd(theta, z0, F, S, dp)

    th = torch.tensor(theta, requires_grad=True)
    z = torch.tensor(z0, requires_grad=True)
    W1 = th[:512].reshape(64, 8); b1 = th[512:576]
    W2 = th[576:4672].reshape(64, 64); b2 = th[4672:4736]
    W3 = th[4736:5184].reshape(7, 64); b3 = th[5184:5191]

    def f(y, t):
        x = torch.cat([y, torch.tensor([t], dtype=torch.float64)])
        return W3 @ torch.tanh(W2 @ torch.tanh(W1 @ x + b1) + b2) + b3

    h = 1.0 / (S * (F - 1))
    y = z
    poses = [torch.cat([y[:4] / torch.linalg.norm(y[:4]), y[4:]])]
    for step in range((F - 1) * S):
        t = step * h
        k1 = f(y, t)
        k2 = f(y + h / 2 * k1, t + h / 2)
        k3 = f(y + h / 2 * k2, t + h / 2)
        k4 = f(y + h * k3, t + h)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        if (step + 1) % S == 0:
            poses.append(torch.cat([y[:4] / torch.linalg.norm(y[:4]), y[4:]]))
    P = torch.stack(poses)
    np.testing.assert_allclose(P.detach().numpy(), co.camera_ode_fwd(theta, z0, F, S), rtol=1e-13, atol=1e-14)
    (P * torch.as_tensor(dp)).sum().backward()
    np.testing.assert_allclose(dth, th.grad.numpy(), rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(dz0, z.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_parameter_count():
    assert co.N_THETA == 5191
