"""FP64 oracle of the Adan optimizer step (the optimizer of Sec. 4.1).

TEST INFRASTRUCTURE ONLY: imported by tests, never by the product path.

The paper trains with Adan (learning rate 0.01 decayed by gamma = 0.99995 per
step) and gives no other setting.  This follows the Adan algorithm (Xie et
al., Adaptive Nesterov Momentum) in its own notation, with these readings:

* momentum coefficients weight the new term: m_k = (1 - b1) m_{k-1} + b1 g_k,
  likewise v (with the gradient difference g_k - g_{k-1}) and n (with the
  square of g_k + (1 - b2)(g_k - g_{k-1})); defaults b1 = 0.02, b2 = 0.08,
  b3 = 0.01 (the algorithm's recommended values), eps = 1e-8, weight decay 0;
* step 0 initialises m_0 = g_0, v_0 = 0, n_0 = g_0^2 and then updates theta;
  step 1 sets v_1 = g_1 - g_0 exactly (the algorithm's stated initialisation),
  every later step follows the recurrences;
* eta_k = lr_k / sqrt(n_k + eps) (eps inside the root, as the algorithm is
  written); theta_{k+1} = (theta_k - eta_k (m_k + (1 - b2) v_k)) / (1 + wd lr_k);
* the learning-rate schedule lr_k = lr_0 gamma^k is the caller's; a step takes
  lr_k as given.
"""
from __future__ import annotations

import numpy as np

DEFAULTS = dict(b1=0.02, b2=0.08, b3=0.01, eps=1e-8, weight_decay=0.0)


def init_state(shape) -> dict:
    return dict(m=np.zeros(shape), v=np.zeros(shape), n=np.zeros(shape), g_prev=np.zeros(shape))


def step(theta, g, state: dict, k: int, lr: float, b1=DEFAULTS["b1"], b2=DEFAULTS["b2"], b3=DEFAULTS["b3"],
         eps=DEFAULTS["eps"], weight_decay=DEFAULTS["weight_decay"]):
    """One Adan step at iteration k (0-based) on FP64 arrays; returns the new
    parameters and updates ``state`` in place."""
    theta = np.asarray(theta, np.float64)
    g = np.asarray(g, np.float64)
    m, v, n, gp = state["m"], state["v"], state["n"], state["g_prev"]
    if k == 0:
        m[...] = g
        v[...] = 0.0
        n[...] = g * g
    else:
        diff = g - gp
        m[...] = (1.0 - b1) * m + b1 * g
        if k == 1:
            v[...] = diff
        else:
            v[...] = (1.0 - b2) * v + b2 * diff
        w = g + (1.0 - b2) * diff
        n[...] = (1.0 - b3) * n + b3 * w * w
    gp[...] = g
    eta = lr / np.sqrt(n + eps)
    return (theta - eta * (m + (1.0 - b2) * v)) / (1.0 + weight_decay * lr)
