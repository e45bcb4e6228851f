"""FP64 oracle for the camera-motion Neural ODE (paper Sec. 3.1 Eq. 1, Sec. 3.4).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

The camera extrinsics of frame f are read from the state z(t_f) of the ODE
dz/dt = f_theta(z, t) started at a learned z(0) (Eq. 1).  Readings of what the
paper leaves to its supplement:

* state z = (qw, qx, qy, qz, tx, ty, tz), world->camera; the pose of a frame
  is (q/|q|, t) of the state at that frame's time;
* frame times t_f = f/(F-1) in [0, 1] (the domain of the motion splines);
* f_theta(z, t) = W3 tanh(W2 tanh(W1 [z; t] + b1) + b2) + b3, an MLP
  8 -> 64 -> 64 -> 7;
* classic fourth-order Runge-Kutta with S sub-steps per frame interval,
  h = 1/(S (F-1));
* gradients are the discrete adjoint: the exact derivative of the computed
  RK4 trajectory (not the continuous adjoint ODE, which differs by O(h^4)).

Parameter vector theta (5191 values, fp32 in the product): W1 [64][8], b1 [64],
W2 [64][64], b2 [64], W3 [7][64], b3 [7], concatenated row-major.
"""
from __future__ import annotations

import numpy as np

STATE = 7
HIDDEN = 64
N_THETA = HIDDEN * (STATE + 1) + HIDDEN + HIDDEN * HIDDEN + HIDDEN + STATE * HIDDEN + STATE


def unpack(theta):
    th = np.asarray(theta, dtype=np.float64)
    assert th.shape == (N_THETA,), th.shape
    o = 0
    W1 = th[o:o + HIDDEN * 8].reshape(HIDDEN, 8); o += HIDDEN * 8
    b1 = th[o:o + HIDDEN]; o += HIDDEN
    W2 = th[o:o + HIDDEN * HIDDEN].reshape(HIDDEN, HIDDEN); o += HIDDEN * HIDDEN
    b2 = th[o:o + HIDDEN]; o += HIDDEN
    W3 = th[o:o + STATE * HIDDEN].reshape(STATE, HIDDEN); o += STATE * HIDDEN
    b3 = th[o:o + STATE]; o += STATE
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, np.ravel(W3), b3]).astype(np.float64)


class MLPField:
    """The vector field f_theta(z, t) of Eq. 1 and its vector-Jacobian product."""

    def __init__(self, theta):
        self.W1, self.b1, self.W2, self.b2, self.W3, self.b3 = unpack(theta)

    def __call__(self, z, t):
        x = np.concatenate([z, [t]])
        h1 = np.tanh(self.W1 @ x + self.b1)
        h2 = np.tanh(self.W2 @ h1 + self.b2)
        return self.W3 @ h2 + self.b3

    def vjp(self, z, t, dy):
        """Return (dL/dz, dL/dtheta) for upstream dL/df = dy."""
        x = np.concatenate([z, [t]])
        h1 = np.tanh(self.W1 @ x + self.b1)
        h2 = np.tanh(self.W2 @ h1 + self.b2)
        dW3 = np.outer(dy, h2)
        db3 = dy.copy()
        da2 = (self.W3.T @ dy) * (1.0 - h2 * h2)
        dW2 = np.outer(da2, h1)
        db2 = da2
        da1 = (self.W2.T @ da2) * (1.0 - h1 * h1)
        dW1 = np.outer(da1, x)
        db1 = da1
        dx = self.W1.T @ da1
        return dx[:STATE], pack(dW1, db1, dW2, db2, dW3, db3)


def rk4_step(field, z, t, h):
    """One classic RK4 step of dz/dt = field(z, t)."""
    k1 = field(z, t)
    k2 = field(z + 0.5 * h * k1, t + 0.5 * h)
    k3 = field(z + 0.5 * h * k2, t + 0.5 * h)
    k4 = field(z + h * k3, t + h)
    return z + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def integrate(field, z0, frames: int, substeps: int):
    """States at the frame times t_f = f/(F-1), f = 0..F-1: array [F][7]."""
    z = np.asarray(z0, dtype=np.float64).copy()
    out = np.empty((frames, z.shape[0]))
    out[0] = z
    if frames == 1:
        return out
    h = 1.0 / (substeps * (frames - 1))
    for f in range(1, frames):
        for s in range(substeps):
            t = ((f - 1) * substeps + s) * h
            z = rk4_step(field, z, t, h)
        out[f] = z
    return out


def states_to_poses(states):
    """Pose (q/|q|, t) of each state row."""
    states = np.asarray(states, dtype=np.float64)
    q = states[:, :4]
    return np.concatenate([q / np.linalg.norm(q, axis=1, keepdims=True), states[:, 4:]], axis=1)


def camera_ode_fwd(theta, z0, frames: int, substeps: int = 4):
    """Poses [F][7] of the camera ODE."""
    return states_to_poses(integrate(MLPField(theta), z0, frames, substeps))


def camera_ode_bwd(theta, z0, frames: int, substeps: int, dposes):
    """Discrete adjoint: (dL/dtheta, dL/dz0) given dL/dposes [F][7]."""
    field = MLPField(theta)
    dposes = np.asarray(dposes, dtype=np.float64)
    states = integrate(field, z0, frames, substeps)

    def pose_cotangent(z, dp):
        q = z[:4]
        nq = np.linalg.norm(q)
        qh = q / nq
        dq = (dp[:4] - qh * np.dot(qh, dp[:4])) / nq
        return np.concatenate([dq, dp[4:]])

    dtheta = np.zeros(N_THETA)
    lam = pose_cotangent(states[frames - 1], dposes[frames - 1])
    if frames > 1:
        h = 1.0 / (substeps * (frames - 1))
        for f in range(frames - 1, 0, -1):
            # recompute the sub-step states of interval [f-1, f]
            zs = [states[f - 1].copy()]
            for s in range(substeps):
                t = ((f - 1) * substeps + s) * h
                zs.append(rk4_step(field, zs[-1], t, h))
            for s in range(substeps - 1, -1, -1):
                t = ((f - 1) * substeps + s) * h
                z = zs[s]
                k1 = field(z, t)
                k2 = field(z + 0.5 * h * k1, t + 0.5 * h)
                k3 = field(z + 0.5 * h * k2, t + 0.5 * h)
                dz = lam.copy()
                dk1 = (h / 6.0) * lam
                dk2 = (h / 3.0) * lam
                dk3 = (h / 3.0) * lam
                dk4 = (h / 6.0) * lam
                gx, gth = field.vjp(z + h * k3, t + h, dk4)
                dz += gx; dk3 += h * gx; dtheta += gth
                gx, gth = field.vjp(z + 0.5 * h * k2, t + 0.5 * h, dk3)
                dz += gx; dk2 += 0.5 * h * gx; dtheta += gth
                gx, gth = field.vjp(z + 0.5 * h * k1, t + 0.5 * h, dk2)
                dz += gx; dk1 += 0.5 * h * gx; dtheta += gth
                gx, gth = field.vjp(z, t, dk1)
                dz += gx; dtheta += gth
                lam = dz
            lam = lam + pose_cotangent(states[f - 1], dposes[f - 1])
    return dtheta, lam
