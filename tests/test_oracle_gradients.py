"""Pins of the oracle's hand-written adjoint.

(i) central finite differences of the oracle's own forward pass, and (ii)
torch float64 autograd through an independently formulated, vectorised
forward model (blending weights via a cumulative product instead of a loop).
Pixels whose discrete decisions sit within 1e-3 (relative) of a threshold get
zero upstream gradient, so no finite-difference step can flip a decision that
matters.
"""
import dataclasses

import numpy as np
import pytest
import torch

import gv_synth
import oracle


def make_case(seed, n=40, W=32, H=24, cubic=False, pose=None, t=0.0, bg=(0.1, 0.2, 0.3)):
    rng = np.random.default_rng(seed)
    cam = gv_synth.make_camera(W, H, float(W), bg=bg)
    mu = np.stack([rng.uniform(-0.8, 0.8, n), rng.uniform(-0.6, 0.6, n), rng.uniform(2, 5, n)])
    s = dict(means=mu, log_scales=rng.normal(-2.4, 0.4, (3, n)), quats=rng.normal(0, 1, (4, n)),
             opacity_logits=rng.normal(0.3, 1.0, n), colors=rng.uniform(0, 1, (3, n)),
             mean_coeffs=rng.normal(0, 0.1, (3, 3, n)) if cubic else None)
    if pose is None:
        pose = np.array([1.0, 0.03, -0.05, 0.02, 0.05, -0.03, 0.1])
    full = oracle.render_frame(s, cam, pose, t)
    dl = rng.normal(0, 1, (W * H, 3))
    stable = (full["margins"] > 1e-3).all(axis=1)
    dl[~stable] = 0.0
    return s, cam, np.asarray(pose, float), t, dl, stable


def loss(s, cam, pose, t, dl):
    r = oracle.render_frame(s, cam, pose, t)
    return float(np.sum(r["color"] * dl))


PARAMS = ["means", "log_scales", "quats", "opacity_logits", "colors"]


@pytest.mark.parametrize("cubic", [False, True])
def test_adjoint_matches_central_differences(cubic):
    s, cam, pose, t, dl, stable = make_case(21 + int(cubic), cubic=cubic, t=0.6 if cubic else 0.0)
    assert stable.mean() > 0.9
    g = oracle.render_frame(s, cam, pose, t, dL_dC=dl)["grads"]
    names = PARAMS + (["mean_coeffs"] if cubic else [])
    rng = np.random.default_rng(0)
    for name in names:
        a = s[name]
        flat = a.reshape(-1)
        idx = rng.choice(flat.size, min(flat.size, 40), replace=False)
        for i in idx:
            h = 1e-6 * max(1.0, abs(flat[i]))
            old = flat[i]
            flat[i] = old + h
            lp = loss(s, cam, pose, t, dl)
            flat[i] = old - h
            lm = loss(s, cam, pose, t, dl)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[i]
            assert an == pytest.approx(fd, rel=2e-5, abs=2e-7 * (1 + np.abs(g[name]).max())), (name, i)
    for k in range(7):
        pp, pm = pose.copy(), pose.copy()
        h = 1e-6
        pp[k] += h
        pm[k] -= h
        fd = (loss(s, cam, pp, t, dl) - loss(s, cam, pm, t, dl)) / (2 * h)
        assert g["pose"][k] == pytest.approx(fd, rel=2e-5, abs=1e-6), ("pose", k)
    for k, name in enumerate(("fx", "fy", "cx", "cy")):
        h = 1e-5 * max(1.0, abs(getattr(cam, name)))
        cp, cm = dataclasses.replace(cam), dataclasses.replace(cam)
        setattr(cp, name, getattr(cam, name) + h)
        setattr(cm, name, getattr(cam, name) - h)
        fd = (loss(s, cp, pose, t, dl) - loss(s, cm, pose, t, dl)) / (2 * h)
        assert g["intrinsics"][k] == pytest.approx(fd, rel=2e-5, abs=1e-7), ("intrinsics", name)


# ---------------------------------------------------------------------------
# independent vectorised forward model in torch float64
# ---------------------------------------------------------------------------

def _rot(q):
    w, x, y, z = q[0], q[1], q[2], q[3]
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]),
    ])


def torch_render(P, cam, t):
    """Image [H*W][3] of the forward model, vectorised over Gaussians."""
    mu = P["means"]
    if "mean_coeffs" in P:
        c = P["mean_coeffs"]
        mu = mu + c[0] * t + c[1] * t ** 2 + c[2] * t ** 3
    qh = P["quats"] / torch.linalg.norm(P["quats"], dim=0, keepdim=True)
    R = _rot(qh).permute(2, 0, 1)                                  # [N][3][3]
    M = R * torch.exp(P["log_scales"]).T[:, None, :]
    Sig = M @ M.transpose(1, 2)
    pq = P["pose"][:4] / torch.linalg.norm(P["pose"][:4])
    Rc = _rot(pq)
    m = Rc @ mu + P["pose"][4:, None]                               # [3][N]
    zinv = 1.0 / m[2]
    if "intrinsics" in P:
        fx, fy, cx, cy = P["intrinsics"][0], P["intrinsics"][1], P["intrinsics"][2], P["intrinsics"][3]
    else:
        fx, fy, cx, cy = cam.fx, cam.fy, cam.cx, cam.cy
    u = fx * m[0] * zinv + cx
    v = fy * m[1] * zinv + cy
    zero = torch.zeros_like(zinv)
    J = torch.stack([torch.stack([fx * zinv, zero, -fx * m[0] * zinv ** 2]),
                     torch.stack([zero, fy * zinv, -fy * m[1] * zinv ** 2])]).permute(2, 0, 1)
    Tm = J @ Rc
    cov = Tm @ Sig @ Tm.transpose(1, 2) + cam.dilation * torch.eye(2, dtype=torch.float64)
    inv = torch.linalg.inv(cov)
    o = torch.sigmoid(P["opacity_logits"])
    # order: fp32 depth key, then index
    key = m[2].detach().numpy().astype(np.float32)
    order = torch.as_tensor(np.lexsort((np.arange(key.size), key)))
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    px = torch.as_tensor(xs.reshape(-1) + 0.5)
    py = torch.as_tensor(ys.reshape(-1) + 0.5)
    dx = px[:, None] - u[order][None, :]
    dy = py[:, None] - v[order][None, :]
    A = inv[order]
    q = A[:, 0, 0] * dx * dx + (A[:, 0, 1] + A[:, 1, 0]) * dx * dy + A[:, 1, 1] * dy * dy
    alpha = torch.clamp(o[order] * torch.exp(-0.5 * q), max=0.99)
    alive = (q <= 9) & (alpha >= 1 / 255)
    a = torch.where(alive, alpha, torch.zeros_like(alpha))
    Tincl = torch.cumprod(1 - a, dim=1)                          # T after each entry
    Texcl = torch.cat([torch.ones_like(Tincl[:, :1]), Tincl[:, :-1]], dim=1)
    stop = alive & (Tincl < 1e-4)
    after = torch.cumsum(stop.to(torch.int64), dim=1) > 0        # the stopping entry and all later ones
    w = torch.where(after, torch.zeros_like(a), a * Texcl)
    Tfin = torch.where(after, torch.ones_like(a), 1 - a).prod(dim=1)
    col = P["colors"][:, order]
    bg = torch.tensor(cam.bg, dtype=torch.float64)
    return w @ col.T + Tfin[:, None] * bg[None, :]


@pytest.mark.parametrize("seed,cubic", [(31, False), (32, True), (33, False)])
def test_adjoint_matches_torch_autograd(seed, cubic):
    s, cam, pose, t, dl, stable = make_case(seed, n=60, cubic=cubic, t=0.35 if cubic else 0.0)
    g = oracle.render_frame(s, cam, pose, t, dL_dC=dl)["grads"]
    P = {k: torch.tensor(s[k], dtype=torch.float64, requires_grad=True) for k in PARAMS}
    if cubic:
        P["mean_coeffs"] = torch.tensor(s["mean_coeffs"], dtype=torch.float64, requires_grad=True)
    P["pose"] = torch.tensor(pose, dtype=torch.float64, requires_grad=True)
    P["intrinsics"] = torch.tensor([cam.fx, cam.fy, cam.cx, cam.cy], dtype=torch.float64, requires_grad=True)
    img = torch_render(P, cam, t)
    ref = oracle.render_frame(s, cam, pose, t)["color"]
    np.testing.assert_allclose(img.detach().numpy(), ref, atol=1e-12)
    (img * torch.as_tensor(dl)).sum().backward()
    for k, v in P.items():
        ref_g = v.grad.numpy()
        got = g[k]
        err = np.linalg.norm(got - ref_g) / max(np.linalg.norm(ref_g), 1e-30)
        assert err < 1e-9, (k, err)


def test_colour_gradient_is_exact_blend_weight():
    """dC/dc_g = alpha_g T_g: with unit upstream gradient on one channel and
    a single Gaussian, dL/dc equals the rendered alpha summed over pixels."""
    cam = gv_synth.make_camera(16, 16, 16.0)
    s = dict(means=np.array([[0.0], [0.0], [3.0]]), log_scales=np.full((3, 1), -1.5),
             quats=np.array([[1.0], [0], [0], [0]]), opacity_logits=np.array([0.4]),
             colors=np.array([[1.0], [1.0], [1.0]]), mean_coeffs=None)
    r = oracle.render_frame(s, cam, [1, 0, 0, 0, 0, 0, 0])
    dl = np.zeros((256, 3))
    dl[:, 1] = 1.0
    g = oracle.render_frame(s, cam, [1, 0, 0, 0, 0, 0, 0], dL_dC=dl)["grads"]
    # with white colour and black background, C = sum of blend weights = 1 - T_final
    assert g["colors"][1, 0] == pytest.approx(np.sum(1.0 - r["T_final"]), rel=1e-12)
    assert g["colors"][0, 0] == 0.0 and g["colors"][2, 0] == 0.0
