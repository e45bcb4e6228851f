"""GPU parity of the fused Adan step (through the C ABI) against the FP64
Adan oracle, and of the intrinsics gradient against the FP64 renderer."""
import numpy as np
import pytest
import torch

import gv_synth
from oracle import adan as adan_ref
from parity_util import GRAD_TOL, rel_err
from test_gpu_parity import check_clip_against_oracle, small_workload

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2501_04782_amd.optim import Adan


def test_adan_matches_oracle_over_steps():
    rng = np.random.default_rng(70)
    shapes = [(3, 1000), (37,), (15, 3, 200)]
    theta = [rng.normal(0, 1, s) for s in shapes]
    params = [torch.from_numpy(t.astype(np.float32)).cuda() for t in theta]
    opt = Adan(params, lr=0.01, gamma=0.99, weight_decay=0.02)
    ref_theta = [t.astype(np.float32).astype(np.float64) for t in theta]
    ref_state = [adan_ref.init_state(s) for s in shapes]
    gmax = [0.0] * len(shapes)
    for k in range(8):
        grads = [rng.normal(0, 1, s) * (10.0 ** rng.uniform(-3, 1, s)) for s in shapes]
        gmax = [max(m, float(np.abs(g).max())) for m, g in zip(gmax, grads)]
        g32 = [g.astype(np.float32) for g in grads]
        opt.step([torch.from_numpy(g).cuda() for g in g32])
        lr = float(np.float32(0.01 * 0.99 ** k))
        for i in range(len(shapes)):
            ref_theta[i] = adan_ref.step(ref_theta[i], g32[i].astype(np.float64), ref_state[i], k, lr,
                                         weight_decay=float(np.float32(0.02)), b1=float(np.float32(0.02)),
                                         b2=float(np.float32(0.08)), b3=float(np.float32(0.01)),
                                         eps=float(np.float32(1e-8)))
    torch.cuda.synchronize()
    # FP32 bar: each recurrence rounds terms as large as the largest gradient
    # (squared for n) once per step, 2^-24 relative, over 8 steps; the
    # parameter moves by at most lr per step (|m + (1-b2) v| / sqrt(n) stays O(1))
    for i in range(len(shapes)):
        got = params[i].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, ref_theta[i], rtol=2e-6, atol=2e-6)
        st = opt.states[i].cpu().numpy().astype(np.float64)
        for j, name in enumerate(("m", "v", "n", "g_prev")):
            scale = gmax[i] ** 2 if name == "n" else gmax[i]
            np.testing.assert_allclose(st[j], ref_state[i][name], rtol=1e-5, atol=1e-6 * scale, err_msg=name)


def test_intrinsics_gradient_in_clip():
    """check_clip_against_oracle compares dL/d(fx, fy, cx, cy) too."""
    w = small_workload(71, 128, 96, 2500, 3, trajectory=True, z=(2.0, 8.0), ls=(-3.2, 0.5), bg=(0.2, 0.3, 0.1))
    out = check_clip_against_oracle(w, "intrinsics gradient")
    assert torch.all(torch.isfinite(out["grads"]["intrinsics"]))
    assert float(out["grads"]["intrinsics"].abs().sum()) > 0
