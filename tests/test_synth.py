"""Seeded input generators: reproducibility, storage rounding, distributions."""
import numpy as np
import torch

import gv_synth


def test_same_seed_same_inputs():
    a = gv_synth.make_workload("frame128_n2k", seed=3)
    b = gv_synth.make_workload("frame128_n2k", seed=3)
    for k in a["scene"].fields():
        assert np.array_equal(getattr(a["scene"], k), getattr(b["scene"], k))
    assert np.array_equal(a["targets"], b["targets"])


def test_bf16_rounding_matches_torch_on_fp32_values():
    rng = np.random.default_rng(0)
    x = rng.normal(0, 3, 100_000).astype(np.float32)
    ours = gv_synth.round_bf16(x.astype(np.float64))
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)
    bits = gv_synth.f64_to_bf16_bits(ours)
    assert np.array_equal(gv_synth.bf16_bits_to_f64(bits), ours)


def test_workload_shapes_and_ranges():
    w = gv_synth.make_workload("clip540p_f50_n200k", targets=False, n=5000, frames=6)
    s = w["scene"]
    assert s.means.shape == (3, 5000) and s.quats.shape == (4, 5000)
    assert s.means[2].min() >= 2.0 and s.means[2].max() <= 10.0
    assert np.allclose(np.linalg.norm(s.quats.astype(np.float64), axis=0), 1.0, atol=1e-6)
    assert w["poses"].shape == (6, 7)
    assert np.allclose(np.linalg.norm(w["poses"][:, :4], axis=1), 1.0, atol=1e-6)
    assert np.abs(w["poses"][:, 4:]).max() <= 0.6 + 1e-6
    assert np.allclose(w["times"], np.arange(6) / 5)
    big = gv_synth.make_workload("clip1080p_f32_n500k_bf16", targets=False, n=1000, frames=4)
    assert big["scene"].dtype == "bf16" and big["scene"].means.dtype == np.uint16
    assert big["scene"].mean_coeffs.shape == (3, 3, 1000)
