"""Pins of the oracle's L2 loss (Sec. 4.1) and of its trajectory-error judge
of the learned camera (Sec. 3.4, Eq. 1: per-frame poses as the reference).

The loss is pinned by hand-computed values, a constant offset in closed form,
central finite differences of its gradient and the per-frame split.  The
trajectory error is pinned by scipy's rotation magnitude, rotations of known
angle (down to 1e-7 rad, where an arccos formula would lose every digit),
camera-centre offsets of known length, the sign and scale freedom of the
quaternion, and the frame averaging.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle


# ---------------------------------------------------------------- L2 loss


def test_l2_hand_computed():
    img = np.array([1.0, 2.0, 3.0, 4.0]).reshape(1, 1, 2, 2)
    tgt = np.zeros_like(img)
    loss, grad = oracle.l2_loss_and_grad(img, tgt)
    assert loss == 7.5  # (1 + 4 + 9 + 16) / 4
    np.testing.assert_array_equal(grad.ravel(), [0.5, 1.0, 1.5, 2.0])  # 2 d / 4


def test_l2_constant_offset_closed_form():
    rng = np.random.default_rng(0)
    tgt = rng.random((3, 3, 5, 7))
    c = -0.37
    loss, grad = oracle.l2_loss_and_grad(tgt + c, tgt)
    assert loss == pytest.approx(c * c, rel=1e-12)
    np.testing.assert_allclose(grad, 2 * c / tgt.size, rtol=1e-9)
    loss0, grad0 = oracle.l2_loss_and_grad(tgt, tgt)
    assert loss0 == 0.0 and not grad0.any()


def test_l2_gradient_finite_differences():
    rng = np.random.default_rng(1)
    img = rng.random((2, 3, 4, 5))
    tgt = rng.random((2, 3, 4, 5))
    _, grad = oracle.l2_loss_and_grad(img, tgt)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 2, 3, 4), (0, 1, 2, 3), (1, 0, 1, 0)]:
        a, b = img.copy(), img.copy()
        a[idx] += h
        b[idx] -= h
        fd = (oracle.l2_loss_and_grad(a, tgt)[0] - oracle.l2_loss_and_grad(b, tgt)[0]) / (2 * h)
        assert fd == pytest.approx(grad[idx], rel=1e-6)


def test_l2_per_frame_shares():
    rng = np.random.default_rng(2)
    img = rng.random((4, 3, 6, 5))
    tgt = rng.random((4, 3, 6, 5))
    loss, _ = oracle.l2_loss_and_grad(img, tgt)
    shares, _ = oracle.l2_loss_and_grad(img, tgt, per_frame=True)
    assert shares.shape == (4,)
    assert shares.sum() == pytest.approx(loss, rel=1e-12)
    # each share is that frame's own mean divided by the number of frames
    for f in range(4):
        own, _ = oracle.l2_loss_and_grad(img[f:f + 1], tgt[f:f + 1])
        assert shares[f] == pytest.approx(own / 4, rel=1e-12)
    with pytest.raises(ValueError):
        oracle.l2_loss_and_grad(img, tgt[:3])


# ---------------------------------------------------------- trajectory error


def pose_of(rot: Rotation, centre) -> np.ndarray:
    """World-to-camera 7-vector (w first) of a camera with orientation rot
    (world-to-camera rotation) and centre `centre`: t = -R c."""
    x, y, z, w = rot.as_quat()
    t = -rot.as_matrix() @ np.asarray(centre, float)
    return np.array([w, x, y, z, *t])


def test_identical_and_equivalent_quaternions():
    rng = np.random.default_rng(3)
    rots = Rotation.random(6, random_state=4)
    poses = np.stack([pose_of(r, rng.normal(0, 1, 3)) for r in rots])
    e = oracle.trajectory_error(poses, poses)
    assert e["translation_rmse"] == 0.0 and e["mean_angle"] == 0.0
    flipped = poses.copy()
    flipped[:, :4] *= -3.0   # -q and 3q describe the same rotation
    e = oracle.trajectory_error(flipped, poses)
    assert e["mean_angle"] < 1e-12 and e["translation_rmse"] < 1e-12


@pytest.mark.parametrize("angle", [1e-7, 0.3, 2.0, 3.1])
def test_rotation_of_known_angle(angle):
    rng = np.random.default_rng(5)
    axis = rng.normal(0, 1, 3)
    axis /= np.linalg.norm(axis)
    base = Rotation.random(random_state=6)
    centre = rng.normal(0, 1, 3)
    ref = pose_of(base, centre)
    # rotate the camera about its own centre: same centre, relative angle `angle`
    got = pose_of(Rotation.from_rotvec(angle * axis) * base, centre)
    e = oracle.trajectory_error(got[None], ref[None])
    assert e["mean_angle"] == pytest.approx(angle, rel=1e-7)
    assert e["translation_rmse"] < 1e-12


def test_against_scipy_magnitude():
    rng = np.random.default_rng(7)
    ra = Rotation.random(20, random_state=8)
    rb = Rotation.random(20, random_state=9)
    a = np.stack([pose_of(r, rng.normal(0, 1, 3)) for r in ra])
    b = np.stack([pose_of(r, rng.normal(0, 1, 3)) for r in rb])
    e = oracle.trajectory_error(a, b)
    expect = (ra * rb.inv()).magnitude()
    np.testing.assert_allclose(e["angle"], expect, rtol=1e-9, atol=1e-12)
    assert e["mean_angle"] == pytest.approx(expect.mean(), rel=1e-9)


def test_centre_offsets_and_frame_average():
    rng = np.random.default_rng(10)
    rots = Rotation.random(3, random_state=11)
    centres = rng.normal(0, 1, (3, 3))
    offsets = np.array([[0.3, 0.0, -0.4], [0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])  # lengths 0.5, 0, 3
    ref = np.stack([pose_of(r, c) for r, c in zip(rots, centres)])
    got = np.stack([pose_of(r, c + d) for r, c, d in zip(rots, centres, offsets)])
    e = oracle.trajectory_error(got, ref)
    np.testing.assert_allclose(e["translation"], [0.5, 0.0, 3.0], atol=1e-12)
    assert e["translation_rmse"] == pytest.approx(np.sqrt((0.25 + 0 + 9) / 3), rel=1e-12)
    assert e["mean_angle"] < 1e-12
    # two frames with different angles average arithmetically
    r0 = Rotation.random(random_state=12)
    ref2 = np.stack([pose_of(r0, [0, 0, 0])] * 2)
    got2 = np.stack([pose_of(Rotation.from_rotvec([0.2, 0, 0]) * r0, [0, 0, 0]),
                     pose_of(Rotation.from_rotvec([0, 0, 0.6]) * r0, [0, 0, 0])])
    assert oracle.trajectory_error(got2, ref2)["mean_angle"] == pytest.approx(0.4, rel=1e-12)
