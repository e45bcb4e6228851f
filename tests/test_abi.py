"""C-ABI library: loads, exports every entry point of include/gv.h, and the
host-only calls validate their arguments (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2501_04782_amd import _lib as L
from paper_2501_04782_amd.raster import Camera

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gv_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = L.load()
    decl = declared_symbols()
    assert len(decl) >= 19
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(L.EXPORTED) == decl


def test_status_strings_and_version():
    lib = L.load()
    assert lib.gv_abi_version() == 5
    for s in range(6):
        assert lib.gv_status_str(s)
    assert lib.gv_status_str(L.GV_ERR_CAPACITY) == b"intersection capacity exceeded"


def cam(w=960, h=540):
    return Camera(w, h, float(w), float(w), w / 2, h / 2)


def test_workspace_sizing_and_validation():
    lib = L.load()
    out = ctypes.c_size_t()
    c = cam()
    assert lib.gv_workspace_bytes(ctypes.byref(c.c()), 1000, 2, 5000, ctypes.byref(out)) == L.GV_OK
    small = out.value
    assert lib.gv_workspace_bytes(ctypes.byref(c.c()), 1000, 2, 50000, ctypes.byref(out)) == L.GV_OK
    assert out.value > small + 45000 * 60  # per-intersection storage
    cap = ctypes.c_int64()
    assert lib.gv_workspace_capacity(ctypes.byref(c.c()), 1000, 2, out.value, ctypes.byref(cap)) == L.GV_OK
    assert 50000 <= cap.value < 50010
    # invalid arguments
    assert lib.gv_workspace_bytes(ctypes.byref(c.c()), -1, 2, 10, ctypes.byref(out)) == L.GV_ERR_INVALID_ARG
    assert lib.gv_workspace_bytes(ctypes.byref(c.c()), 10, 0, 10, ctypes.byref(out)) == L.GV_ERR_INVALID_ARG
    assert lib.gv_workspace_bytes(ctypes.byref(c.c()), 10, 1, -5, ctypes.byref(out)) == L.GV_ERR_INVALID_ARG
    assert lib.gv_workspace_bytes(None, 10, 1, 5, ctypes.byref(out)) == L.GV_ERR_INVALID_ARG
    bad = cam()
    bad.width = 0
    assert lib.gv_workspace_bytes(ctypes.byref(bad.c()), 10, 1, 5, ctypes.byref(out)) == L.GV_ERR_INVALID_ARG
    bad = cam()
    bad.near_plane = 0.0
    assert lib.gv_workspace_bytes(ctypes.byref(bad.c()), 10, 1, 5, ctypes.byref(out)) == L.GV_ERR_INVALID_ARG
    bad = cam()
    bad.fx = float("nan")
    assert lib.gv_workspace_bytes(ctypes.byref(bad.c()), 10, 1, 5, ctypes.byref(out)) == L.GV_ERR_INVALID_ARG


def test_entry_points_reject_bad_arguments_before_touching_the_device():
    lib = L.load()
    c = cam(64, 48)
    sc = L.GvScene()
    sc.n, sc.dtype = 10, 7  # unknown dtype
    assert lib.gv_render_fwd(ctypes.byref(sc), ctypes.byref(c.c()), ctypes.c_void_p(256), 0.0,
                             ctypes.c_void_p(256), None, ctypes.c_void_p(256), 1 << 20, None) == L.GV_ERR_INVALID_ARG
    sc.dtype = L.GV_F32  # null parameter pointers with n > 0
    assert lib.gv_render_fwd(ctypes.byref(sc), ctypes.byref(c.c()), ctypes.c_void_p(256), 0.0,
                             ctypes.c_void_p(256), None, ctypes.c_void_p(256), 1 << 20, None) == L.GV_ERR_INVALID_ARG
    sc.n = 0  # valid empty scene but misaligned workspace
    assert lib.gv_render_fwd(ctypes.byref(sc), ctypes.byref(c.c()), ctypes.c_void_p(256), 0.0,
                             ctypes.c_void_p(256), None, ctypes.c_void_p(257), 1 << 20, None) == L.GV_ERR_WORKSPACE
    # workspace too small
    assert lib.gv_render_fwd(ctypes.byref(sc), ctypes.byref(c.c()), ctypes.c_void_p(256), 0.0,
                             ctypes.c_void_p(256), None, ctypes.c_void_p(256), 16, None) == L.GV_ERR_WORKSPACE
    # batch: unknown flag, missing targets for the L2 loss, zero frames
    g = L.GvGrads()
    for flags, frames in [(64, 2), (L.GV_FWD | L.GV_LOSS_L2, 2), (L.GV_FWD, 0), (0, 2)]:
        st = lib.gv_render_batch(ctypes.byref(sc), ctypes.byref(c.c()), ctypes.c_void_p(256), None, frames, None,
                                 None, flags, ctypes.c_void_p(256), None, ctypes.byref(g), None,
                                 ctypes.c_void_p(256), 1 << 30, None)
        assert st == L.GV_ERR_INVALID_ARG, (flags, frames)
    # fit graph: exactly one of targets / dL_dimages, and the ODE buffers are required
    h = ctypes.c_void_p()
    for tg, dl in [(None, None), (ctypes.c_void_p(256), ctypes.c_void_p(256))]:
        st = lib.gv_fit_graph_create(ctypes.byref(sc), ctypes.byref(c.c()), ctypes.c_void_p(256),
                                     ctypes.c_void_p(256), 4, ctypes.c_void_p(256), 1 << 20, None, 3, tg, dl,
                                     ctypes.c_void_p(256), ctypes.c_void_p(256), None, ctypes.byref(g),
                                     ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256),
                                     ctypes.c_void_p(256), 1 << 30, ctypes.byref(h))
        assert st == L.GV_ERR_INVALID_ARG
    # camera ODE
    sz = ctypes.c_size_t()
    assert lib.gv_camera_ode_workspace_bytes(100, 4, ctypes.byref(sz)) == L.GV_OK and sz.value > 396 * 4 * 136 * 4
    assert lib.gv_camera_ode_workspace_bytes(0, 4, ctypes.byref(sz)) == L.GV_ERR_INVALID_ARG
    assert lib.gv_camera_ode_fwd(None, None, 10, 4, None, None, 0, None) == L.GV_ERR_INVALID_ARG
    # trajectory error: argument checks happen before any launch
    assert lib.gv_pose_error(None, None, 10, None, None, None) == L.GV_ERR_INVALID_ARG
    dummy = ctypes.c_void_p(256)
    assert lib.gv_pose_error(dummy, dummy, 0, dummy, dummy, None) == L.GV_ERR_INVALID_ARG


def test_tuning_table_validation():
    lib = L.load()
    t = L.GvTuning()
    assert lib.gv_get_tuning(ctypes.byref(t)) == L.GV_OK
    old = (t.batch, t.sort_cap, t.compact, t.bwd_batch)
    assert t.batch in (64, 128, 256) and t.sort_cap in (512, 1024, 2048, 4096) and 0 <= t.compact <= 63
    assert t.bwd_batch in (64, 128, 256)
    t2 = L.GvTuning()
    t2.batch, t2.sort_cap, t2.compact = 128, 2048, 64  # kernel choice out of range
    assert lib.gv_set_tuning(ctypes.byref(t2)) == L.GV_ERR_INVALID_ARG
    t2.compact = 0
    t2.batch, t2.sort_cap = 100, 4096
    assert lib.gv_set_tuning(ctypes.byref(t2)) == L.GV_ERR_INVALID_ARG
    t2.batch, t2.sort_cap, t2.bwd_batch = 128, 2048, 96
    assert lib.gv_set_tuning(ctypes.byref(t2)) == L.GV_ERR_INVALID_ARG
    t2.bwd_batch = 0  # same as batch
    assert lib.gv_set_tuning(ctypes.byref(t2)) == L.GV_OK
    assert lib.gv_get_tuning(ctypes.byref(t)) == L.GV_OK
    assert (t.batch, t.sort_cap, t.bwd_batch) == (128, 2048, 128)
    t2.batch, t2.sort_cap, t2.compact, t2.bwd_batch = old
    assert lib.gv_set_tuning(ctypes.byref(t2)) == L.GV_OK
    assert lib.gv_get_tuning(ctypes.byref(t)) == L.GV_OK and (t.batch, t.sort_cap, t.compact, t.bwd_batch) == old


def test_dynamic_scene_validation():
    """B-spline / polynomial / SH scene fields are checked before anything is
    enqueued (no GPU needed: the calls fail on the host)."""
    lib = L.load()
    cam = L.GvCamera(64, 48, 64.0, 64.0, 32.0, 24.0, 0.01, 0.3)
    fake = 0x1000  # never dereferenced: validation fails first
    sz = ctypes.c_size_t()
    assert lib.gv_workspace_bytes(ctypes.byref(cam), 10, 1, 1000, ctypes.byref(sz)) == L.GV_OK

    def scene(**kw):
        s = L.GvScene()
        s.n, s.dtype = 10, L.GV_F32
        s.means = s.log_scales = s.quats = s.opacity_logits = s.colors = fake
        for k, v in kw.items():
            setattr(s, k, v)
        return s

    pose = fake
    bad = [scene(n_ctrl=3, ctrl=fake), scene(n_ctrl=L.GV_MAX_CTRL + 1, ctrl=fake), scene(n_ctrl=5, ctrl=None),
           scene(n_ctrl=0, ctrl=fake), scene(n_ctrl=5, ctrl=fake, mean_coeffs=fake),
           scene(sh_degree=4, sh=fake), scene(sh_degree=2, sh=None), scene(sh_degree=0, sh=fake),
           scene(sh_degree=-1, sh=fake)]
    for s in bad:
        st = lib.gv_project_fwd(ctypes.byref(s), ctypes.byref(cam), pose, 0.0, fake, fake, None, 0, None)
        assert st == L.GV_ERR_INVALID_ARG
    # a well-formed dynamic scene passes validation and stops at the missing workspace
    good = [scene(n_ctrl=5, ctrl=fake, means=None), scene(n_ctrl=4, ctrl=fake, scale_coeffs=fake, quat_coeffs=fake),
            scene(scale_coeffs=fake), scene(sh_degree=3, sh=fake), scene(sh_degree=1, sh=fake, n_ctrl=6, ctrl=fake)]
    for s in good:
        st = lib.gv_project_fwd(ctypes.byref(s), ctypes.byref(cam), pose, 0.0, fake, fake, None, 0, None)
        assert st == L.GV_ERR_WORKSPACE


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_LIB", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "libgv.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        L.load()


def test_adan_argument_validation():
    """gv_adan_step checks its arguments on the host (no GPU needed)."""
    lib = L.load()
    fake = 0x1000
    P = (ctypes.c_void_p * 2)(fake, fake)
    C = (ctypes.c_int64 * 2)(10, 5)
    ok = L.GvAdanParams(0.01, 0.02, 0.08, 0.01, 1e-8, 0.0, 0, 0)
    assert lib.gv_adan_step(0, P, P, P, C, ctypes.byref(ok), None) == L.GV_ERR_INVALID_ARG
    assert lib.gv_adan_step(L.GV_ADAN_MAX_TENSORS + 1, P, P, P, C, ctypes.byref(ok), None) == L.GV_ERR_INVALID_ARG
    for field, value in (("step", -1), ("beta1", 1.5), ("beta3", -0.1), ("eps", 0.0), ("lr", float("nan")),
                         ("weight_decay", -1.0)):
        hp = L.GvAdanParams(0.01, 0.02, 0.08, 0.01, 1e-8, 0.0, 0, 0)
        setattr(hp, field, value)
        assert lib.gv_adan_step(2, P, P, P, C, ctypes.byref(hp), None) == L.GV_ERR_INVALID_ARG, field
    Z = (ctypes.c_int64 * 2)(0, 0)
    assert lib.gv_adan_step(2, P, P, P, Z, ctypes.byref(ok), None) == L.GV_OK  # nothing to do, nothing launched
    N = (ctypes.c_void_p * 2)(fake, None)
    assert lib.gv_adan_step(2, P, N, P, C, ctypes.byref(ok), None) == L.GV_ERR_INVALID_ARG


def test_pyramid_sizes_and_validation():
    lib = L.load()
    n = ctypes.c_int64()
    assert lib.gv_pyramid_floats(6, 540, 960, 4, ctypes.byref(n)) == L.GV_OK
    assert n.value == 6 * (270 * 480 + 135 * 240 + 68 * 120)
    assert lib.gv_pyramid_floats(1, 7, 5, 1, ctypes.byref(n)) == L.GV_OK and n.value == 0
    assert lib.gv_pyramid_floats(0, 7, 5, 2, ctypes.byref(n)) == L.GV_ERR_INVALID_ARG
    assert lib.gv_pyramid_floats(1, 7, 5, 17, ctypes.byref(n)) == L.GV_ERR_INVALID_ARG
    assert lib.gv_gaussian_pyramid(None, 1, 8, 8, 2, 0x1000, None) == L.GV_ERR_INVALID_ARG
    assert lib.gv_gaussian_pyramid(0x1000, 1, 8, 8, 2, None, None) == L.GV_ERR_INVALID_ARG
