"""bench.py's host-side logic (no GPU): the one-GPU contract, the per-unit
byte and operation figures of the roofline, the counter-profile summary, and
a static check that every global name its functions use is defined."""
import ast
import builtins
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_stage_bytes_per_unit_figures():
    # benchmark clip: 50 frames of 960x540, 31,917,790 intersections per step
    K, P, F = 31_917_790, 960 * 540, 50
    assert bench.stage_bytes("composite_bwd", 200_000, 190_000, K, P, F) == F * P * 20 + K * 76
    assert bench.stage_bytes("composite_bwd", 200_000, 190_000, K, P, F) == pytest.approx(2.944e9, rel=1e-3)
    assert bench.stage_bytes("composite_fwd", 200_000, 190_000, K, P, F) == K * 40 + F * P * 32
    assert bench.stage_bytes("sort", 1, 1, K, P, F) == 24 * K


def test_alu_peaks():
    assert bench.ALU_PEAK == pytest.approx(157.3e12)
    assert bench.ALU_PEAK_NONPACKED == pytest.approx(78.6432e12)
    assert bench.LDS_PEAK == pytest.approx(256 * 128 * 2.4e9)


def test_counters_summary():
    c = dict(avg_ms=4.0, SQ_INSTS_VALU=2.0e9, GRBM_GUI_ACTIVE=8 * 9.6e6, SQ_THREAD_CYCLES_VALU=4.0e11,
             SQ_ACTIVE_INST_VALU=1.0e10, SQ_LDS_IDX_ACTIVE=1.2288e9, SQ_LDS_BANK_CONFLICT=2.4576e8,
             SQ_INSTS_LDS_LOAD_BANDWIDTH=1e9, SQ_INSTS_LDS_STORE_BANDWIDTH=1e8)
    out = bench.counters_summary(c, pairs=1.0e9)
    assert out["clock_ghz"] == pytest.approx(2.4)
    assert out["valu_lane_insts_per_pair"] == pytest.approx(128.0)
    assert out["valu_issue_share"] == pytest.approx(2.0e9 * 4 / (9.6e6 * 1024), abs=1e-3)
    assert out["valu_lane_util"] == pytest.approx(0.625)
    assert out["lds_util"] == pytest.approx(0.5)
    assert out["lds_bank_conflict_share"] == pytest.approx(0.1)
    assert out["lds_bytes"] == pytest.approx(64 * 1.1e9)


def test_no_undefined_globals():
    """Every name a function of bench.py loads is local, a module global or a builtin."""
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    defined = set(dir(builtins)) | {"__file__"}
    for n in tree.body:
        if isinstance(n, (ast.FunctionDef, ast.ClassDef)):
            defined.add(n.name)
        elif isinstance(n, ast.Assign):
            defined.update(t.id for t in n.targets if isinstance(t, ast.Name))
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            defined.update((a.asname or a.name).split(".")[0] for a in n.names)
    missing = []
    for f in (n for n in tree.body if isinstance(n, ast.FunctionDef)):  # nested functions see these locals
        local = set()
        for x in ast.walk(f):
            if isinstance(x, ast.Name) and isinstance(x.ctx, ast.Store):
                local.add(x.id)
            elif isinstance(x, ast.arg):
                local.add(x.arg)
            elif isinstance(x, (ast.Import, ast.ImportFrom)):
                local.update((a.asname or a.name).split(".")[0] for a in x.names)
            elif isinstance(x, ast.FunctionDef):
                local.add(x.name)
        missing += [(f.name, x.id) for x in ast.walk(f)
                    if isinstance(x, ast.Name) and isinstance(x.ctx, ast.Load) and x.id not in local | defined]
    assert not missing, missing
