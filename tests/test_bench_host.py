"""Host-side logic of bench.py (no GPU): the one-GPU contract and the use of
the committed HBM counter summary."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

PLAN = {"tile": 1024, "grid_blocks": 1024, "march_slots": 2, "march_planes": 16, "march_items": 256}


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _summary():
    with open(os.path.join(ROOT, "profiles", "traffic_3d_bumps_128.json")) as f:
        return json.load(f)


def test_traffic_follows_the_fused_pass_plan(monkeypatch):
    d = _summary()
    ent = d["kernels"]["lanczos_step:c128"]
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: d["sources"])
    plan = dict(ent["tiling"])
    assert bench.load_traffic("lanczos_step", "c128", plan) == ent["hbm_bytes_per_launch"]
    # the grid-stride tiling of the other kernels does not change the pass's bytes
    plan2 = dict(plan, tile=512, grid_blocks=2048)
    assert bench.load_traffic("lanczos_step", "c128", plan2) == ent["hbm_bytes_per_launch"]
    # another plan of the fused pass, another precision: no counted traffic
    assert bench.load_traffic("lanczos_step", "c128", dict(plan, march_planes=8, march_items=512)) is None
    assert bench.load_traffic("lanczos_step", "c64", plan) is None


def test_traffic_needs_the_profiled_sources(monkeypatch):
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "0" * 16)
    assert bench.load_traffic("lanczos_step", "c128", PLAN) is None
