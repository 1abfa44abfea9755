"""The benchmark's output contract: one JSON line with the fields the
measurement is read from, and a clear refusal of multi-GPU runs."""
import io
import json
import os
import subprocess
import sys
from contextlib import redirect_stdout

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_single_thread_oracle_child():
    """The CPU baseline's single-thread run (a child process on one OpenMP
    thread, no GPU) prints the whole tiny frame's time as one JSON line."""
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-tiny-child"],
                       capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-500:]
    d = json.loads(r.stdout.strip().splitlines()[-1])
    assert d["threads"] == 1 and (d["W"], d["H"]) == (256, 256) and d["seconds"] > 0


@pytest.mark.gpu
def test_bench_line_fields(monkeypatch):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "tiny_x2", "--steps", "2", "--warmup", "1",
                                      "--no-cpu-baseline"])
    print("bench tiny_x2, 2 steps", flush=True)
    buf = io.StringIO()
    with redirect_stdout(buf):
        bench.main()
    line = json.loads(buf.getvalue().strip().splitlines()[-1])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in line, k
    assert line["n_gpus"] == 1 and line["steps"] == 2 and line["warmup"] == 1
    assert line["value"] > 0 and line["ms_per_step"] > 0 and line["higher_is_better"] is True
    assert "workload" in line["config"]
    roof = line["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert roof["bound"] == "alu" and roof["peak"] == 39.32
    # both printed rounded: frac to 4 decimals, achieved to 3
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], abs=1e-4)
    # the work behind it: 16 lane-op slots per evaluated and 35 more per
    # blended fragment, over the launch time
    fr = line["fragments"]
    assert fr["lowres_evaluated"] >= fr["lowres_blended"] > 0
    ops = 16 * fr["lowres_evaluated"] + 35 * fr["lowres_blended"]
    # (ms_per_launch is printed to 4 decimals: a few percent on the tiny frame)
    assert roof["achieved"] == pytest.approx(ops / (roof["ms_per_launch"] * 1e-3) / 1e12, rel=0.03)
    for st in ("project", "bin_sort"):
        sr = line["stage_rooflines"][st]
        assert sr["bound"] == "hbm" and 0 < sr["frac"] < 1
    assert roof["traffic"] is None  # counters were taken on the scene workload only
    assert 0 < line["upscaler_roofline"]["frac"] < 1
    orbit = line["orbit_cameras"]
    assert len(orbit["ms_per_frame"]) == 8 and len(orbit["direct_best_ms_per_frame"]) == 8
    assert orbit["median_value"] > 0 and orbit["median_speedup_vs_best_direct"] > 0
