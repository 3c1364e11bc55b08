"""The benchmark's output contract on a small workload: one JSON line with the metric, the
roofline object of the dominant kernel, the CPU baseline of the oracle and the sweeps."""
import json
import subprocess
import sys
from pathlib import Path

import pytest

pytestmark = pytest.mark.gpu
ROOT = Path(__file__).resolve().parents[1]


def test_bench_json_line():
    cmd = [sys.executable, "-u", str(ROOT / "bench.py"), "--target-tris", "20000", "--steps", "2", "--warmup", "2",
           "--snapshots", "40", "--modes", "16", "--hidden", "32", "--epochs", "20", "--window", "16",
           "--batch", "3", "--batch-steps", "1", "--batch-window", "4", "--cpu-steps", "1", "--spmv-sweep", "0",
           "--cg-sweep", "0", "--level-warmup", "1", "--level-steps", "2", "--bfs-nx", "60"]
    r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=600)
    print(r.stderr[-3000:], flush=True)
    assert r.returncode == 0, r.stderr[-3000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "paths", "batch", "levels",
                "backward_step", "max_abs_u_first_last", "kinetic_energy_first_last"):
        assert key in line, key
    assert line["n_gpus"] == 1 and line["steps"] == 2 and line["warmup"] == 2 and line["value"] > 0
    assert line["config"]["workload"] and line["config"]["path"] in line["paths"]
    roof = line["roofline"]
    assert roof["bound"] == "hbm" and roof["peak"] == 8000.0 and roof["unit"] == "GB/s"
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3 and roof["avg_us"] > 0
    cpu = line["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["cores"] >= 1 and cpu["value"] > 0 and cpu["sample"]
    assert cpu["nproc"] >= 1 and cpu["cpu_model"] and cpu["openmp"]["cores"] == cpu["nproc"]
    # every reported path is within the 1e-6 bar of plain FP64 when it is the chosen one, at its restart
    # and after its timed steps, and the flow stays bounded
    chosen = line["paths"][line["config"]["path"]]
    assert chosen["rel_err_vs_fp64"] <= 1e-6 and chosen["rel_err_vs_fp64_after_timed_steps"] <= 1e-6
    assert max(line["max_abs_u_first_last"]) < 5.0
    assert [p["levels"] for p in line["levels"]["points"]] == [3, 2, 1, 0]
    assert len({p["resolution"].split(":")[0] for p in line["levels"]["points"]}) == 1  # one fine mesh
    assert [p["levels"] for p in line["backward_step"]["points"]] == [1, 0]
    b = line["batch"]
    assert b["instances"] == 3 and b["rel_err_vs_single_instance_gpu"] <= 1e-6
