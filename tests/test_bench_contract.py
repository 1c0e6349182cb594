"""The benchmark's output line (one JSON object on stdout) keeps its contract:
the required keys, a roofline object for the dominant kernel and, on request,
the CPU-oracle baseline.  Runs bench.py briefly in a child process."""
import json
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    return json.loads(lines[0])


@pytest.mark.gpu
def test_headline_line():
    d = _run("--steps", "20", "--warmup", "20", "--timed-steps", "10", "--no-copy-bw", "--cpu-steps", "2")
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 20
    assert d["value"] > 0 and d["dtype"] == "f32" and d["vs_baseline"] is None
    assert "workload" in d["config"]
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12 and 0 < r["frac"] < 1
    assert d["config"]["grid"] == [8192, 8192]
    m = d["mall_resident_2048"]
    assert m["grid"] == [2048, 2048] and m["value"] > 0 and 0 < m["roofline"]["frac"] < 1
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0 and c["sample"]
    assert "cpu_model" in c and "cpu_mhz_max" in c


def test_more_than_one_gpu_is_refused():
    # no GPU needed: the run stops before touching one
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_run_record_appends_line_with_provenance(tmp_path, capsys):
    # the JSONL record: the printed line plus time, command, source hashes and
    # host; a stand-in for torch supplies the GPU name off the GPU
    sys.path.insert(0, ROOT)
    import bench

    class _Cuda:
        @staticmethod
        def get_device_name(i):
            return "stand-in GPU"

    class _Torch:
        cuda = _Cuda()
        __version__ = "0"

        class version:
            hip = None

    class _Args:
        record = str(tmp_path / "runs.jsonl")

    line = {"metric": "m", "value": 1.0}
    bench.emit(line, _Args(), _Torch())
    bench.emit(dict(line, value=2.0), _Args(), _Torch())
    assert json.loads(capsys.readouterr().out.splitlines()[0]) == line
    recs = [json.loads(ln) for ln in open(_Args.record)]
    assert [r["value"] for r in recs] == [1.0, 2.0]
    rec = recs[0]["record"]
    assert rec["gpu"] == "stand-in GPU" and rec["host"]["logical_cpus"] >= 1
    assert set(rec["source_hashes"]) == {"step2d", "x_sweep"} and all(len(v) == 16 for v in rec["source_hashes"].values())
