"""bench.py prints one JSON line with the agreed fields.

bench.main() runs in this process on a small R-MAT graph (scale 14) with a
short CPU baseline: the line must carry the metric, value and unit, the step
bookkeeping, the roofline object (HBM bound at the 8 TB/s peak, frac =
achieved / peak) and the CPU-oracle baseline.  A request for several GPUs is
refused with its own message (no GPU needed for that).
"""
import json
import os
import sys

import pytest

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.gpu
def test_bench_json_line(monkeypatch, capsys):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    monkeypatch.setattr(sys, "argv", ["bench.py", "--scale", "14", "--steps", "2", "--warmup",
                                      "1", "--cpu-seconds", "1"])
    bench.main()
    out = capsys.readouterr().out
    lines = [ln for ln in out.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, out
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["unit"] == "GTEPS" and d["value"] > 0 and d["higher_is_better"] is True
    assert d["config"]["workload"].startswith("rmat14")
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] > 0 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1 and c["sample"]
    q = d["quality"]
    assert -0.5 <= q["q_async"] <= 1 and -0.5 <= q["q_det"] <= 1
    assert q["q_exact_oracle"] == c["exact_rule_run"]["q"]
    assert 1 <= q["det_iterations"] <= 20


def _json_line(out):
    lines = [ln for ln in out.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, out
    return json.loads(lines[0])


@pytest.mark.gpu
def test_bench_batch_and_serve_lines(monkeypatch, capsys):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "batch", "--batch-graphs", "16",
                                      "--steps", "1", "--warmup", "1", "--capture",
                                      "--autotune"])
    bench.main()
    d = _json_line(capsys.readouterr().out)
    assert d["unit"] == "graphs/s" and d["value"] > 0 and d["identical_labels_and_iterations"]
    assert d["config"]["captured"] is True and d["config"]["autotuned"] is True
    assert d["default_shape_graphs_per_s"] > 0 and d["autotune"]["batch_ms_by_blocks"]
    assert d["cpu_baseline"]["labels_equal_gpu_batched"] is True
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "serve", "--requests", "12",
                                      "--serve-max-scale", "14", "--serve-loads", "1.0",
                                      "--warmup", "1"])
    bench.main()
    d = _json_line(capsys.readouterr().out)
    assert d["unit"] == "graphs/s" and d["value"] > 0 and d["identical_to_alone"]
    assert d["config"]["overlapped_admission"] is True
    assert d["p99_ms"] >= d["p50_ms"] > 0


def test_bench_refuses_several_gpus(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as ei:
        bench.main()
    assert ei.value.code != 0
    assert "one GPU" in capsys.readouterr().err
