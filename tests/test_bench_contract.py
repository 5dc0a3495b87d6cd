"""bench.py on the host: the one-GPU refusal, and that every committed HBM
traffic summary parses and still matches the kernel sources it was taken on
(a stale figure would make the bench report ``traffic`` as null)."""
import glob
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from profile_summary import CLASSES, source_digest  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _traffic_blocks():
    out = {}
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md"))):
        text = open(path).read()
        assert "```json" in text, path
        block = text.split("```json", 1)[1].split("```", 1)[0]
        out[os.path.basename(path)] = json.loads(block)
    return out


def test_traffic_summaries_are_current():
    blocks = _traffic_blocks()
    assert blocks, "no HBM traffic summaries under profiles/"
    for name, per_workload in blocks.items():
        for workload, table in per_workload.items():
            assert table, (name, workload)
            for cls, entry in table.items():
                assert cls in CLASSES, (name, cls)
                assert entry["bytes_per_launch"] > 0, (name, cls)
                assert entry["digest"] == source_digest(cls), \
                    f"{name}: {cls} sources changed since the counters were taken"


def test_bench_reads_the_traffic_figures():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    for per_workload in _traffic_blocks().values():
        for workload, table in per_workload.items():
            for cls, entry in table.items():
                assert bench.measured_traffic(workload, cls) == entry["bytes_per_launch"]
    assert bench.measured_traffic("no_such_workload", "apply_dot") is None
