"""The parts of bench.py that need no GPU: the single-GPU refusal, the HBM-traffic lookup
in the committed counter summary (valid only for the kernel sources it was taken on), and
the CPU-baseline record of the oracle."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(args, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                       text=True, timeout=60, env=dict(os.environ, **env))
    assert r.returncode == 2
    assert "single-GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_comes_from_a_current_counter_summary(tmp_path, monkeypatch):
    from paper_2605_14505_amd.profsummary import kernel_source_hash

    key = "step_256_27x19_fp32_fp32_shift"
    path = os.path.join(ROOT, "profiles", f"{key}_counters.txt")
    kv = dict(line.split(" = ", 1) for line in open(path) if " = " in line and not line.startswith("#"))
    traffic, src = bench.read_traffic(key, 256 ** 3, 368)
    if kv["source_hash"].strip() == kernel_source_hash():
        assert traffic == float(kv["hbm_bytes_per_launch"])
        assert src == os.path.relpath(path, ROOT)
        # within a few percent of the algorithmic bytes (the scaled counters read them to
        # rounding): no wasted re-reads
        assert 0.995 <= traffic / (368 * 256 ** 3) < 1.05
    else:
        assert traffic is None and "predate" in src
    assert bench.read_traffic("no_such_workload", 1, 1) == (None, "no counter summary")
    # a summary taken on other sources is not used
    stale = tmp_path / "profiles"
    stale.mkdir()
    (stale / f"{key}_counters.txt").write_text("source_hash = 0000\nhbm_bytes_per_launch = 1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic(key, 256 ** 3, 368) == (None, "counters predate the current kernel sources")


def test_cpu_baseline_record():
    rec = bench.cpu_baseline(8, 1, "shift")
    assert set(rec) == {"value", "unit", "cores", "kind", "sample"}
    assert rec["unit"] == "MLUPS" and rec["kind"] == "oracle" and rec["cores"] == 1
    assert rec["value"] > 0
    assert "8^3" in rec["sample"]


def test_source_hash_follows_code_not_comments():
    # the counters' source hash ignores comments and layout, and sees any change of code
    from paper_2605_14505_amd.profsummary import code_only
    a = "int f(int x) {  // doubles\n  return 2 * x; /* one line */\n}\n"
    b = "int f(int x) {\n  /* a longer\n     comment */ return 2 * x;\n}  // done\n"
    c = "int f(int x) {\n  return 3 * x;\n}\n"
    assert code_only(a) == code_only(b) == "int f(int x) { return 2 * x; }"
    assert code_only(c) != code_only(a)
