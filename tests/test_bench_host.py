"""Host-side checks of the benchmark script: the one-GPU contract and the
guard on the committed HBM traffic counters.  CPU only."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "one gpu" in r.stderr.lower()
    assert r.stdout.strip() == ""


def test_traffic_record_is_used_only_for_its_workload_and_sources(tmp_path):
    """measured_traffic returns the recorded bytes per launch when the
    workload matches and the kernel's sources hash to the recorded value,
    and None otherwise (another workload, a changed source, no record)."""
    B = load_bench()
    src = tmp_path / "k.hip"
    src.write_text("// kernel source\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    (tmp_path / "profiles").mkdir()
    rec = {"k": {"workload": "w", "fetch_kib_per_launch": 3.0, "write_kib_per_launch": 5.0,
                 "scale_fetch": 1.0, "scale_write": 2.0, "source_sha256_16": digest,
                 "sources": ["k.hip"]}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    B.ROOT = str(tmp_path)
    assert B.measured_traffic("k", "w") == 1024.0 * (3.0 + 10.0)
    assert B.measured_traffic("k", "other") is None
    assert B.measured_traffic("missing", "w") is None
    src.write_text("// kernel source, changed\n")
    assert B.measured_traffic("k", "w") is None


def test_committed_traffic_records_name_existing_sources_and_known_workloads():
    """Every record of profiles/traffic.json names source files that exist and
    a workload the benchmark knows (whether its hash is current is what the
    benchmark checks at run time)."""
    recs = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    bench_text = open(os.path.join(ROOT, "bench.py")).read()
    assert recs
    for kernel, rec in recs.items():
        for f in rec["sources"]:
            assert os.path.exists(os.path.join(ROOT, f)), (kernel, f)
        assert '"%s"' % rec["workload"] in bench_text, (kernel, rec["workload"])
        assert rec["fetch_kib_per_launch"] > 0 and rec["write_kib_per_launch"] > 0
