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


def test_golden_lookup_requires_the_same_input_bytes(tmp_path):
    """The benchmark's eigenvalue gate for the large block inputs uses the
    cached oracle solve only for the exact input bytes it was computed on."""
    import numpy as np
    from paper_1008_0201_amd import workloads as W
    B = load_bench()
    G = np.asfortranarray(np.arange(12.0).reshape(4, 3) + 0.5)
    (tmp_path / "x.json").write_text(json.dumps({"input_sha256": W.input_sha256(G), "oracle": "o",
                                                 "sweeps": 3}))
    np.save(tmp_path / "x.lam.npy", np.array([1.0, 2.0, 3.0]))
    B.GOLDEN = str(tmp_path)
    B.GOLDEN_OF = {"wl": "x"}
    lam, meta = B.golden_eigs("wl", G)
    assert list(lam) == [1.0, 2.0, 3.0] and meta["sweeps"] == 3
    G2 = G.copy()
    G2[1, 2] = np.nextafter(G2[1, 2], 1e9)
    lam2, why = B.golden_eigs("wl", G2)
    assert lam2 is None and "differ" in why["reason"]
    assert B.golden_eigs("other", G)[0] is None


def test_committed_golden_records_are_complete():
    """Each cached oracle solve under tests/golden/ has its eigenvalues, the
    input hash, the oracle configuration and the command that made it."""
    import glob
    import numpy as np
    B = load_bench()
    names = set(B.GOLDEN_OF.values())
    for path in glob.glob(os.path.join(ROOT, "tests", "golden", "*.json")):
        meta = json.load(open(path))
        name = os.path.basename(path)[:-len(".json")]
        assert name in names, name
        lam = np.load(path[:-len(".json")] + ".lam.npy", allow_pickle=False)
        assert lam.shape == (meta["n"],) and np.all(np.isfinite(lam))
        assert len(meta["input_sha256"]) == 64 and meta["status"] == 0
        assert meta["command"].startswith("python tests/golden/make_block_golden.py")
        if "truth" in meta:
            # the high-precision solve of the same input, for the gate's (1.2) fallback
            lam80 = np.load(path[:-len(".json")] + ".lam80.npy", allow_pickle=False)
            assert lam80.shape == (meta["n"],) and np.all(np.isfinite(lam80))
            assert meta["truth"]["command"].startswith("python tests/golden/make_block_golden.py --truth")
            assert meta["kappa_colscaled"] >= 1.0
