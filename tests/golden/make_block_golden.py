"""Writes the eigenvalues of the large block workloads, computed once by the
oracle (oracle/, FP64), to tests/golden/: the benchmark and the GPU tests
look them up by the SHA-256 of the input bytes instead of running a CPU solve
of an hour or more each time.

TEST INFRASTRUCTURE: calls only oracle/ (and the input generators of
paper_1008_0201_amd/workloads.py, which hold none of the method's
arithmetic).  The oracle runs the block method of Alg. 3.4 (block-oriented,
b = 32, modified modulus block ordering; for the indefinite workload full
block with the sign-pivoted Cholesky of Alg. 3.3) with the disjoint pivots
of each step spread over all host cores; that threaded run is bit for bit
the sequential oracle (tests/test_oracle_pins.py pins it).

    python tests/golden/make_block_golden.py spd-graded-T-n8192 [...]
    python tests/golden/make_block_golden.py --truth hyperbolic-graded-n4096 [...]

Each workload gives <name>.lam.npy (eigenvalues in column order) and
<name>.json (input hash, oracle configuration, status, sweeps, time, host).
--truth adds, for a workload already cached, the same oracle run in 80-bit
long double (<name>.lam80.npy, whose error is smaller by 2^11 than an FP64
run's) and kappa_2 of the factor with its columns scaled to unit norm: the
high-precision reference and the condition number of the relative accuracy
bound (1.2) that the eigenvalue gate falls back to (oracle/gates.py).
"""
import json
import os
import platform
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_1008_0201_amd import workloads as W  # noqa: E402


def workload(name):
    """(Workload, oracle options) of a golden workload."""
    if name == "spd-graded-T-n8192":
        return W.graded_spd_transposed(8192, lam_decades=3.0), dict(b=32, full_block=False)
    if name == "spd-graded-T-n4096":
        return W.graded_spd_transposed(4096, lam_decades=3.0), dict(b=32, full_block=False)
    if name == "hyperbolic-graded-n4096":
        return (W.graded_hyperbolic(4096, k=6, grade=2.0),
                dict(b=32, full_block=True, sign_pivot=True))
    raise SystemExit("unknown golden workload %r" % name)


def host():
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo")
                 if l.startswith("model name")][0]
    except (OSError, IndexError):
        model = platform.processor()
    return "%s, %d logical CPUs" % (model, os.cpu_count())


def truth(names):
    from oracle import gates
    for name in names:
        wl, opt = workload(name)
        meta_path = os.path.join(HERE, name + ".json")
        meta = json.load(open(meta_path))
        if meta["input_sha256"] != W.input_sha256(wl.G):
            raise SystemExit("%s: input differs from the cached FP64 solve" % name)
        t = time.perf_counter()
        r = O.block_jevd(wl.G, wl.J, wl.n * 1e-19, want_v=False, nthreads=0, prec="l", **opt)
        dt = time.perf_counter() - t
        if r.status != 0:
            raise SystemExit("%s: 80-bit oracle status %d" % (name, r.status))
        np.save(os.path.join(HERE, name + ".lam80.npy"), r.lam)
        meta["truth"] = {"oracle": "block_jevd 80-bit long double " + json.dumps(opt),
                         "tol": wl.n * 1e-19, "sweeps": r.sweeps, "seconds": round(dt, 1),
                         "command": "python tests/golden/make_block_golden.py --truth " + name}
        meta["kappa_colscaled"] = gates.kappa_colscaled(wl.G)
        with open(meta_path, "w") as f:
            json.dump(meta, f, indent=1)
            f.write("\n")
        print(json.dumps(meta["truth"]), meta["kappa_colscaled"], flush=True)


def main(names):
    for name in names:
        t = time.perf_counter()
        wl, opt = workload(name)
        gen_s = time.perf_counter() - t
        sha = W.input_sha256(wl.G)
        t = time.perf_counter()
        r = O.block_jevd(wl.G, wl.J, wl.tol, want_v=False, nthreads=0, **opt)
        dt = time.perf_counter() - t
        if r.status != 0:
            raise SystemExit("%s: oracle status %d" % (name, r.status))
        np.save(os.path.join(HERE, name + ".lam.npy"), r.lam)
        meta = {"workload": name, "n": wl.n, "m": wl.m, "tol": wl.tol,
                "input_sha256": sha, "oracle": "block_jevd FP64 " + json.dumps(opt),
                "status": r.status, "sweeps": r.sweeps, "breakdowns": r.extra,
                "rotations_per_sweep": [int(x) for x in r.rot],
                "seconds": round(dt, 1), "input_generation_s": round(gen_s, 1),
                "threads": os.cpu_count(), "host": host(),
                "command": "python tests/golden/make_block_golden.py " + name}
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(meta, f, indent=1)
            f.write("\n")
        print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    if sys.argv[1:2] == ["--truth"]:
        truth(sys.argv[2:])
    else:
        main(sys.argv[1:])
