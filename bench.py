#!/usr/bin/env python3
"""Benchmark of the one-sided Jacobi eigensolver on one MI355X.

A step is one complete solve (all sweeps to convergence, plus the
eigenvalue/eigenvector finalisation) of one synthetic input that is already
resident in device memory: the working copy of G is restored from a pristine
device copy (a device-to-device copy of m*n*8 bytes, inside the step) and
jacobi_evd runs on it.  Prints one JSON line.

Metric: one-sided Jacobi effective GFLOP/s = sweeps * W / t, with the nominal
work per sweep W = P (12 m + 6 n) for P pairs per sweep (three dot products,
the rotation of the G pair and of the V pair per pair), counted only when the
eigenvalues agree with the CPU oracle to a relative error <= 1e-12.

Workloads (seeded, synthetic; see paper_1008_0201_amd/workloads.py):
  hyperbolic-graded-n1024 (default): G = B diag(10^U(-3,3)), B ~ N(0,1),
      1024 x 1024, J = diag(+1 x 512, -1 x 512), modified modulus, tol n eps
  spd-gaussian-n64: G ~ N(0,1) 64 x 64, J = I, row-cyclic, tol 64 eps
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def pairs_per_sweep(n, ordering):
    if ordering == 0:
        return n * (n - 1) // 2
    if n % 2 == 0:
        return n * (n // 2) if ordering == 2 else n * (n - 1) // 2
    return n * (n - 1) // 2


def make_workload(name):
    from paper_1008_0201_amd import workloads as W
    if name == "hyperbolic-graded-n1024":
        return W.graded_hyperbolic(1024), 0
    if name == "spd-gaussian-n64":
        return W.spd_gaussian(64, ordering=W.ROWCYCLIC, tol_factor=64), 0
    raise SystemExit("unknown workload %r" % name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="hyperbolic-graded-n1024")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (profiling runs); no accuracy gate then")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this solver has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1008_0201_amd import jevd

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    wl, variant = make_workload(args.workload)
    m, n = wl.m, wl.n
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    G0 = torch.from_numpy(np.ascontiguousarray(wl.G.T)).to(dev).T      # pristine, column-major
    Gd = torch.empty((n, m), dtype=torch.float64, device=dev).T
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    U = torch.empty((n, m), dtype=torch.float64, device=dev).T
    V = torch.empty((n, n), dtype=torch.float64, device=dev).T
    Jb = None if wl.J is None else wl.J.tobytes()
    h = jevd.jevd_create(stream.cuda_stream)
    opts = jevd.jevd_default_opts()
    opts.ordering = wl.ordering
    opts.variant = variant

    def step():
        Gd.copy_(G0)
        st, sweeps = jevd.jacobi_evd(h, m, n, Gd.data_ptr(), m, Jb, wl.tol, opts, lam.data_ptr(),
                                     U.data_ptr(), m, V.data_ptr(), n)
        if st != 0:
            raise RuntimeError("jacobi_evd: %s" % jevd.jevd_strerror(st))
        return sweeps

    for _ in range(args.warmup):
        step()
    jevd.jevd_set_timing(h, True)
    kms, klaunch = 0.0, 0
    sweeps_seen = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sweeps_seen.append(step())
        info = jevd.jevd_get_info(h)
        kms += info.kernel_ms[jevd.K_PAIR_STEP]
        klaunch += info.kernel_launches[jevd.K_PAIR_STEP]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    jevd.jevd_set_timing(h, False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    sweeps = sweeps_seen[-1]
    P = pairs_per_sweep(n, wl.ordering)
    work = P * (12.0 * m + 6.0 * n)
    gflops = sweeps * work / (ms_per_step * 1e-3) / 1e9
    lam_gpu = np.sort(lam.cpu().numpy())

    # roofline of the dominant kernel: nominal pair-stream bytes per launch
    # (32 (m + n) bytes per pair: read and write both columns of G and of V)
    if wl.ordering == 0:
        pairs_per_launch = None
    else:
        steps_per_sweep = n
        pairs_per_launch = P / steps_per_sweep
    roofline = None
    if klaunch and pairs_per_launch:
        avg_ms = kms / klaunch
        bytes_per_launch = pairs_per_launch * 32.0 * (m + n)
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": "k_pair_step", "avg_launch_us": round(avg_ms * 1e3, 3),
                    "bytes_per_launch": bytes_per_launch}

    cpu = None
    gate = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        t = time.perf_counter()
        ref = O.jevd(wl.G, wl.J, wl.tol, wl.ordering, want_v=True)
        dt = time.perf_counter() - t
        err = float(np.max(np.abs(lam_gpu - np.sort(ref.lam)) / np.abs(np.sort(ref.lam))))
        gate = {"rel_eig_err_vs_oracle": err, "ok": err <= 1e-12,
                "sweeps_gpu": sweeps, "sweeps_oracle": ref.sweeps}
        cpu = {"value": round(ref.sweeps * work / dt / 1e9, 4), "unit": "GFLOP/s", "cores": 1,
               "kind": "oracle",
               "sample": "one complete solve of the same input (%d sweeps, with V) by the plain "
                         "single-threaded C oracle, %.1f s" % (ref.sweeps, dt)}
    ok = gate is None or gate["ok"]
    out = {
        "metric": "one-sided Jacobi eff. GFLOP/s at rel eig err <=1e-12",
        "value": round(gflops, 2) if ok else None,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "solves_per_s": round(1e3 / ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded)",
        "config": {"workload": wl.name, "m": m, "n": n,
                   "J": "I" if wl.J is None else "+%d/-%d" % (int((wl.J > 0).sum()), int((wl.J < 0).sum())),
                   "ordering": ["row-cyclic", "modulus", "modified modulus"][wl.ordering],
                   "variant": "pointwise", "tol": wl.tol, "sweeps": sweeps, "want_U": True,
                   "want_V": True},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy": gate,
    }
    jevd.jevd_destroy(h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
