"""Host tests of the accuracy gate (oracle/gates.py): the figures it uses
and its decision rule.  CPU only."""
import numpy as np

from oracle import gates


def test_kappa_of_scaled_columns():
    # column scaling removed: a diagonal factor has kappa 1 after scaling
    assert abs(gates.kappa_colscaled(np.diag([1e-8, 1.0, 1e8])) - 1.0) < 1e-12
    # zero columns are ignored
    G = np.array([[1.0, 0.0, 1.0], [0.0, 0.0, 1.0]])
    B = np.array([[1.0, 2 ** -0.5], [0.0, 2 ** -0.5]])
    assert abs(gates.kappa_colscaled(G) - np.linalg.cond(B)) < 1e-12
    assert abs(gates.bound_12(np.eye(4)) - 64 * 4 * 2.0 ** -53) < 1e-30


def test_rel_err_sorts_and_handles_zero():
    assert gates.rel_err([3.0, 1.0, 0.0], [0.0, 1.0, 3.0]) == 0.0
    assert abs(gates.rel_err([1.0, 2.0 + 2e-12], [2.0, 1.0]) - 1e-12) < 1e-15


def test_gate_rule():
    G = np.eye(3)
    lam = np.array([1.0, 2.0, 3.0])
    ok = gates.eig_gate(G, lam, lam)
    assert ok["ok"] and "rel_eig_err_vs_high_precision" not in ok
    off = lam * (1 + 1e-11)
    # no high-precision run available: the FP64 check decides
    assert not gates.eig_gate(G, off, lam)["ok"]
    bnd = gates.bound_12(G)
    # the fallback accepts an error within the bound against the truth ...
    r = gates.eig_gate(G, lam * (1 + 0.5 * bnd), lam * (1 + 1e-11), truth=lambda: lam)
    assert r["ok"] and r["rel_eig_err_vs_high_precision"] <= bnd
    # ... and rejects one beyond it
    r = gates.eig_gate(G, lam * (1 + 4 * bnd), lam * (1 + 1e-11), truth=lambda: lam)
    assert not r["ok"]
