"""Accuracy gates of the parity checks.

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's accuracy
gate; the product path never imports it.

The eigenvalue gate is fixed in advance:

1. The GPU eigenvalues must lie within a relative error of 1e-12 of the FP64
   oracle's, after sorting both (the rel. eig. err of the metric).
2. Two correct FP64 executions of the method that differ only in their
   rounding order can lie further apart than that on an ill-conditioned
   input: each is within the relative accuracy bound (1.2) of the exact
   eigenvalues, and that bound grows with the condition of the scaled
   factor.  Where check 1 fails, the GPU eigenvalues are compared with a
   high-precision run of the oracle (80-bit or binary128, whose own error is
   smaller by a factor of 2^11 or more) and must meet the bound
       max_i |lambda_i - lambda_i^true| / |lambda_i^true|
           <= 64 n u kappa_2(B),   u = 2^-53,
   with B the factor with its columns scaled to unit norm (the one-sided
   method transforms columns; Sec. 1, (1.2)).  The constant 64 is the one the
   oracle's own pins use for the same bound.
"""
import numpy as np

U = 2.0 ** -53
REL_TOL = 1e-12


def rel_err(a, b):
    """max_i |a_i - b_i| / |b_i| after sorting both (b_i = 0 counts as 1)."""
    a, b = np.sort(np.asarray(a, dtype=np.float64)), np.sort(np.asarray(b, dtype=np.float64))
    den = np.where(b != 0, np.abs(b), 1.0)
    return float(np.max(np.abs(a - b) / den))


def kappa_colscaled(G):
    """kappa_2 of G with its nonzero columns scaled to unit norm."""
    G = np.asarray(G, dtype=np.float64)
    nrm = np.sqrt(np.sum(G * G, axis=0))
    keep = nrm > 0
    B = G[:, keep] / nrm[keep][None, :]
    return float(np.linalg.cond(B))


def bound_12(G):
    """The a-priori relative error bound 64 n u kappa_2(B) of the gate."""
    n = np.asarray(G).shape[1]
    return 64.0 * n * U * kappa_colscaled(G)


def eig_gate(G, lam_gpu, lam_fp64, truth=None, kappa=None):
    """Applies the gate.  lam_fp64: the FP64 oracle's eigenvalues; truth: a
    callable returning a high-precision oracle run's eigenvalues (called
    only when check 1 fails); kappa: kappa_colscaled(G) if already known.
    Returns a dict with 'ok' and the figures."""
    err = rel_err(lam_gpu, lam_fp64)
    out = {"rel_eig_err_vs_oracle": err, "limit": REL_TOL, "ok": err <= REL_TOL}
    if out["ok"] or truth is None:
        return out
    lam_true = truth()
    e_gpu = rel_err(lam_gpu, lam_true)
    n = np.asarray(G).shape[1]
    bnd = 64.0 * n * U * (kappa if kappa is not None else kappa_colscaled(G))
    out.update({"rel_eig_err_vs_high_precision": e_gpu,
                "fp64_oracle_err_vs_high_precision": rel_err(lam_fp64, lam_true),
                "bound_64_n_u_kappa": bnd, "ok": e_gpu <= bnd})
    return out
