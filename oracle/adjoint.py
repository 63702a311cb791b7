"""Oracle of the adjoint (reverse-mode derivative) of the eigen-decomposition
that one-sided Jacobi delivers, for the loss
    L(G) = sum_i w_i lambda_i + <C, U>.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg may call this module; the product path never imports it, and
it imports nothing of the product.  Plain numpy in FP64.

Setting (Sec. 1 and Sec. 2.1).  The solver factors H = G J G^T (G m x n,
m >= n, full column rank, J = diag(+-1)) through a J-orthogonal V
(V^T J V = J) with G V = U Sigma: the columns of U are orthonormal
eigenvectors of H and lambda_i = j_i sigma_i^2 its nonzero eigenvalues.

Canonical outputs.  The column order and the column signs that the
iteration leaves are a by-product of its rotation sequence; the loss is
defined on a canonical form instead (eigenpairs sorted by decreasing
lambda, ties by position; each u_i signed so that its entry of largest
magnitude, the first such, is positive; the columns of V and the signs j_i
permuted and signed alike).  Both choices are locally constant in G for a
simple spectrum, so they do not enter the derivative.

Adjoint (first-order perturbation theory of a symmetric matrix with simple
nonzero eigenvalues):
  d lambda_i = u_i^T dH u_i,
  d u_i      = sum_{k != i} u_k u_k^T dH u_i / (lambda_i - lambda_k)
               + (I - U U^T) dH u_i / lambda_i      (the m - n zero eigenvalues),
  dH         = dG J G^T + G J dG^T.
Hence <dL/dH, dH> = <X, dH> with
  X = U diag(w) U^T + U (F o U^T C) U^T + (I - U U^T) C Lambda^{-1} U^T,
  F_ki = 1 / (lambda_i - lambda_k) (k != i), F_ii = 0,
and, pulled back through dH, dL/dG = (X + X^T) G J.  Two exact zeros are
left out rather than formed: the transpose of the last term of X multiplies
(I - U U^T) G, which vanishes because the columns of G lie in the range of U
(full column rank), and for m = n that term is empty.  Formed in floating
point they are rounding noise of size eps |G| / min |lambda_i|.
"""
import numpy as np


def canonical(lam, U, V, J=None):
    """Canonical form of one solver output (see the module docstring).
    lam (n), U (m x n), V (n x n or None), J (n signs of the input columns
    or None).  Returns (lam, U, V, j) with j_i the sign of the i-th
    canonical eigenvalue's column (+1 for J = I)."""
    lam = np.asarray(lam, dtype=np.float64)
    n = lam.shape[0]
    order = np.argsort(-lam, kind="stable")
    lam_c = lam[order]
    U_c = np.array(U, dtype=np.float64)[:, order]
    big = np.argmax(np.abs(U_c), axis=0)
    s = np.sign(U_c[big, np.arange(n)])
    s[s == 0] = 1.0
    U_c = U_c * s[None, :]
    V_c = None if V is None else np.array(V, dtype=np.float64)[:, order] * s[None, :]
    j = np.ones(n) if J is None else np.asarray(J, dtype=np.float64)[order]
    return lam_c, U_c, V_c, j


def loss(lam, U, w, C):
    """L = sum_i w_i lambda_i + <C, U> on canonical outputs."""
    out = 0.0
    if w is not None:
        out += float(np.dot(w, lam))
    if C is not None:
        out += float(np.sum(C * U))
    return out


def adjoint(G, J, lam, U, w=None, C=None):
    """dL/dG for canonical (lam, U) of H = G J G^T (J None: identity)."""
    G = np.asarray(G, dtype=np.float64)
    m, n = G.shape
    Jd = np.ones(n) if J is None else np.asarray(J, dtype=np.float64)
    X = np.zeros((m, m))
    if w is not None:
        X += U @ np.diag(w) @ U.T
    if C is not None:
        F = np.zeros((n, n))
        for k in range(n):
            for i in range(n):
                if k != i:
                    F[k, i] = 1.0 / (lam[i] - lam[k])
        X += U @ (F * (U.T @ C)) @ U.T
    out = (X + X.T) @ G @ np.diag(Jd)
    if C is not None and m > n:
        out += (np.eye(m) - U @ U.T) @ C @ np.diag(1.0 / lam) @ U.T @ G @ np.diag(Jd)
    return out
