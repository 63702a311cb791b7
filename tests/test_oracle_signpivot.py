"""Pins of the oracle's sign-pivoted Cholesky (Alg. 3.3) and of the block
solves that use it (HBSC / HFSC, Alg. 3.4), against facts that do not come
from the oracle: LAPACK's Cholesky with diagonal pivoting (dpstrf, through
scipy) for the J = I case, for A_11 and for the Schur complement S formed
here with numpy; the Gram identity P^T A P = R_S^T R_S; Sylvester's law of
inertia; and the exact spectra / binary128 solves used for the other block
pins.  CPU only."""
import numpy as np
import pytest
import scipy.linalg.lapack as lapack

from paper_1008_0201_amd import workloads as W

EPS = W.DBL_EPS


def dpstrf_upper(A):
    """(R, perm) with A[perm][:, perm] = R^T R, by LAPACK."""
    c, piv, rank, info = lapack.dpstrf(np.array(A, order="F"), lower=0)
    assert info == 0 and rank == A.shape[0]
    return np.triu(c), piv - 1


def gram_case(w, npos, seed, decades=2.0):
    g = np.random.default_rng(seed)
    B = g.standard_normal((3 * w, w)) * (10.0 ** g.uniform(-decades, decades, size=w))[None, :]
    A = B.T @ B
    JP = np.ones(w, dtype=np.int8)
    JP[g.permutation(w)[: w - npos]] = -1
    return A, JP


@pytest.mark.parametrize("w", [1, 5, 16, 33])
def test_identity_signature_is_lapack_pivoted_cholesky(orc, w):
    A, JP = gram_case(w, w, 10 + w)
    st, RS, perm, npos = orc.sp_cholesky(A, JP)
    R, piv = dpstrf_upper(A)
    assert st == 0 and npos == w
    assert list(perm) == list(piv)
    assert np.max(np.abs(RS - R)) <= 64 * EPS * np.max(np.abs(R))


@pytest.mark.parametrize("w", [1, 6, 17])
def test_negative_signature_is_reversed_pivoted_cholesky(orc, w):
    """J_P = -I: the pivoted factor with its columns (and P) reversed."""
    A, JP = gram_case(w, 0, 20 + w)
    st, RS, perm, npos = orc.sp_cholesky(A, JP)
    R, piv = dpstrf_upper(A)
    assert st == 0 and npos == 0
    assert list(perm) == list(piv[::-1])
    assert np.max(np.abs(RS - R[:, ::-1])) <= 64 * EPS * np.max(np.abs(R))


@pytest.mark.parametrize("w,npos", [(8, 3), (16, 9), (32, 16), (7, 1), (7, 6)])
def test_mixed_signature_blocks(orc, w, npos):
    """(3.5)-(3.7): R11 and P1 from A11, R12 from R11^T R12 = P1^T A12, R22
    and P2 from S = A22 - R12^T R12, then the second block column reversed."""
    A, JP = gram_case(w, npos, 30 + w + npos)
    st, RS, perm, k = orc.sp_cholesky(A, JP)
    assert st == 0 and k == npos
    pos = np.flatnonzero(JP > 0)
    neg = np.flatnonzero(JP < 0)
    R11, p1 = dpstrf_upper(A[np.ix_(pos, pos)])
    R12 = np.linalg.solve(R11.T, A[np.ix_(pos[p1], neg)])
    S = A[np.ix_(neg, neg)] - R12.T @ R12
    R22, p2 = dpstrf_upper(S)
    want = np.zeros((w, w))
    want[:npos, :npos] = R11
    want[:npos, npos:] = (R12[:, p2])[:, ::-1]
    want[npos:, npos:] = R22[:, ::-1]
    scale = np.max(np.abs(want))
    assert list(perm[:npos]) == list(pos[p1])
    assert list(perm[npos:]) == list(neg[p2][::-1])
    assert np.max(np.abs(RS - want)) <= 1e3 * EPS * scale
    # the Gram identity and the signs of the permuted positions
    P = np.eye(w)[:, perm]
    assert np.max(np.abs(RS.T @ RS - P.T @ A @ P)) <= 64 * w * EPS * np.max(np.abs(A))
    assert np.all(JP[perm][:npos] > 0) and np.all(JP[perm][npos:] < 0)


def test_breakdown_is_reported(orc):
    A, JP = gram_case(6, 3, 5)
    A[:, 2] = 0.0
    A[2, :] = 0.0
    st, RS, perm, npos = orc.sp_cholesky(A, JP)
    assert st == 1


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("full_block", [False, True])
@pytest.mark.parametrize("n,b", [(64, 8), (96, 12), (100, 10)])
def test_sign_pivoted_block_solve(orc, n, b, full_block, mixed):
    """HBSC / HFSC reach the eigenvalues of the binary128 pointwise solve
    within the double oracle's own accuracy, keep the inertia of J, and
    their V satisfies V^T J V = J_final with J_final = sign(lambda).  With
    J sorted (+ first) the pivoting never moves a sign between columns; with
    a mixed J it does."""
    wl = W.graded_hyperbolic(n, k=400 + n, grade=1.5)
    if mixed:
        wl.J = W.random_signature(n, np.random.default_rng(n))
    r = orc.block_jevd(wl.G, wl.J, wl.tol, b=b, full_block=full_block, sign_pivot=True)
    assert r.status == 0
    q = orc.jevd(wl.G, wl.J, wl.tol, orc.MODMODULUS, want_v=False, prec="q")
    d = orc.jevd(wl.G, wl.J, wl.tol, orc.MODMODULUS, want_v=False)
    rel = lambda a, b_: float(np.max(np.abs(np.sort(a) - np.sort(b_)) / np.abs(np.sort(b_))))
    assert rel(r.lam, q.lam) <= max(1e-12, 8 * rel(d.lam, q.lam))
    assert np.all(np.sign(r.lam) == r.J)
    assert int((r.J > 0).sum()) == int((wl.J > 0).sum())           # inertia
    V = r.V
    vmax = np.max(np.sum(V * V, axis=0))
    jin = wl.J.astype(float)
    assert np.max(np.abs(V.T @ (jin[:, None] * V) - np.diag(r.J.astype(float)))) <= 10 * n * EPS * vmax
    GV = (wl.G.astype(np.longdouble) @ V.astype(np.longdouble)).astype(np.float64)
    scale = np.sqrt(np.sum((np.abs(wl.G) @ np.abs(V)) ** 2, axis=0))
    assert np.max(np.abs(GV - r.G).sum(axis=0) / scale) <= 100 * n * EPS


def test_sign_pivoted_known_spectrum_trig(orc):
    """J = I: the diagonally pivoted variant on Q diag(lambda) Q^T factors."""
    g = np.random.default_rng(77)
    n = 64
    Q = W.haar_orthogonal(n, g)
    s = np.sort(10.0 ** g.uniform(-3, 0, size=n))
    G = (Q * np.sqrt(s)[None, :]) @ W.haar_orthogonal(n, g).T
    r = orc.block_jevd(G, None, None, b=8, full_block=True, sign_pivot=True)
    assert r.status == 0
    assert np.max(np.abs(np.sort(r.lam) - s) / s) <= 1e-12
    assert np.all(r.J == 1)
