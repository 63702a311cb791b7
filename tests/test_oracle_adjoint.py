"""Pins of the adjoint oracle (oracle/adjoint.py) against facts that do not
come from its own formula: central finite differences of the loss computed
with the oracle's forward solve, the textbook singular-value derivative
d sigma_i / dG = u_i v_i^T through numpy's SVD, and three invariances of
the loss (C along U; scaling G; J-orthogonal mixing of the columns of G).
A mutation check plants plausible mistakes in a copy of the oracle and
requires a pin to fail.  CPU only."""
import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_adjoint(path=None):
    path = path or os.path.join(ROOT, "oracle", "adjoint.py")
    spec = importlib.util.spec_from_file_location("adjoint_under_test", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def forward(orc, A, G, J, prec="l"):
    """Canonical (lam, U, V, j) of the oracle's solve of H = G J G^T."""
    r = orc.jevd(G, J, None, orc.MODMODULUS, want_v=True, prec=prec)
    assert r.status == 0
    return A.canonical(r.lam, r.U, r.V, J)


def separated_case(kind, m, n, seed):
    """G with a simple, well separated spectrum (min |lambda_i - lambda_k| /
    max |lambda| >= 0.02)."""
    g = np.random.default_rng(seed)
    for _ in range(200):
        if kind == "trig":
            Q1 = np.linalg.qr(g.standard_normal((m, m)))[0][:, :n]
            Q2 = np.linalg.qr(g.standard_normal((n, n)))[0]
            s = g.permutation(np.linspace(1.0, 3.0, n))
            G = (Q1 * s[None, :]) @ Q2.T
            J = None
        else:
            G = g.standard_normal((m, n)) * (10.0 ** g.uniform(-0.4, 0.4, size=n))[None, :]
            J = np.ones(n, dtype=np.int8)
            J[g.permutation(n)[: n // 2]] = -1
        jj = np.ones(n) if J is None else J.astype(float)
        lam = np.linalg.eigvalsh(G @ np.diag(jj) @ G.T)
        lam = lam[np.argsort(-np.abs(lam))][:n]
        gaps = np.abs(lam[:, None] - lam[None, :]) + np.eye(n) * 1e300
        if gaps.min() >= 0.02 * np.abs(lam).max():
            return G, J, g
    raise AssertionError("no separated case found")


CASES = [("trig", 6, 6, 1), ("trig", 9, 7, 2), ("hyp", 6, 6, 3), ("hyp", 10, 8, 4),
         ("hyp", 12, 12, 5)]


def fd_check(A, orc, G, J, w, C, g, ndir=4, h=1e-5, rtol=2e-7):
    lam, U, V, j = forward(orc, A, G, J)
    grad = A.adjoint(G, J, lam, U, w, C)
    for _ in range(ndir):
        E = g.standard_normal(G.shape)
        lp = A.loss(*forward(orc, A, G + h * E, J)[:2], w, C)
        lm = A.loss(*forward(orc, A, G - h * E, J)[:2], w, C)
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(grad * E))
        scale = np.linalg.norm(grad) * np.linalg.norm(E)
        assert abs(fd - an) <= rtol * scale, (fd, an)


@pytest.mark.parametrize("kind,m,n,seed", CASES)
def test_adjoint_matches_finite_differences(orc, kind, m, n, seed):
    A = load_adjoint()
    G, J, g = separated_case(kind, m, n, seed)
    w = g.standard_normal(n)
    C = g.standard_normal((m, n))
    fd_check(A, orc, G, J, w, C, g)
    fd_check(A, orc, G, J, None, C, g, ndir=2)
    fd_check(A, orc, G, J, w, None, g, ndir=2)


@pytest.mark.parametrize("m,n", [(5, 5), (8, 6)])
def test_eigenvalue_part_matches_textbook_svd_derivative(orc, m, n):
    """J = I: lambda_i = sigma_i^2 and d sigma_i / dG = u_i v_i^T, so the
    w-part of the adjoint is sum_i 2 w_i sigma_i u_i v_i^T (numpy's SVD)."""
    A = load_adjoint()
    G, J, g = separated_case("trig", m, n, 11 + n)
    w = g.standard_normal(n)
    lam, U, V, j = forward(orc, A, G, None, prec="d")
    got = A.adjoint(G, None, lam, U, w, None)
    Us, s, Vt = np.linalg.svd(G, full_matrices=False)
    # pair numpy's singular values with the oracle's eigenvalues by value
    ws = np.array([w[np.argmin(np.abs(lam - si * si))] for si in s])
    want = sum(2 * ws[i] * s[i] * np.outer(Us[:, i], Vt[i, :]) for i in range(n))
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("kind,m,n,seed", CASES)
def test_invariances(orc, kind, m, n, seed):
    A = load_adjoint()
    G, J, g = separated_case(kind, m, n, seed)
    lam, U, V, j = forward(orc, A, G, J, prec="d")
    jj = np.ones(n) if J is None else J.astype(float)
    w = g.standard_normal(n)
    C = g.standard_normal((m, n))
    # C along the columns of U: <C, U> = sum c_i is constant, so no gradient
    c = g.standard_normal(n)
    gz = A.adjoint(G, J, lam, U, None, U * c[None, :])
    assert np.max(np.abs(gz)) <= 1e-12 * np.max(np.abs(c)) * np.max(np.abs(G))
    # scaling: lambda(a G) = a^2 lambda, U(a G) = U, so <dL/dG, G> = 2 w.lambda
    grad = A.adjoint(G, J, lam, U, w, C)
    assert abs(np.sum(grad * G) - 2 * np.dot(w, lam)) <= 1e-10 * np.abs(w).sum() * np.abs(lam).max()
    # J-orthogonal mixing: H(G Q) = H(G) for Q^T J Q = J, whose tangent at I is
    # A = J S with S antisymmetric, so <dL/dG, G J S> = 0
    S = g.standard_normal((n, n))
    S = S - S.T
    t = np.sum(grad * (G @ np.diag(jj) @ S))
    assert abs(t) <= 1e-10 * np.linalg.norm(grad) * np.linalg.norm(G @ S)


MUTANTS = {
    "transpose-term-dropped": ("out = (X + X.T) @ G @ np.diag(Jd)", "out = 2 * X @ G @ np.diag(Jd)"),
    "gap-sign-flipped": ("F[k, i] = 1.0 / (lam[i] - lam[k])", "F[k, i] = 1.0 / (lam[k] - lam[i])"),
    "complement-dropped": ("out += (np.eye(m) - U @ U.T) @ C @ np.diag(1.0 / lam) @ U.T @ G @ np.diag(Jd)",
                           "pass"),
    "signature-dropped": ("out = (X + X.T) @ G @ np.diag(Jd)", "out = (X + X.T) @ G"),
    "operands-transposed": ("X += U @ (F * (U.T @ C)) @ U.T", "X += U @ (F * (C.T @ U)) @ U.T"),
    "weights-halved": ("X += U @ np.diag(w) @ U.T", "X += 0.5 * U @ np.diag(w) @ U.T"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_adjoint_mistake(orc, tmp_path, name):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "adjoint.py")).read()
    assert src.count(old) == 1
    path = tmp_path / "adjoint_mutant.py"
    path.write_text(src.replace(old, new))
    A = load_adjoint(str(path))
    failed = False
    for kind, m, n, seed in CASES:
        G, J, g = separated_case(kind, m, n, seed)
        w = g.standard_normal(n)
        C = g.standard_normal((m, n))
        try:
            fd_check(A, orc, G, J, w, C, g, ndir=2)
        except AssertionError:
            failed = True
            break
    assert failed, "pins did not catch mutant %s" % name
