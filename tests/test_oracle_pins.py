"""Pins of the oracle against what the paper and the mathematics fix, not
against itself: the paper's worked example, closed forms, matrices with a
known spectrum, brute force on tiny inputs, high-precision library
eigensolvers, invariants and the rotation error bound (A.3).  CPU only.

Each pin is chosen so that a plausible mistake in the oracle (a wrong sign
in a rotation formula, a dropped term, a transposed operand, a wrong
threshold or index) makes at least one of them fail; test_oracle_mutants.py
plants such mistakes and checks exactly that.
"""
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from paper_1008_0201_amd import workloads as W

EPS = W.DBL_EPS          # 2^-52, the eps of the tolerances
U = EPS / 2              # unit roundoff of the appendix's error model
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- helpers
def _mp_matrix_GJGt(G, J):
    """Exact H = G J G^T of an FP64 G, in mpmath (all products and sums exact
    at the working precision used by the callers)."""
    m, n = G.shape
    Gm = [[mpmath.mpf(float(G[i, k])) for k in range(n)] for i in range(m)]
    j = [1 if J is None else int(J[k]) for k in range(n)]
    H = mpmath.matrix(m, m)
    for a in range(m):
        for b in range(a, m):
            s = mpmath.mpf(0)
            for k in range(n):
                s += j[k] * Gm[a][k] * Gm[b][k]
            H[a, b] = s
            H[b, a] = s
    return H


def _eig_mpmath(G, J, dps=90):
    """Eigenvalues of H = G J G^T by mpmath's symmetric eigensolver at high
    precision (a library routine, independent of the Jacobi code here)."""
    with mpmath.workdps(dps):
        H = _mp_matrix_GJGt(G, J)
        E = mpmath.eigsy(H, eigvals_only=True)
        return np.array(sorted(float(e) for e in E))


def _charpoly_roots(G, J):
    """Brute force for tiny n: exact rational H = G J G^T, its characteristic
    polynomial by the Faddeev-LeVerrier recursion, roots by mpmath.polyroots
    at 60+ digits."""
    m, n = G.shape
    Gf = [[Fraction(float(G[i, k])) for k in range(n)] for i in range(m)]
    j = [1 if J is None else int(J[k]) for k in range(n)]
    H = [[sum(j[k] * Gf[a][k] * Gf[b][k] for k in range(n)) for b in range(m)] for a in range(m)]
    # Faddeev-LeVerrier: c_m = 1, M_k = H M_{k-1} + c_{m-k+1} I, c_{m-k} = -tr(H M_k)/k
    c = [Fraction(0)] * (m + 1)
    c[m] = Fraction(1)
    Mk = [[Fraction(0)] * m for _ in range(m)]
    for k in range(1, m + 1):
        HM = [[sum(H[a][t] * Mk[t][b] for t in range(m)) for b in range(m)] for a in range(m)]
        Mk = [[HM[a][b] + (c[m - k + 1] if a == b else 0) for b in range(m)] for a in range(m)]
        HMk = [[sum(H[a][t] * Mk[t][b] for t in range(m)) for b in range(m)] for a in range(m)]
        c[m - k] = -sum(HMk[a][a] for a in range(m)) / k
    coeffs = [c[m - i] for i in range(m + 1)]          # highest degree first
    with mpmath.workdps(80):
        cm = [mpmath.mpf(x.numerator) / x.denominator for x in coeffs]
        roots = mpmath.polyroots(cm, maxsteps=500, extraprec=400)
        return np.array(sorted(float(mpmath.re(r)) for r in roots))


def _rel(a, b):
    a = np.sort(np.asarray(a, dtype=np.float64))
    b = np.sort(np.asarray(b, dtype=np.float64))
    return np.max(np.abs(a - b) / np.abs(b))


def _load_example1():
    sec, data = None, {}
    with open(os.path.join(GOLDEN, "example1.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.isupper() or line.replace("_", "").isupper():
                sec = line
                data[sec] = []
                continue
            data[sec].append(line.split())
    s32 = np.sqrt(3.0) / np.sqrt(2.0)
    s12 = 1.0 / np.sqrt(2.0)
    val = {"s32": s32, "-s32": -s32, "s12": s12, "-s12": -s12}
    conv = lambda t: val[t] if t in val else float(t)  # noqa: E731
    R = np.array([[conv(t) for t in row] for row in data["R"]])
    H = np.array([[float(t) for t in row] for row in data["H"]])
    J = np.array([int(t) for t in data["J"][0]], dtype=np.int8)
    lam = np.array([float(t) for t in data["EIGENVALUES"][0]])
    first = {tuple(int(t) for t in row) for row in data["FIRST_STEP"]}
    return H, R, J, lam, first


# ---------------------------------------------------- the paper's example
def test_example1_fixture_consistent():
    H, R, J, lam, first = _load_example1()
    assert np.allclose(R.T @ np.diag(J) @ R, H, atol=1e-15)
    assert np.allclose(np.linalg.eigvalsh(H), lam, atol=1e-14)


@pytest.mark.parametrize("kind", ["rowcyclic", "modulus", "modmodulus", "block1", "block2fb"])
def test_example1_eigenvalues(orc, kind):
    H, R, J, lam, first = _load_example1()
    G = R.T.copy()
    if kind.startswith("block"):
        res = orc.block_jevd(G, J, tol=4 * EPS, b=1 if kind == "block1" else 2,
                             full_block=kind.endswith("fb"))
    else:
        o = {"rowcyclic": orc.ROWCYCLIC, "modulus": orc.MODULUS, "modmodulus": orc.MODMODULUS}[kind]
        res = orc.jevd(G, J, tol=4 * EPS, ordering_kind=o)
    assert res.status == 0
    assert _rel(res.lam, lam) <= 1e-14
    # inertia: three positive, one negative eigenvalue, as many as +1/-1 in J
    assert np.sum(res.lam > 0) == np.sum(J > 0) == 3
    # eigenvectors of H
    Uv = res.U
    for i in range(4):
        assert np.linalg.norm(H @ Uv[:, i] - res.lam[i] * Uv[:, i]) <= 1e-14 * 3


# -------------------------------------------------------- closed-form 2x2
@pytest.mark.parametrize("m", [2, 3, 7])
@pytest.mark.parametrize("sig", [(1, 1), (1, -1), (-1, 1), (-1, -1)])
@pytest.mark.parametrize("seed", range(6))
def test_two_columns_closed_form(orc, m, sig, seed):
    g = np.random.default_rng(1000 + seed)
    G = g.standard_normal((m, 2)) * (10.0 ** g.uniform(-3, 3, size=2))
    J = np.array(sig, dtype=np.int8)
    # nonzero eigenvalues of G J G^T are those of M = J G^T G (2x2):
    # lambda = tr/2 +- sqrt(tr^2/4 - det), small one as det / big (stable)
    with mpmath.workdps(60):
        g11 = mpmath.fsum(mpmath.mpf(float(x)) ** 2 for x in G[:, 0])
        g22 = mpmath.fsum(mpmath.mpf(float(x)) ** 2 for x in G[:, 1])
        g12 = mpmath.fsum(mpmath.mpf(float(a)) * mpmath.mpf(float(b)) for a, b in G)
        tr = sig[0] * g11 + sig[1] * g22
        det = sig[0] * sig[1] * (g11 * g22 - g12 ** 2)
        disc = mpmath.sqrt(tr ** 2 / 4 - det)
        big = tr / 2 + (disc if tr >= 0 else -disc)
        small = det / big
        truth = sorted([float(big), float(small)])
    # relative accuracy (1.2) scales with the condition of the column-scaled G
    kB = np.linalg.cond(G / np.sqrt(np.sum(G * G, axis=0))[None, :])
    res = orc.jevd(G, J, tol=2 * EPS, ordering_kind=orc.ROWCYCLIC)
    assert res.status == 0
    assert res.sweeps in (2, 3)          # one rotation, then a sweep that rotates nothing
    assert res.rot[0] == 1
    assert _rel(res.lam, truth) <= 16 * U * kB
    # with two columns the modified modulus visits the pair twice a sweep
    res = orc.jevd(G, J, tol=2 * EPS, ordering_kind=orc.MODMODULUS)
    assert res.status == 0 and res.sweeps in (2, 3) and res.rot[0] in (1, 2)
    assert _rel(res.lam, truth) <= 16 * U * kB


# ------------------------------------------------ no rotation is needed
@pytest.mark.parametrize("J", [None, np.array([1, -1, -1, 1, 1, -1], dtype=np.int8)])
def test_orthogonal_columns_untouched(orc, J):
    g = np.random.default_rng(7)
    m, n = 9, 6
    G = np.zeros((m, n))
    support = np.array_split(np.arange(m), n)       # disjoint supports
    for k, rows in enumerate(support):
        G[rows, k] = g.standard_normal(len(rows)) * 10.0 ** g.uniform(-5, 5)
    res = orc.jevd(G, J, ordering_kind=orc.MODMODULUS)
    assert res.status == 0 and res.sweeps == 1 and res.rot[0] == 0
    assert np.array_equal(res.V, np.eye(n))
    assert np.array_equal(res.G, G)
    jj = np.ones(n) if J is None else J.astype(float)
    exact = jj * np.array([sum(x * x for x in G[:, k]) for k in range(n)])
    assert np.array_equal(res.lam, exact)


def test_diagonal_factor(orc):
    d = np.array([3.0, -1e-3, 7e5, 2.0, 1e-8])
    G = np.diag(d)
    J = np.array([1, -1, 1, 1, -1], dtype=np.int8)
    res = orc.jevd(G, J, ordering_kind=orc.MODMODULUS)
    assert res.status == 0 and res.sweeps == 1
    assert np.array_equal(res.lam, J * d * d)


# --------------------------------------------------- known spectra
@pytest.mark.parametrize("n", [16, 41])
def test_known_spectrum_positive_definite(orc, n):
    g = np.random.default_rng(11 + n)
    Q = W.haar_orthogonal(n, g)
    lam = 10.0 ** g.uniform(-2, 0, size=n)
    G = (Q * np.sqrt(lam)[None, :]) @ Q.T          # G G^T = Q diag(lam) Q^T
    kappa = np.sqrt(lam.max() / lam.min())
    for kind in (orc.ROWCYCLIC, orc.MODMODULUS):
        res = orc.jevd(G, None, ordering_kind=kind)
        assert res.status == 0
        assert _rel(res.lam, lam) <= 50 * n * EPS * kappa


def _plane_product_J_orthogonal(n, J, g, count):
    """Product of random plane transforms that preserve J: a rotation on a
    pair of equal signs, a hyperbolic transform with |tanh| <= 0.5 on a pair
    of opposite signs.  Built in long double."""
    V = np.eye(n, dtype=np.longdouble)
    for _ in range(count):
        p, q = sorted(g.choice(n, size=2, replace=False))
        if J[p] == J[q]:
            th = np.longdouble(g.uniform(-np.pi, np.pi))
            c, s = np.cos(th), np.sin(th)
            vp, vq = V[:, p].copy(), V[:, q].copy()
            V[:, p], V[:, q] = c * vp - s * vq, s * vp + c * vq
        else:
            t = np.longdouble(g.uniform(-0.5, 0.5))
            ch = 1 / np.sqrt((1 - t) * (1 + t))
            sh = ch * t
            vp, vq = V[:, p].copy(), V[:, q].copy()
            V[:, p], V[:, q] = ch * vp + sh * vq, sh * vp + ch * vq
    return V


@pytest.mark.parametrize("n", [8, 24])
@pytest.mark.parametrize("seed", [0, 1])
def test_known_spectrum_hyperbolic(orc, n, seed):
    """G = U Sigma V^{-1} with U orthogonal and V J-orthogonal: V^{-1} = J V^T J,
    and H = G J G^T = U (Sigma^2 J) U^T, so lambda_i = j_i sigma_i^2."""
    g = np.random.default_rng(100 * n + seed)
    J = np.ones(n, dtype=np.int8)
    J[g.permutation(n)[: n // 2 - 1]] = -1
    Jl = J.astype(np.longdouble)
    Vt = _plane_product_J_orthogonal(n, J, g, 3 * n)
    Uo = _plane_product_J_orthogonal(n, np.ones(n, dtype=np.int8), g, 4 * n)
    sigma = 10.0 ** g.uniform(-0.5, 0.5, size=n)
    Vinv = (Jl[:, None] * Vt.T) * Jl[None, :]
    G = ((Uo * sigma.astype(np.longdouble)[None, :]) @ Vinv).astype(np.float64)
    truth = J * sigma ** 2
    kappa = np.linalg.cond(G)
    res = orc.jevd(G, J, ordering_kind=orc.MODMODULUS)
    assert res.status == 0
    assert _rel(res.lam, truth) <= 20 * n * EPS * kappa
    assert np.sum(res.lam > 0) == np.sum(J > 0)


# ---------------------------------------------- brute force, tiny n
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("case", ["gauss", "graded", "indef", "indef-graded"])
def test_brute_force_charpoly(orc, n, case):
    g = np.random.default_rng(hash((n, case)) % 2**32)
    G = g.standard_normal((n, n))
    if "graded" in case:
        G = G * (10.0 ** g.uniform(-6, 6, size=n))[None, :]
    J = None
    if "indef" in case:
        J = np.ones(n, dtype=np.int8)
        J[g.permutation(n)[: max(1, n // 2)]] = -1
    truth = _charpoly_roots(G, J)
    # relative accuracy is governed by the condition of the column-scaled G
    B = G / np.sqrt(np.sum(G * G, axis=0))[None, :]
    kappa = np.linalg.cond(B)
    for kind in (orc.ROWCYCLIC, orc.MODMODULUS):
        res = orc.jevd(G, J, tol=n * EPS, ordering_kind=kind)
        assert res.status == 0
        assert _rel(res.lam, truth) <= 64 * n * U * kappa


# -------------------------------------- relative accuracy on graded input
@pytest.mark.parametrize("shape", ["rows", "cols", "cols-indef"])
def test_graded_relative_accuracy(orc, shape):
    n = 24
    if shape == "rows":
        G = W.graded_rows(n, n, k=900, decades=8.0, cond_decades=2.0)
        J = None
        B = G / np.sqrt(np.sum(G * G, axis=1))[:, None]   # row scaling removed
    else:
        G = W.graded_cols(n, n, k=901, decades=8.0)
        J = None
        if shape == "cols-indef":
            J = np.ones(n, dtype=np.int8)
            J[::3] = -1
        B = G / np.sqrt(np.sum(G * G, axis=0))[None, :]
    truth = _eig_mpmath(G, J)
    kappa_s = np.linalg.cond(B)
    H = G @ np.diag(np.ones(n) if J is None else J.astype(float)) @ G.T
    assert np.linalg.cond(H) > 1e12                          # badly conditioned H ...
    res = orc.jevd(G, J, ordering_kind=orc.MODMODULUS)
    assert res.status == 0
    err = _rel(res.lam, truth)
    assert err <= 64 * n * U * kappa_s                      # ... yet relative accuracy (1.2)
    # negative control: an absolute-accuracy dense solver on H is far worse
    dense = np.linalg.eigvalsh(H)
    assert _rel(dense, truth) > 1e3 * max(err, 1e-16)


@pytest.mark.parametrize("n", [40, 64])
def test_fp64_against_quad_precision_run(orc, n):
    """Same method in __float128 and in long double: the FP64 run must agree
    to the relative accuracy bound (1.2)."""
    G = W.graded_cols(n, n, k=902 + n, decades=6.0)
    J = np.ones(n, dtype=np.int8)
    J[n // 3:] = -1
    d = orc.jevd(G, J)
    q = orc.jevd(G, J, tol=n * 1e-32, prec="q")
    ld = orc.jevd(G, J, tol=n * 1e-19, prec="l")
    assert d.status == q.status == ld.status == 0
    B = G / np.sqrt(np.sum(G * G, axis=0))[None, :]
    assert _rel(d.lam, q.lam) <= 64 * n * U * np.linalg.cond(B)
    assert _rel(ld.lam, q.lam) <= 1e-15


# -------------------------------------------------------- invariants
@pytest.mark.parametrize("kind", ["pd", "indef"])
def test_invariants(orc, kind):
    n = 48
    g = np.random.default_rng(5)
    G = g.standard_normal((n + 5, n)) * (10.0 ** g.uniform(-3, 3, size=n))[None, :]
    J = None if kind == "pd" else np.where(g.uniform(size=n) < 0.4, -1, 1).astype(np.int8)
    jj = np.ones(n) if J is None else J.astype(float)
    res = orc.jevd(G, J, ordering_kind=orc.MODMODULUS)
    assert res.status == 0
    # trace: sum lambda_i = tr(G J G^T) = sum_k j_k ||g_k||^2
    tr0 = np.sum(jj * np.sum(G * G, axis=0))
    assert abs(np.sum(res.lam) - tr0) <= 8 * n * U * np.sum(np.abs(res.lam))
    # V^T J V = J (Sec. 1, J-orthogonality of the hyperbolic SVD)
    V = res.V
    vmax = np.max(np.sum(V * V, axis=0))
    assert np.max(np.abs(V.T @ (jj[:, None] * V) - np.diag(jj))) <= 10 * n * EPS * vmax
    # the final iterate is G V (columnwise, relative to the column and ||v||)
    GV = (G.astype(np.longdouble) @ V.astype(np.longdouble)).astype(np.float64)
    colnorm = np.sqrt(np.sum(res.G ** 2, axis=0))
    rowscale = np.sqrt(np.sum((np.abs(G) @ np.abs(V)) ** 2, axis=0))
    assert np.max(np.abs(GV - res.G).sum(axis=0) / rowscale) <= 100 * n * EPS
    assert np.all(colnorm > 0)
    # columns of the final iterate are orthogonal: max |U^T U - I| <= 10 n eps
    Uv = res.U
    assert np.max(np.abs(Uv.T @ Uv - np.eye(n))) <= 10 * n * EPS
    # inertia (Sylvester): as many positive eigenvalues as +1 in J
    assert np.sum(res.lam > 0) == np.sum(jj > 0)


# ---------------------------------------------------- rotation parameters
def _exact_rotation(app, aqq, apq, same):
    with mpmath.workdps(60):
        a, d, b = mpmath.mpf(app), mpmath.mpf(aqq), mpmath.mpf(apq)
        if same:
            z = (d - a) / (2 * b)
            t = (1 if z >= 0 else -1) / (abs(z) + mpmath.sqrt(1 + z * z))
            c = 1 / mpmath.sqrt(1 + t * t)
        else:
            z = (a + d) / (2 * b)
            t = -(1 if z >= 0 else -1) / (abs(z) + mpmath.sqrt(z * z - 1))
            c = 1 / mpmath.sqrt(1 - t * t)
        return c, c * t


@pytest.mark.parametrize("seed", range(200))
def test_rotation_error_bound_A3(orc, seed):
    """(A.3): computed cos and sin have relative error <= 5u/(1-5u)."""
    g = np.random.default_rng(seed)
    app, aqq = 10.0 ** g.uniform(-8, 8, size=2)
    apq = g.uniform(-1, 1) * np.sqrt(app * aqq) * 10.0 ** g.uniform(-6, 0)
    c, s, cl = orc.rotation(app, aqq, apq, True)
    ce, se = _exact_rotation(app, aqq, apq, True)
    bound = 5 * U / (1 - 5 * U)
    assert not cl
    assert abs((c - ce) / ce) <= bound
    assert abs((s - se) / se) <= bound


@pytest.mark.parametrize("seed", range(100))
def test_rotation_annihilates_and_preserves_J(orc, seed):
    """Applying the computed transform exactly to the exact pivot leaves an
    off-diagonal entry of a few ulps; the hyperbolic one keeps Q^T J Q = J."""
    g = np.random.default_rng(10_000 + seed)
    x = g.standard_normal(5) * 10.0 ** g.uniform(-4, 4)
    y = g.standard_normal(5) * 10.0 ** g.uniform(-4, 4)
    app, aqq, apq = float(x @ x), float(y @ y), float(x @ y)
    for same in (True, False):
        c, s, cl = orc.rotation(app, aqq, apq, same)
        with mpmath.workdps(50):
            a, d, b = mpmath.mpf(app), mpmath.mpf(aqq), mpmath.mpf(apq)
            C, S = mpmath.mpf(c), mpmath.mpf(s)
            if same:      # columns (c x - s y, s x + c y)
                off = C * S * (a - d) + (C * C - S * S) * b
                app2, aqq2 = C * C * a - 2 * C * S * b + S * S * d, S * S * a + 2 * C * S * b + C * C * d
                jdev = abs(C * C + S * S - 1)
            else:         # columns (c x + s y, s x + c y)
                off = C * S * (a + d) + (C * C + S * S) * b
                app2, aqq2 = C * C * a + 2 * C * S * b + S * S * d, S * S * a + 2 * C * S * b + C * C * d
                jdev = abs(C * C - S * S - 1)
            rel_off = abs(off) / mpmath.sqrt(app2 * aqq2)
            scale = max(1.0, float(C * C + S * S))
        assert float(rel_off) <= 8 * U * scale
        assert float(jdev) <= 8 * U * scale


def test_rotation_special_cases(orc):
    # app == aqq: zeta = -0 when apq < 0; sgn(-0) is taken as +1, so t = 1
    c, s, cl = orc.rotation(2.0, 2.0, -1.0, True)
    assert c == s == 1 / np.sqrt(2.0) or abs(c - s) == 0
    assert s > 0
    # rounding makes |zeta| <= 1 for a hyperbolic pair: the clamp tanh = -sgn(zeta) 0.9
    c, s, cl = orc.rotation(1.0, 1.0, 1.0, False)
    assert cl and abs(s / c + 0.9) <= 2 * EPS
    c, s, cl = orc.rotation(1.0, 1.0, -1.0, False)
    assert cl and abs(s / c - 0.9) <= 2 * EPS
    # huge |zeta|: t -> 1/(2 zeta) without overflow
    c, s, cl = orc.rotation(1e160, 1.0, 1.0, True)
    assert c == 1.0 and s == 1 / (2 * ((1.0 - 1e160) / 2.0))
    c, s, cl = orc.rotation(1e160, 1.0, 1.0, False)
    assert c == 1.0 and s == -1 / (2 * ((1e160 + 1.0) / 2.0))


# ------------------------------------------------------ status and resume
def test_status_codes(orc):
    G = np.random.default_rng(3).standard_normal((12, 10))
    r = orc.jevd(G, None, max_sweeps=1)
    assert r.status == -3 and r.sweeps == 1                   # not converged
    G2 = G.copy()
    G2[3, 4] = np.nan
    assert orc.jevd(G2, None).status == -2                     # non-finite
    assert orc.jevd(G, np.array([1, 2] + [1] * 8, dtype=np.int8)).status == -1
    assert orc.jevd(G.T.copy(), None).status == -1             # m < n
    # a zero column is never rotated and gives lambda = 0
    G3 = G.copy()
    G3[:, 2] = 0
    r = orc.jevd(G3, None)
    assert r.status == 0 and r.lam[2] == 0 and np.all(r.U[:, 2] == 0)


def test_rank_deficient_hyperbolic_pair_clamps(orc):
    """Two equal columns with opposite signs: a_pp + a_qq = 2|a_pq|, so the
    hyperbolic transform hits the clamp (Sec. 3.2); the problem violates the
    full-rank assumption and does not converge."""
    g = np.random.default_rng(4)
    x = g.standard_normal(6)
    G = np.stack([x, x], axis=1)
    r = orc.jevd(G, np.array([1, -1], dtype=np.int8), max_sweeps=5)
    assert r.extra >= 1
    assert r.status in (-3, 0)


def test_resume_from_iterate(orc):
    G = W.graded_cols(40, 32, k=77, decades=3.0)
    J = np.ones(32, dtype=np.int8)
    J[10:] = -1
    full = orc.jevd(G, J)
    part = orc.jevd(G, J, max_sweeps=3)
    assert part.status == -3 and part.sweeps == 3
    rest = orc.jevd(part.G, J, V0=part.V)
    assert rest.status == 0
    assert np.array_equal(rest.lam, full.lam)                 # same arithmetic, same order
    assert np.array_equal(rest.V, full.V)
    assert part.sweeps + rest.sweeps == full.sweeps


# ------------------------------------------------------------ block oracle
@pytest.mark.parametrize("n,b", [(32, 4), (48, 8), (30, 4), (37, 5), (64, 16)])
@pytest.mark.parametrize("full_block", [False, True])
@pytest.mark.parametrize("indef", [False, True])
def test_block_oracle_matches_definition(orc, n, b, full_block, indef):
    G = W.graded_cols(n + 3, n, k=500 + n + b, decades=4.0)
    J = None
    if indef:
        J = np.ones(n, dtype=np.int8)
        J[n // 2:] = -1
    truth = _eig_mpmath(G, J, dps=60) if n <= 40 else orc.jevd(G, J, tol=n * 1e-32, prec="q").lam
    res = orc.block_jevd(G, J, b=b, full_block=full_block)
    assert res.status == 0
    # a full-column-rank, modestly conditioned pivot has a positive definite
    # Gram, so its Cholesky factorisation never breaks down (Sec. 3.2)
    assert res.extra == 0
    B = G / np.sqrt(np.sum(G * G, axis=0))[None, :]
    nonzero = truth[np.abs(truth) > 0] if n <= 40 else truth
    lam = np.sort(res.lam)
    if n <= 40:     # H is (n+3)x(n+3) of rank n: drop its 3 zero eigenvalues
        idx = np.argsort(np.abs(truth))[3:]
        nonzero = truth[idx]
    assert _rel(lam, nonzero) <= 64 * n * U * np.linalg.cond(B)
    jj = np.ones(n) if J is None else J.astype(float)
    V = res.V
    vmax = np.max(np.sum(V * V, axis=0))
    assert np.max(np.abs(V.T @ (jj[:, None] * V) - np.diag(jj))) <= 10 * n * EPS * vmax
    Uv = res.U
    assert np.max(np.abs(Uv.T @ Uv - np.eye(n))) <= 10 * n * EPS


def test_block_single_pivot_is_whole_matrix(orc):
    """With two blocks the only pivot is the whole matrix; full block then
    diagonalises it in the first step, and the second sweep rotates nothing
    (or very little)."""
    n = 20
    G = W.graded_cols(n, n, k=601, decades=2.0)
    res = orc.block_jevd(G, None, b=n // 2, full_block=True)
    assert res.status == 0 and res.extra == 0
    assert res.sweeps <= 3
    truth = _eig_mpmath(G, None, dps=60)
    assert _rel(res.lam, truth) <= 1e-13


# ------------------------------------- threaded block oracle and step sample
@pytest.mark.parametrize("n,b,full_block,sign_pivot,indef",
                         [(96, 8, False, False, False), (96, 8, True, False, True),
                          (100, 8, False, True, True), (70, 6, True, True, False)])
def test_block_oracle_threaded_is_sequential(orc, n, b, full_block, sign_pivot, indef):
    """The threaded driver (the pivots of a step on several threads, used for
    the large cached solves) is bit for bit the sequential oracle, which the
    pins above tie to the definition: the pivots of a step are disjoint
    (Sec. 3), so only the order in which they run differs.  Uneven widths
    (n = 100, b = 8 and n = 70, b = 6) included."""
    if indef:
        wl = W.graded_hyperbolic(n, k=50 + n, grade=2.0)
        G, J = wl.G, wl.J
    else:
        G, J = W.graded_cols(n, n, k=60 + n, decades=3.0), None
    seq = orc.block_jevd(G, J, b=b, full_block=full_block, sign_pivot=sign_pivot)
    par = orc.block_jevd(G, J, b=b, full_block=full_block, sign_pivot=sign_pivot, nthreads=4)
    assert seq.status == par.status == 0
    assert seq.sweeps == par.sweeps and np.array_equal(seq.rot, par.rot)
    assert np.array_equal(seq.G, par.G) and np.array_equal(seq.V, par.V)
    assert np.array_equal(seq.lam, par.lam) and np.array_equal(seq.J, par.J)
    assert seq.extra == par.extra


@pytest.mark.parametrize("full_block,sign_pivot,nthreads", [(False, False, 1), (True, False, 3),
                                                            (False, True, 1), (True, True, 2)])
def test_block_steps_sample_is_the_first_sweep(orc, full_block, sign_pivot, nthreads):
    """The bounded sample that the benchmark times (orc_block_steps): all N
    steps of it are exactly one sweep of the block oracle (same G, bit for
    bit), and its first k steps are a prefix of that sweep (running the
    remaining steps would be the same computation)."""
    n, b = 64, 8
    wl = W.graded_hyperbolic(n, k=71, grade=2.0)
    J = wl.J if sign_pivot or full_block else None
    one = orc.block_jevd(wl.G, J, b=b, full_block=full_block, sign_pivot=sign_pivot,
                         max_sweeps=1, want_v=False)
    assert one.status in (0, -3)
    N = 2 * ((n + 2 * b - 1) // (2 * b))
    st, Gs = orc.block_steps(wl.G, J, b=b, full_block=full_block, steps=N,
                             sign_pivot=sign_pivot, nthreads=nthreads)
    assert st == one.status
    assert np.array_equal(Gs, one.G)
    st3, G3 = orc.block_steps(wl.G, J, b=b, full_block=full_block, steps=3,
                              sign_pivot=sign_pivot, nthreads=nthreads)
    st3s, G3s = orc.block_steps(wl.G, J, b=b, full_block=full_block, steps=3,
                                sign_pivot=sign_pivot, nthreads=1)
    assert np.array_equal(G3, G3s) and not np.array_equal(G3, wl.G)
