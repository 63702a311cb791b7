"""Seeded synthetic inputs (G, J, tol, ordering) for the one-sided Jacobi solver.

This module holds input generation only, none of the method's arithmetic:
it is shared by the tests, the benchmark, the smoke check and the oracle
side, and imports neither the GPU binding nor the oracle.

The paper measured on symmetric matrices with entries uniform in [-5, 5],
factored by a Bunch-Parlett decomposition (Sec. 4); neither those matrices
nor that factorisation code is available, so the generators below produce
factors G (and signatures J) directly, with the shapes, scalings and sign
mixes of the workloads the solver is quoted on.  Each workload fixes its own
seed (10080200 + k), uses numpy's PCG64 generator and FP64, so that the
oracle and the GPU consume identical bytes.

Matrices are returned Fortran-ordered (column-major), as the library wants.
"""
import numpy as np

SEED_BASE = 10080200
DBL_EPS = float(np.finfo(np.float64).eps)   # 2**-52

ROWCYCLIC, MODULUS, MODMODULUS = 0, 1, 2


def rng(k):
    return np.random.Generator(np.random.PCG64(SEED_BASE + k))


def haar_orthogonal(n, g):
    """Haar-distributed orthogonal matrix: QR of an N(0,1) matrix with the
    column signs fixed by sign(diag(R))."""
    A = g.standard_normal((n, n))
    Q, R = np.linalg.qr(A)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


class Workload:
    """One solver input: G (m x n, F-order), J (int8 or None), tol, ordering."""

    def __init__(self, name, G, J, tol, ordering, note=""):
        self.name = name
        self.G = np.asfortranarray(G, dtype=np.float64)
        self.J = None if J is None else np.ascontiguousarray(J, dtype=np.int8)
        self.tol = float(tol)
        self.ordering = ordering
        self.note = note

    @property
    def m(self):
        return self.G.shape[0]

    @property
    def n(self):
        return self.G.shape[1]


def spd_gaussian(n=64, k=0, ordering=ROWCYCLIC, tol_factor=None):
    """Positive definite case H = G G^T with G ~ N(0,1) (n x n), J = I.
    At n = 64 with the row-cyclic ordering and tol = 64 eps this is the
    small single-matrix workload."""
    g = rng(k)
    G = g.standard_normal((n, n))
    tol = (tol_factor if tol_factor is not None else n) * DBL_EPS
    return Workload("spd-gaussian-n%d" % n, G, None, tol, ordering)


def graded_hyperbolic(n=1024, k=1, m=None, grade=3.0, ordering=MODMODULUS):
    """Indefinite case H = G J G^T: G = B diag(10^u), B ~ N(0,1) (m x n),
    u_j ~ U(-grade, grade); J = diag(+1 x n/2, -1 x n - n/2); tol = n eps.
    At n = 1024 this is the hyperbolic workload of the benchmark."""
    g = rng(k)
    m = n if m is None else m
    B = g.standard_normal((m, n))
    u = g.uniform(-grade, grade, size=n)
    G = B * (10.0 ** u)[None, :]
    J = np.ones(n, dtype=np.int8)
    J[n // 2:] = -1
    return Workload("hyperbolic-graded-n%d" % n, G, J, n * DBL_EPS, ordering)


# The QR and the product of the row-graded recipe below run in OpenBLAS, whose
# results depend on the CPU kernel it picks and on its thread count.  So that
# every machine produces the same bytes (eigenvalues of an input can then be
# computed once, on any machine, and looked up by the input's SHA-256), that
# recipe runs in a child process with both fixed: the AVX2 (Haswell) kernels,
# which every x86-64 host here has, and 8 threads.  OpenBLAS uses no more
# threads than the CPUs the process may run on, so a process restricted to
# fewer than 8 CPUs (an affinity mask) gets other bytes; it is warned, and
# lookups of cached results by SHA-256 then report that the input differs.
FIXED_BLAS_ENV = {"OPENBLAS_CORETYPE": "Haswell", "OPENBLAS_NUM_THREADS": "8",
                  "OMP_NUM_THREADS": "8"}


def _graded_spd_factor_here(n, k, lam_decades, row_decades):
    g = rng(k)
    Q = haar_orthogonal(n, g)
    lam = 10.0 ** g.uniform(-lam_decades, 0.0, size=n)
    d = 10.0 ** g.uniform(-row_decades, row_decades, size=n)
    A = (Q * lam[None, :]) @ Q.T
    return d[:, None] * A


def _graded_spd_factor_fixed_blas(n, k, lam_decades, row_decades):
    """_graded_spd_factor_here in a child process with FIXED_BLAS_ENV."""
    import os
    import subprocess
    import sys
    import tempfile
    here = os.path.dirname(os.path.abspath(__file__))
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    if ncpu < int(FIXED_BLAS_ENV["OPENBLAS_NUM_THREADS"]):
        print("workloads: only %d CPUs allowed; the generated factor will differ from the "
              "one made with %s threads" % (ncpu, FIXED_BLAS_ENV["OPENBLAS_NUM_THREADS"]),
              file=sys.stderr)
    env = dict(os.environ)
    env.update(FIXED_BLAS_ENV)
    with tempfile.TemporaryDirectory() as td:
        out = os.path.join(td, "G.npy")
        code = ("import sys, numpy as np; sys.path.insert(0, %r); "
                "from paper_1008_0201_amd import workloads as W; "
                "np.save(%r, W._graded_spd_factor_here(%d, %d, %r, %r))"
                % (os.path.dirname(here), out, n, k, float(lam_decades), float(row_decades)))
        subprocess.run([sys.executable, "-c", code], env=env, check=True)
        return np.load(out)


def graded_spd_known_factor(n=8192, k=2, lam_decades=6.0, row_decades=4.0,
                            ordering=MODMODULUS):
    """Positive definite, row-graded: G = D Q diag(lam) Q^T with Q Haar,
    lam_k = 10^U(-lam_decades, 0) and D = diag(10^U(-row_decades, row_decades));
    J = I, tol = n eps.  At n = 8192 this is the block-sweep workload.  The
    same bytes on every machine (FIXED_BLAS_ENV)."""
    G = _graded_spd_factor_fixed_blas(n, k, lam_decades, row_decades)
    return Workload("spd-rowgraded-n%d" % n, G, None, n * DBL_EPS, ordering)


def input_sha256(G):
    """SHA-256 (hex) of a factor's bytes in column-major order."""
    import hashlib
    return hashlib.sha256(np.asfortranarray(G, dtype=np.float64).tobytes(order="F")).hexdigest()


def graded_spd_transposed(n=8192, k=2, lam_decades=3.0, row_decades=4.0):
    """The factor the trigonometric algorithm works on for the row-graded
    recipe above: the paper's trigonometric method transforms G^* from the
    right (Sec. 2.1), so the solver receives F = G^T = Q diag(lam) Q^T D,
    which is column-graded.  H = G G^T and F F^T = G^T G have the same
    eigenvalues.  lam_decades = 3 (lam = 10^U(-3,0)) keeps
    kappa(Q diag(lam) Q^T) = 1e3, for which FP64 relative accuracy of
    1e-12 is attainable; lam_decades = 6 is the literal recipe."""
    wl = graded_spd_known_factor(n, k=k, lam_decades=lam_decades, row_decades=row_decades)
    name = "spd-graded-T-n%d%s" % (n, "" if lam_decades == 3.0 else "-lam%g" % lam_decades)
    return Workload(name, np.asfortranarray(wl.G.T), None, wl.tol, MODMODULUS)


def random_signature(n, g, lo=0.3, hi=0.7):
    """J with round(rho n) entries -1 at random positions, rho ~ U(lo, hi)."""
    rho = g.uniform(lo, hi)
    J = np.ones(n, dtype=np.int8)
    neg = g.permutation(n)[: int(round(rho * n))]
    J[neg] = -1
    return J


def batch_uneven(count=4096, nmin=16, nmax=256, k=3):
    """Many independent instances with n_i ~ U{nmin..nmax}: even i positive
    definite (G ~ N(0,1), J = I), odd i indefinite (random J with 30-70 %
    negative signs, G = B diag(10^U(-2,2)))."""
    g = rng(k)
    out = []
    for i in range(count):
        n = int(g.integers(nmin, nmax + 1))
        if i % 2 == 0:
            G = g.standard_normal((n, n))
            J = None
        else:
            B = g.standard_normal((n, n))
            G = B * (10.0 ** g.uniform(-2.0, 2.0, size=n))[None, :]
            J = random_signature(n, g)
        out.append(Workload("batch-%d-n%d" % (i, n), G, J, n * DBL_EPS, MODMODULUS))
    return out


def graded_rows(m, n, k, decades=8.0, cond_decades=2.0, J=None):
    """Row-graded factor G = D B with B = Q1 diag(s) Q2^T, s log-uniform over
    cond_decades (so kappa(B) <= 10^cond_decades) and D = diag(10^U(-d, d)).
    Used for the relative-accuracy pins: kappa(H) is huge, kappa(B) is not."""
    g = rng(k)
    Q1 = haar_orthogonal(m, g)[:, :n]
    Q2 = haar_orthogonal(n, g)
    s = 10.0 ** g.uniform(-cond_decades, 0.0, size=n)
    B = (Q1 * s[None, :]) @ Q2.T
    d = 10.0 ** g.uniform(-decades, decades, size=m)
    return np.asfortranarray(d[:, None] * B)


def graded_cols(m, n, k, decades=8.0):
    """Column-graded factor G = B diag(10^U(-d, d)), B ~ N(0,1)."""
    g = rng(k)
    B = g.standard_normal((m, n))
    return np.asfortranarray(B * (10.0 ** g.uniform(-decades, decades, size=n))[None, :])


def adjoint_batch(count=256, n=128, k=5, m=None):
    """Batch for the differentiated solve: count indefinite instances of the
    uneven-batch recipe's odd kind at one size (G = B diag(10^U(-2,2)),
    B ~ N(0,1), random J with 30-70 % negative signs), with the loss weights
    w ~ N(0,1)^n and C ~ N(0,1)^{m x n} of L = sum_i w_i lambda_i + <C, U>.
    Returns (G (count, m, n), J (count, n) int8, w (count, n), C (count, m, n))."""
    g = rng(k)
    m = n if m is None else m
    G = np.empty((count, m, n))
    J = np.empty((count, n), dtype=np.int8)
    for i in range(count):
        B = g.standard_normal((m, n))
        G[i] = B * (10.0 ** g.uniform(-2.0, 2.0, size=n))[None, :]
        J[i] = random_signature(n, g)
    w = g.standard_normal((count, n))
    C = g.standard_normal((count, m, n))
    return G, J, w, C
