"""ctypes front end of the one-sided Jacobi oracle (plain C, liboracle.so).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg may call this module; the product path (the HIP library and
its Python binding) never imports it, and this module imports nothing of
the product.

Every function takes and returns numpy FP64 arrays.  ``prec`` selects the
internal arithmetic of the C code: 'd' (double), 'l' (x87 long double,
64-bit mantissa) or 'q' (__float128); inputs are converted once on entry and
results rounded once to double on exit, so 'q' runs serve as truth for the
accuracy pins.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB lets the mutation tests point this front end at a copy of the
# oracle with a deliberately planted mistake (built in a temporary folder).
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

ROWCYCLIC, MODULUS, MODMODULUS = 0, 1, 2
STATUS = {0: "ok", -1: "einval", -2: "enonfinite", -3: "enoconv", -5: "enomem"}

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_llp = ctypes.POINTER(ctypes.c_longlong)
_cp = ctypes.c_void_p


def lib():
    """Load liboracle.so (building it first if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # noqa: F401  (package-relative import)
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_ordering.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _ip, _ip]
        L.orc_ordering.restype = ctypes.c_int
        for s in "dlq":
            f = getattr(L, "orc_jevd_" + s)
            f.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _cp,
                          ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          _dp, _dp, ctypes.c_int, _ip, _llp, _llp]
            f.restype = ctypes.c_int
            f = getattr(L, "orc_block_jevd_" + s)
            f.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _cp,
                          ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _ip,
                          _llp, _llp]
            f.restype = ctypes.c_int
            f = getattr(L, "orc_block_jevd_sp_" + s)
            f.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _cp,
                          ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _ip,
                          _llp, _llp, _cp]
            f.restype = ctypes.c_int
            f = getattr(L, "orc_sp_cholesky_" + s)
            f.argtypes = [ctypes.c_int, _dp, _cp, _dp, _ip, _ip]
            f.restype = ctypes.c_int
            f = getattr(L, "orc_block_steps_" + s)
            f.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _cp, ctypes.c_double,
                          ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int]
            f.restype = ctypes.c_int
            f = getattr(L, "orc_block_jevd_mt_" + s)
            f.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _cp,
                          ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int, _ip,
                          _llp, _llp, _cp, ctypes.c_int]
            f.restype = ctypes.c_int
            f = getattr(L, "orc_rotation_" + s)
            f.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                          ctypes.c_int, _dp, _dp]
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def ordering(n, kind):
    """List of steps; each step is a list of 0-based pairs (i, j), i < j."""
    L = lib()
    npairs = ctypes.c_int(0)
    nsteps = L.orc_ordering(n, kind, None, None, ctypes.byref(npairs))
    if nsteps < 0:
        raise ValueError("bad ordering arguments")
    starts = np.zeros(nsteps + 1, dtype=np.int32)
    pairs = np.zeros(2 * max(npairs.value, 1), dtype=np.int32)
    L.orc_ordering(n, kind, _ptr(starts, _ip), _ptr(pairs, _ip), None)
    return [[(int(pairs[2 * e]), int(pairs[2 * e + 1])) for e in range(starts[s], starts[s + 1])]
            for s in range(nsteps)]


class Result:
    """Outputs of one oracle solve."""

    def __init__(self, status, G, lam, V, sweeps, rot, extra):
        self.status = status
        self.G = G            # final iterate G V (m x n)
        self.lam = lam        # j_i ||g_i||^2 of the final iterate
        self.V = V            # accumulated transform (n x n) or None
        self.sweeps = sweeps  # sweeps executed, including the last one without rotations
        self.rot = rot        # rotations applied in each sweep
        self.extra = extra    # clamps (pointwise) or Cholesky breakdowns (block)

    @property
    def U(self):
        """Eigenvectors: the columns of G V normalised (zero columns stay zero)."""
        nrm = np.sqrt(np.sum(self.G * self.G, axis=0))
        safe = np.where(nrm > 0, nrm, 1.0)
        return self.G / safe


def _prep(G, J, want_v, V0):
    G = np.array(G, dtype=np.float64, order="F", copy=True)
    m, n = G.shape
    Jb = None
    if J is not None:
        Jb = np.ascontiguousarray(np.asarray(J).astype(np.int8))
        if Jb.shape != (n,):
            raise ValueError("J must have n entries")
    V = None
    if want_v or V0 is not None:
        V = np.array(V0 if V0 is not None else np.zeros((n, n)), dtype=np.float64,
                     order="F", copy=True)
    return G, m, n, Jb, V


def jevd(G, J=None, tol=None, ordering_kind=MODMODULUS, max_sweeps=50, want_v=True,
         V0=None, prec="d"):
    """Pointwise one-sided Jacobi; see oracle/jacobi.c.  tol=None means n*DBL_EPSILON."""
    G, m, n, Jb, V = _prep(G, J, want_v, V0)
    if tol is None:
        tol = n * np.finfo(np.float64).eps
    lam = np.zeros(n)
    sweeps = ctypes.c_int(0)
    rot = np.zeros(max(max_sweeps, 1), dtype=np.int64)
    ncl = ctypes.c_longlong(0)
    f = getattr(lib(), "orc_jevd_" + prec)
    st = f(m, n, _ptr(G), m, None if Jb is None else Jb.ctypes.data_as(_cp), float(tol),
           ordering_kind, max_sweeps, 1 if V0 is not None else 0, _ptr(lam),
           None if V is None else _ptr(V), n, ctypes.byref(sweeps), _ptr(rot, _llp),
           ctypes.byref(ncl))
    return Result(st, G, lam, V, sweeps.value, rot[:sweeps.value].copy(), ncl.value)


def block_jevd(G, J=None, tol=None, b=8, full_block=False, max_sweeps=50, max_inner=30,
               want_v=True, V0=None, prec="d", sign_pivot=False, nthreads=1):
    """Block one-sided Jacobi; see oracle/jacobi.c.  sign_pivot selects the
    sign-pivoted Cholesky of Alg. 3.3 (HBSC / HFSC); the result's .J then
    holds the final column signs (the pivoting permutes them).  nthreads > 1
    (or <= 0: all cores) spreads the disjoint pivots of each step over
    threads (orc_block_jevd_mt), with results bit for bit those of the
    sequential run."""
    G, m, n, Jb, V = _prep(G, J, want_v, V0)
    if tol is None:
        tol = n * np.finfo(np.float64).eps
    lam = np.zeros(n)
    sweeps = ctypes.c_int(0)
    rot = np.zeros(max(max_sweeps, 1), dtype=np.int64)
    nbr = ctypes.c_longlong(0)
    Jp = None if Jb is None else Jb.ctypes.data_as(_cp)
    args = [m, n, _ptr(G), m, Jp, float(tol), b, 1 if full_block else 0, max_sweeps, max_inner,
            1 if V0 is not None else 0, _ptr(lam), None if V is None else _ptr(V), n,
            ctypes.byref(sweeps), _ptr(rot, _llp), ctypes.byref(nbr)]
    Jout = np.ones(n, dtype=np.int8)
    if nthreads != 1:
        st = getattr(lib(), "orc_block_jevd_mt_" + prec)(
            *args[:8], 1 if sign_pivot else 0, *args[8:], Jout.ctypes.data_as(_cp), int(nthreads))
        if not sign_pivot and Jb is not None:
            Jout = Jb.copy()
    elif sign_pivot:
        st = getattr(lib(), "orc_block_jevd_sp_" + prec)(*args, Jout.ctypes.data_as(_cp))
    else:
        st = getattr(lib(), "orc_block_jevd_" + prec)(*args)
        if Jb is not None:
            Jout = Jb.copy()
    r = Result(st, G, lam, V, sweeps.value, rot[:sweeps.value].copy(), nbr.value)
    r.J = Jout
    return r


def sp_cholesky(A, JP, prec="d"):
    """Alg. 3.3 on one symmetric w x w Gram A with signs JP: returns
    (status, R_S, perm, npos) with P^T A P = R_S^T R_S, P = I[:, perm]."""
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    w = A.shape[0]
    Jb = np.ascontiguousarray(np.asarray(JP).astype(np.int8))
    RS = np.zeros((w, w), order="F")
    perm = np.zeros(w, dtype=np.int32)
    npos = ctypes.c_int(0)
    st = getattr(lib(), "orc_sp_cholesky_" + prec)(w, _ptr(A), Jb.ctypes.data_as(_cp), _ptr(RS),
                                                 _ptr(perm, _ip), ctypes.byref(npos))
    return st, RS, perm, npos.value


def block_steps(G, J=None, tol=None, b=32, full_block=False, max_inner=30, steps=1, prec="d",
                sign_pivot=False, nthreads=1):
    """The first `steps` outer steps of one block sweep (a bounded sample of
    the block algorithm's work); returns (status, G after those steps).
    nthreads as for block_jevd."""
    G, m, n, Jb, _ = _prep(G, J, False, None)
    if tol is None:
        tol = n * np.finfo(np.float64).eps
    f = getattr(lib(), "orc_block_steps_" + prec)
    st = f(m, n, _ptr(G), m, None if Jb is None else Jb.ctypes.data_as(_cp), float(tol), b,
           1 if full_block else 0, max_inner, steps, 1 if sign_pivot else 0, int(nthreads))
    return st, G


def rotation(app, aqq, apq, same_sign, prec="d"):
    """(c, s, clamped) of the 2x2 transform for the Gram (app, aqq, apq)."""
    c = ctypes.c_double(0)
    s = ctypes.c_double(0)
    f = getattr(lib(), "orc_rotation_" + prec)
    cl = f(float(app), float(aqq), float(apq), 1 if same_sign else 0, ctypes.byref(c),
           ctypes.byref(s))
    return c.value, s.value, bool(cl)
