"""Thin ctypes binding of libjevd.so (include/jevd.h).

The functions below carry the names of the C entry points and only marshal
arguments: every step of the solve runs in the HIP library.  There is no CPU
fallback: if libjevd.so is missing or cannot be loaded, loading raises.
PyTorch is used only for device memory and streams (``evd``).
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjevd.so")

JEVD_OK, JEVD_EINVAL, JEVD_ENONFINITE, JEVD_ENOCONV, JEVD_EHIP, JEVD_ENOMEM = 0, -1, -2, -3, -4, -5
ORD_ROWCYCLIC, ORD_MODULUS, ORD_MODMODULUS = 0, 1, 2
VAR_POINTWISE, VAR_BLOCK_ORIENTED, VAR_FULL_BLOCK, VAR_AUTO = 0, 1, 2, 3
PIVOT_NONE, PIVOT_SIGN = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
INFO_MAX_SWEEPS = 64

EXPORTS = ("jevd_default_opts", "jevd_create", "jevd_destroy", "jacobi_evd", "jevd_validate",
           "jevd_get_info", "jevd_set_timing", "jevd_strerror", "jevd_ordering",
           "jevd_batch_create", "jevd_batch_run", "jevd_batch_results", "jevd_batch_destroy",
           "jacobi_evd_batched", "jevd_canonicalize", "jevd_adjoint", "jevd_adjoint_noalloc",
           "jevd_autotune",
           "jevd_tune_file", "jevd_tune_lookup", "jevd_tune_record", "jevd_mfma_f64_rate",
           "jevd_batch_waves", "jevd_batch_autotune", "jevd_batch_tune_lookup",
           "jevd_batch_tune_record")
BATCH_CLASSES = 4
K_PAIR_STEP, K_GRAM, K_PIVOT_SOLVE, K_UPDATE = 0, 1, 2, 3


class jevd_opts(ctypes.Structure):
    _fields_ = [("ordering", ctypes.c_int), ("variant", ctypes.c_int), ("block", ctypes.c_int),
                ("max_sweeps", ctypes.c_int), ("max_inner", ctypes.c_int),
                ("accumulate_v", ctypes.c_int), ("pivot", ctypes.c_int),
                ("precision", ctypes.c_int)]


class jevd_info(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int), ("variant", ctypes.c_int), ("block", ctypes.c_int),
                ("ordering", ctypes.c_int), ("rotations", ctypes.c_longlong * INFO_MAX_SWEEPS),
                ("clamps", ctypes.c_longlong), ("breakdowns", ctypes.c_longlong),
                ("kernel_ms", ctypes.c_double * 4), ("kernel_launches", ctypes.c_longlong * 4),
                ("sweeps_low", ctypes.c_int), ("v_deferred", ctypes.c_int),
                ("steps_per_launch", ctypes.c_int)]


class JevdError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what or "jevd", jevd_strerror(status), status))


_lib = None
_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)


def lib():
    """Load libjevd.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libjevd.so not found at %s: build it with "
                              "python -c 'import __graft_entry__ as g; g.build()'" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        L.jevd_default_opts.argtypes = [ctypes.POINTER(jevd_opts)]
        L.jevd_create.argtypes = [ctypes.POINTER(_vp), _vp]
        L.jevd_destroy.argtypes = [_vp]
        L.jacobi_evd.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp,
                                 ctypes.c_double, ctypes.POINTER(jevd_opts), _vp, _vp, ctypes.c_int,
                                 _vp, ctypes.c_int, _ip]
        L.jevd_validate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_double,
                                    ctypes.POINTER(jevd_opts), _vp, ctypes.c_int, _vp, ctypes.c_int]
        L.jevd_get_info.argtypes = [_vp, ctypes.POINTER(jevd_info)]
        L.jevd_set_timing.argtypes = [_vp, ctypes.c_int]
        L.jevd_strerror.argtypes = [ctypes.c_int]
        L.jevd_strerror.restype = ctypes.c_char_p
        L.jevd_ordering.argtypes = [ctypes.c_int, ctypes.c_int, _ip, _ip, _ip, _ip]
        batch_args = [_vp, ctypes.c_int, _ip, _ip, _vp, _ip, _vp, _vp, ctypes.POINTER(jevd_opts),
                      _vp, _vp, _ip, _vp, _ip]
        L.jevd_batch_create.argtypes = batch_args + [ctypes.POINTER(_vp)]
        L.jevd_batch_run.argtypes = [_vp, _vp]
        L.jevd_batch_results.argtypes = [_vp, _ip, _ip]
        L.jevd_batch_destroy.argtypes = [_vp]
        L.jacobi_evd_batched.argtypes = batch_args + [_ip, _ip]
        _i, _ll = ctypes.c_int, ctypes.c_longlong
        L.jevd_canonicalize.argtypes = [_vp, _i, _i, _i, _vp, _ll, _vp, _i, _ll, _vp, _i, _ll,
                                        _vp, _vp, _vp]
        L.jevd_adjoint.argtypes = [_vp, _i, _i, _i, _vp, _i, _ll, _vp, _ll, _vp, _ll, _vp, _i, _ll,
                                   _vp, _ll, _vp, _i, _ll, _vp, _i, _ll]
        L.jevd_adjoint_noalloc.argtypes = L.jevd_adjoint.argtypes
        _dp = ctypes.POINTER(ctypes.c_double)
        L.jevd_autotune.argtypes = [_vp, _i, _i, _vp, _i, _vp, ctypes.c_double,
                                    ctypes.POINTER(jevd_opts), _i, _ip, _ip, _dp]
        L.jevd_tune_file.argtypes = [ctypes.c_char_p]
        L.jevd_tune_lookup.argtypes = [_i, _i, _ip, _ip, _dp]
        L.jevd_tune_record.argtypes = [_i, _i, _i, _i, ctypes.c_double]
        L.jevd_mfma_f64_rate.argtypes = [_vp, _i, _i, _dp]
        L.jevd_batch_waves.argtypes = [_vp, _ip]
        L.jevd_batch_autotune.argtypes = [_vp, _i, _ip]
        L.jevd_batch_tune_lookup.argtypes = [_i, _ip, _dp]
        L.jevd_batch_tune_record.argtypes = [_i, _i, ctypes.c_double]
        for name in EXPORTS:
            if name != "jevd_strerror":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


# ------------------------------------------------------------ C entry points
def jevd_default_opts():
    o = jevd_opts()
    lib().jevd_default_opts(ctypes.byref(o))
    return o


def jevd_strerror(status):
    return lib().jevd_strerror(int(status)).decode()


def jevd_create(stream=0):
    h = _vp()
    st = lib().jevd_create(ctypes.byref(h), _vp(int(stream)) if stream else None)
    if st != JEVD_OK:
        raise JevdError(st, "jevd_create")
    return h


def jevd_destroy(h):
    return lib().jevd_destroy(h)


def jacobi_evd(h, m, n, G_ptr, ldg, J_host, tol, opts, lambda_ptr, U_ptr, ldu, V_ptr, ldv):
    """Raw call with device pointers (ints) and a host J (bytes-like of int8 or
    None).  Returns (status, sweeps)."""
    sweeps = ctypes.c_int(0)
    Jbuf = None
    if J_host is not None:
        Jbuf = (ctypes.c_byte * n).from_buffer_copy(bytes(J_host))
    st = lib().jacobi_evd(h, m, n, _vp(G_ptr), ldg, ctypes.cast(Jbuf, _vp) if Jbuf is not None else None,
                          float(tol), ctypes.byref(opts) if opts is not None else None,
                          _vp(lambda_ptr) if lambda_ptr else None, _vp(U_ptr) if U_ptr else None,
                          ldu, _vp(V_ptr) if V_ptr else None, ldv, ctypes.byref(sweeps))
    return st, sweeps.value


def jevd_autotune(h, m, n, G_ptr, ldg, J_host, tol, opts, want_v):
    """Measures the candidate configurations on a copy of the device matrix
    at G_ptr and records the fastest.  Returns (status, block, variant, ms)."""
    Jbuf = None
    if J_host is not None:
        Jbuf = (ctypes.c_byte * n).from_buffer_copy(bytes(J_host))
    b, v, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    st = lib().jevd_autotune(h, m, n, _vp(G_ptr), ldg,
                             ctypes.cast(Jbuf, _vp) if Jbuf is not None else None, float(tol),
                             ctypes.byref(opts) if opts is not None else None, 1 if want_v else 0,
                             ctypes.byref(b), ctypes.byref(v), ctypes.byref(ms))
    return st, b.value, v.value, ms.value


def jevd_tune_file(path):
    return lib().jevd_tune_file(None if path is None else os.fsencode(path))


def jevd_tune_lookup(m, n):
    """Returns (status, block, variant, ms) of the tune table's record."""
    b, v, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    st = lib().jevd_tune_lookup(m, n, ctypes.byref(b), ctypes.byref(v), ctypes.byref(ms))
    return st, b.value, v.value, ms.value


def jevd_tune_record(m, n, block, variant, ms):
    return lib().jevd_tune_record(m, n, block, variant, float(ms))


def jevd_validate(m, n, ldg, J_host, tol, opts, has_U, ldu, has_V, ldv):
    Jbuf = None
    if J_host is not None:
        Jbuf = (ctypes.c_byte * len(J_host)).from_buffer_copy(bytes(J_host))
    return lib().jevd_validate(m, n, ldg, ctypes.cast(Jbuf, _vp) if Jbuf is not None else None,
                               float(tol), ctypes.byref(opts) if opts is not None else None,
                               _vp(8) if has_U else None, ldu, _vp(8) if has_V else None, ldv)


def jevd_get_info(h):
    info = jevd_info()
    st = lib().jevd_get_info(h, ctypes.byref(info))
    if st != JEVD_OK:
        raise JevdError(st, "jevd_get_info")
    return info


def jevd_set_timing(h, on):
    st = lib().jevd_set_timing(h, 1 if on else 0)
    if st != JEVD_OK:
        raise JevdError(st, "jevd_set_timing")


def jevd_mfma_f64_rate(h, waves_per_simd=4, iters=2048):
    """TFLOP/s the GPU sustains on independent FP64 MFMAs from registers."""
    t = ctypes.c_double(0.0)
    st = lib().jevd_mfma_f64_rate(h, int(waves_per_simd), int(iters), ctypes.byref(t))
    if st != JEVD_OK:
        raise JevdError(st, "jevd_mfma_f64_rate")
    return t.value


def jevd_batch_waves(plan):
    """Wavefronts per workgroup of each size class of a plan (0: empty)."""
    w = (ctypes.c_int * BATCH_CLASSES)()
    st = lib().jevd_batch_waves(plan, w)
    if st != JEVD_OK:
        raise JevdError(st, "jevd_batch_waves")
    return list(w)


def jevd_batch_autotune(h, want_v=True):
    """Measures the batched solve's workgroup sizes per size class; returns
    the choices (also recorded in the tune table)."""
    w = (ctypes.c_int * BATCH_CLASSES)()
    st = lib().jevd_batch_autotune(h, 1 if want_v else 0, w)
    if st != JEVD_OK:
        raise JevdError(st, "jevd_batch_autotune")
    return list(w)


def jevd_batch_tune_lookup(size_class):
    """Returns (status, waves, ms) of the table's record for a size class."""
    w, ms = ctypes.c_int(0), ctypes.c_double(0.0)
    st = lib().jevd_batch_tune_lookup(int(size_class), ctypes.byref(w), ctypes.byref(ms))
    return st, w.value, ms.value


def jevd_batch_tune_record(size_class, waves, ms):
    return lib().jevd_batch_tune_record(int(size_class), int(waves), float(ms))


def jevd_ordering(n, ordering):
    """Steps of 0-based pairs, as the solver runs them (host only)."""
    ns, npr = ctypes.c_int(0), ctypes.c_int(0)
    st = lib().jevd_ordering(n, ordering, None, None, ctypes.byref(ns), ctypes.byref(npr))
    if st != JEVD_OK:
        raise JevdError(st, "jevd_ordering")
    starts = (ctypes.c_int * (ns.value + 1))()
    pairs = (ctypes.c_int * max(1, 2 * npr.value))()
    lib().jevd_ordering(n, ordering, starts, pairs, None, None)
    return [[(pairs[2 * e], pairs[2 * e + 1]) for e in range(starts[k], starts[k + 1])]
            for k in range(ns.value)]


class _BatchArgs:
    """Host arrays of one batch (lengths = batch), kept alive with the plan."""

    def __init__(self, m, n, G_ptrs, ldg, J_list, tol, lam_ptrs, U_ptrs, ldu, V_ptrs, ldv):
        b = len(m)
        ia = ctypes.c_int * b
        pa = _vp * b
        self.batch = b
        self.m, self.n, self.ldg = ia(*m), ia(*n), ia(*ldg)
        self.G = pa(*[_vp(p) for p in G_ptrs])
        self.Jbufs = []
        self.J = None
        if J_list is not None and any(j is not None for j in J_list):
            self.J = pa()
            for i, j in enumerate(J_list):
                if j is not None:
                    buf = (ctypes.c_byte * len(bytes(j))).from_buffer_copy(bytes(j))
                    self.Jbufs.append(buf)
                    self.J[i] = ctypes.cast(buf, _vp)
        self.tol = None if tol is None else (ctypes.c_double * b)(*[float(t) for t in tol])

        def ptrs(lst):
            return None if lst is None else pa(*[_vp(p) if p else None for p in lst])

        self.lam, self.U, self.V = ptrs(lam_ptrs), ptrs(U_ptrs), ptrs(V_ptrs)
        self.ldu = None if ldu is None else ia(*ldu)
        self.ldv = None if ldv is None else ia(*ldv)

    def call_args(self, h, opts):
        return (h, self.batch, self.m, self.n, self.G, self.ldg, self.J, self.tol,
                ctypes.byref(opts) if opts is not None else None, self.lam, self.U, self.ldu,
                self.V, self.ldv)


def jevd_batch_create(h, m, n, G_ptrs, ldg, J_list, tol, opts, lam_ptrs, U_ptrs, ldu, V_ptrs, ldv):
    """Raw plan creation: lists of ints (device pointers as ints, 0 = NULL),
    J_list of bytes-like int8 or None.  Returns (status, plan, keepalive)."""
    a = _BatchArgs(m, n, G_ptrs, ldg, J_list, tol, lam_ptrs, U_ptrs, ldu, V_ptrs, ldv)
    plan = _vp()
    st = lib().jevd_batch_create(*a.call_args(h, opts), ctypes.byref(plan))
    return st, plan, a


def jevd_batch_run(plan, stream=0):
    return lib().jevd_batch_run(plan, _vp(int(stream)) if stream else None)


def jevd_batch_results(plan, batch):
    sw, stv = (ctypes.c_int * batch)(), (ctypes.c_int * batch)()
    st = lib().jevd_batch_results(plan, sw, stv)
    return st, list(sw), list(stv)


def jevd_batch_destroy(plan):
    return lib().jevd_batch_destroy(plan)


def jacobi_evd_batched(h, m, n, G_ptrs, ldg, J_list, tol, opts, lam_ptrs, U_ptrs, ldu, V_ptrs, ldv):
    """Returns (status, sweeps list, status list)."""
    a = _BatchArgs(m, n, G_ptrs, ldg, J_list, tol, lam_ptrs, U_ptrs, ldu, V_ptrs, ldv)
    sw, stv = (ctypes.c_int * a.batch)(), (ctypes.c_int * a.batch)()
    st = lib().jacobi_evd_batched(*a.call_args(h, opts), sw, stv)
    return st, list(sw), list(stv)


def _p(x):
    return _vp(int(x)) if x else None


def jevd_canonicalize(h, batch, m, n, lam, slam, U, ldu, su, V, ldv, sv, lam_out, U_out, V_out):
    """Raw call; pointers are device addresses as ints (0 = NULL)."""
    return lib().jevd_canonicalize(h, batch, m, n, _p(lam), slam, _p(U), ldu, su, _p(V), ldv, sv,
                                   _p(lam_out), _p(U_out), _p(V_out))


def jevd_adjoint(h, batch, m, n, G, ldg, sg, J, sj, lam, slam, U, ldu, su, w, sw, C, ldc, sc, dG,
                 ldd, sd):
    """Raw call; pointers are device addresses as ints (0 = NULL); J is a
    device int8 array."""
    return lib().jevd_adjoint(h, batch, m, n, _p(G), ldg, sg, _p(J), sj, _p(lam), slam, _p(U), ldu,
                              su, _p(w), sw, _p(C), ldc, sc, _p(dG), ldd, sd)


def jevd_adjoint_noalloc(h, batch, m, n, G, ldg, sg, J, sj, lam, slam, U, ldu, su, w, sw, C, ldc,
                         sc, dG, ldd, sd):
    """jevd_adjoint on the library's fixed scratch (no allocation); same
    arguments."""
    return lib().jevd_adjoint_noalloc(h, batch, m, n, _p(G), ldg, sg, _p(J), sj, _p(lam), slam, _p(U),
                                      ldu, su, _p(w), sw, _p(C), ldc, sc, _p(dG), ldd, sd)


# ----------------------------------------------------------- torch front end
class Solver:
    """Owns a handle bound to the current device and torch's current stream."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("jevd needs a ROCm GPU; none is visible")
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        self.h = jevd_create(s.cuda_stream)

    def close(self):
        if self.h:
            jevd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def evd(self, G, J=None, tol=0.0, ordering=ORD_MODMODULUS, variant=VAR_AUTO, block=0,
            max_sweeps=50, max_inner=30, want_U=True, want_V=True, V0=None, check=True,
            pivot=PIVOT_NONE, precision=PREC_FP64):
        """Solve in place on the device tensor G (float64, column-major: pass
        a tensor whose .T is contiguous, or any (m, n) tensor with stride
        (1, ldg)).  Returns (lam, U, V, sweeps, status)."""
        import torch
        if G.dtype != torch.float64 or not G.is_cuda:
            raise TypeError("G must be a float64 device tensor")
        m, n = G.shape
        if G.stride(0) != 1:
            raise ValueError("G must be column-major (stride(0) == 1)")
        ldg = G.stride(1) if n > 1 else m
        dev = G.device
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        U = torch.empty((n, m), dtype=torch.float64, device=dev).T if want_U else None
        V = None
        o = jevd_default_opts()
        o.ordering, o.variant, o.block = ordering, variant, block
        o.max_sweeps, o.max_inner = max_sweeps, max_inner
        o.pivot = pivot
        o.precision = precision
        if V0 is not None:
            V = V0
            o.accumulate_v = 1
        elif want_V:
            V = torch.empty((n, n), dtype=torch.float64, device=dev).T
        Jb = None
        if J is not None:
            import numpy as np
            Jb = np.ascontiguousarray(np.asarray(J.cpu() if hasattr(J, "cpu") else J).astype(np.int8)).tobytes()
        st, sweeps = jacobi_evd(self.h, m, n, G.data_ptr(), ldg, Jb, tol, o, lam.data_ptr(),
                                U.data_ptr() if U is not None else 0, m,
                                V.data_ptr() if V is not None else 0, n if V is None else V.stride(1))
        if check and st not in (JEVD_OK,):
            raise JevdError(st, "jacobi_evd")
        return lam, U, V, sweeps, st

    def batch_plan(self, Gs, Js=None, tols=None, ordering=ORD_MODMODULUS, max_sweeps=50,
                   want_U=True, want_V=True):
        """Plan for the device tensors Gs (float64, column-major, solved in
        place).  Returns a BatchPlan holding lam/U/V output tensors."""
        return BatchPlan(self, Gs, Js, tols, ordering, max_sweeps, want_U, want_V)

    def evd_batched(self, Gs, Js=None, tols=None, ordering=ORD_MODMODULUS, max_sweeps=50,
                    want_U=True, want_V=True, check=True):
        """One batched solve.  Returns (lams, Us, Vs, sweeps, statuses)."""
        plan = self.batch_plan(Gs, Js, tols, ordering, max_sweeps, want_U, want_V)
        try:
            plan.run()
            st, sweeps, stv = plan.results()
            if check and st != JEVD_OK:
                raise JevdError(st, "jevd_batch_results")
            return plan.lams, plan.Us, plan.Vs, sweeps, stv
        finally:
            plan.close()

    def info(self):
        return jevd_get_info(self.h)

    def set_timing(self, on):
        jevd_set_timing(self.h, on)


class BatchPlan:
    """A jevd_batch_t over torch device tensors (see Solver.batch_plan)."""

    def __init__(self, solver, Gs, Js, tols, ordering, max_sweeps, want_U, want_V):
        import torch
        import numpy as np
        self.solver = solver
        self.plan = None
        m, n, ldg, gp, Jl = [], [], [], [], []
        self.lams, self.Us, self.Vs = [], [], []
        for i, G in enumerate(Gs):
            if G.dtype != torch.float64 or not G.is_cuda or G.stride(0) != 1:
                raise TypeError("batch entry %d: G must be a column-major float64 device tensor" % i)
            mi, ni = G.shape
            m.append(mi)
            n.append(ni)
            ldg.append(G.stride(1) if ni > 1 else mi)
            gp.append(G.data_ptr())
            J = None if Js is None else Js[i]
            Jl.append(None if J is None else
                      np.ascontiguousarray(np.asarray(J.cpu() if hasattr(J, "cpu") else J)
                                           .astype(np.int8)).tobytes())
            self.lams.append(torch.empty(ni, dtype=torch.float64, device=G.device))
            self.Us.append(torch.empty((ni, mi), dtype=torch.float64, device=G.device).T
                           if want_U else None)
            self.Vs.append(torch.empty((ni, ni), dtype=torch.float64, device=G.device).T
                           if want_V else None)
        o = jevd_default_opts()
        o.ordering, o.variant, o.max_sweeps = ordering, VAR_POINTWISE, max_sweeps
        st, plan, self._keep = jevd_batch_create(
            solver.h, m, n, gp, ldg, Jl if Js is not None else None, tols, o,
            [t.data_ptr() for t in self.lams],
            [u.data_ptr() for u in self.Us] if want_U else None, m if want_U else None,
            [v.data_ptr() for v in self.Vs] if want_V else None, n if want_V else None)
        if st != JEVD_OK:
            raise JevdError(st, "jevd_batch_create")
        self.plan = plan
        self.batch = len(m)

    def run(self, stream=None):
        st = jevd_batch_run(self.plan, stream.cuda_stream if stream is not None else 0)
        if st != JEVD_OK:
            raise JevdError(st, "jevd_batch_run")

    def results(self):
        return jevd_batch_results(self.plan, self.batch)

    def close(self):
        if self.plan:
            jevd_batch_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
