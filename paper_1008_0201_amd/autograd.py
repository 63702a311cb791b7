"""torch.autograd front end of the batched solver and its adjoint.

``eigh_jacobi(G, J)`` takes a batch of factors G (B x m x n, float64, on the
GPU, m >= n) and signatures J (B x n of +-1, or None for J = I) and returns
the eigenvalues lam (B x n) and orthonormal eigenvectors U (B x m x n) of
H_b = G_b J_b G_b^T in canonical form (eigenpairs sorted by decreasing
lambda, each u_i signed so that its entry of largest magnitude is
positive).  The forward pass is one batched one-sided Jacobi solve
(jevd_batch_run) plus jevd_canonicalize; the backward pass is jevd_adjoint.
Every step runs in the HIP library; this module only moves pointers and
tensors.  There is no CPU path.
"""
import atexit
import collections

import torch

from . import jevd as B

_solvers = {}
# Batch plans bound to workspace tensors, reused by forwards of the same
# shape, signatures, tolerance and stream; least recently used first.
_plans = collections.OrderedDict()
_PLAN_CACHE_MAX = 4


def _solver():
    """One library handle per (device, current stream)."""
    dev = torch.cuda.current_device()
    st = torch.cuda.current_stream()
    key = (dev, st.cuda_stream)
    s = _solvers.get(key)
    if s is None:
        s = B.Solver(st)
        _solvers[key] = s
    return s, key


def _ptrs(t, count, per):
    base = t.data_ptr()
    return [base + 8 * per * b for b in range(count)]


class _Plan:
    """A batch plan and the workspace it is bound to: the working copy of G
    (column-major instances, ld = m) and the solver's lam, U and V, which the
    forward canonicalises into fresh tensors.  A plan may be run again
    (jevd_batch_run restarts the queue and sets V to I), and the forwards
    that share it run in order on one stream, so a forward's copy into the
    workspace runs after the previous forward's last read of it."""

    def __init__(self, s, nb, m, n, Jh, tol, max_sweeps, device):
        self.Gw = torch.empty((nb, n, m), dtype=torch.float64, device=device)
        self.lam = torch.empty((nb, n), dtype=torch.float64, device=device)
        self.U = torch.empty((nb, n, m), dtype=torch.float64, device=device)
        self.V = torch.empty((nb, n, n), dtype=torch.float64, device=device)
        o = B.jevd_default_opts()
        o.variant = B.VAR_POINTWISE
        o.max_sweeps = max_sweeps
        st, self.plan, self.keep = B.jevd_batch_create(
            s.h, [m] * nb, [n] * nb, _ptrs(self.Gw, nb, m * n), [m] * nb, Jh,
            None if tol is None else [tol] * nb, o, _ptrs(self.lam, nb, n),
            _ptrs(self.U, nb, m * n), [m] * nb, _ptrs(self.V, nb, n * n), [n] * nb)
        if st != B.JEVD_OK:
            self.plan = None
            raise B.JevdError(st, "jevd_batch_create")

    def close(self):
        if self.plan is not None:
            B.jevd_batch_destroy(self.plan)
            self.plan = None


def _plan_for(s, skey, nb, m, n, Jh, tol, max_sweeps, device):
    key = (skey, nb, m, n, None if Jh is None else b"".join(Jh), tol, max_sweeps)
    p = _plans.get(key)
    if p is not None:
        _plans.move_to_end(key)
        return p
    while len(_plans) >= _PLAN_CACHE_MAX:
        _plans.popitem(last=False)[1].close()
    p = _Plan(s, nb, m, n, Jh, tol, max_sweeps, device)
    _plans[key] = p
    return p


@atexit.register
def _release():
    """Plans go before the handles they were created on."""
    while _plans:
        _plans.popitem()[1].close()
    for s in _solvers.values():
        s.close()
    _solvers.clear()


class JacobiEVD(torch.autograd.Function):
    @staticmethod
    def forward(ctx, G, J, tol, max_sweeps):
        if G.dtype != torch.float64 or not G.is_cuda or G.dim() != 3:
            raise TypeError("G must be a (B, m, n) float64 GPU tensor")
        nb, m, n = G.shape
        if m < n:
            raise ValueError("need m >= n")
        s, skey = _solver()
        Gc = G.detach().transpose(1, 2).contiguous()     # column-major instances, ld = m
        Jh = None
        Jd = None
        if J is not None:
            Jd = J.to(device=G.device, dtype=torch.int8).contiguous()
            Jh = [bytes(row) for row in Jd.cpu().numpy()]
        p = _plan_for(s, skey, nb, m, n, Jh, tol, max_sweeps, G.device)
        p.Gw.copy_(Gc)
        lam, U, V = p.lam, p.U, p.V
        st = B.jevd_batch_run(p.plan)
        if st != B.JEVD_OK:
            raise B.JevdError(st, "jevd_batch_run")
        st, sweeps, stv = B.jevd_batch_results(p.plan, nb)
        if st != B.JEVD_OK:
            raise B.JevdError(st, "instance %d" % next(i for i, x in enumerate(stv) if x))
        lam_c = torch.empty_like(lam)
        U_c = torch.empty_like(U)
        V_c = torch.empty_like(V)
        st = B.jevd_canonicalize(s.h, nb, m, n, lam.data_ptr(), n, U.data_ptr(), m, m * n,
                                 V.data_ptr(), n, n * n, lam_c.data_ptr(), U_c.data_ptr(),
                                 V_c.data_ptr())
        if st != B.JEVD_OK:
            raise B.JevdError(st, "jevd_canonicalize")
        ctx.save_for_backward(Gc, lam_c, U_c, *(() if Jd is None else (Jd,)))
        ctx.shape = (nb, m, n)
        ctx.has_j = Jd is not None
        ctx.sweeps = sweeps
        return lam_c, U_c.transpose(1, 2)

    @staticmethod
    def backward(ctx, g_lam, g_U):
        nb, m, n = ctx.shape
        saved = ctx.saved_tensors
        Gc, lam_c, U_c = saved[:3]
        Jd = saved[3] if ctx.has_j else None
        s, _ = _solver()
        w = None if g_lam is None else g_lam.detach().to(torch.float64).contiguous()
        C = None if g_U is None else g_U.detach().to(torch.float64).transpose(1, 2).contiguous()
        dG = torch.empty_like(Gc)
        st = B.jevd_adjoint(s.h, nb, m, n, Gc.data_ptr(), m, m * n,
                            0 if Jd is None else Jd.data_ptr(), n, lam_c.data_ptr(), n,
                            U_c.data_ptr(), m, m * n, 0 if w is None else w.data_ptr(), n,
                            0 if C is None else C.data_ptr(), m, m * n, dG.data_ptr(), m, m * n)
        if st != B.JEVD_OK:
            raise B.JevdError(st, "jevd_adjoint")
        return dG.transpose(1, 2), None, None, None


def eigh_jacobi(G, J=None, tol=None, max_sweeps=50):
    """(lam, U) of H_b = G_b J_b G_b^T, differentiable in G (see the module
    docstring).  tol None: n eps per instance."""
    return JacobiEVD.apply(G, J, tol, max_sweeps)
