"""GPU parity of the sign-pivoted block variants (Alg. 3.3 in the pivot
solve: HBSC / HFSC; diagonal pivoting for J = I) against the oracle's
sign-pivoted block solve on the same seeded inputs: eigenvalues as for the
unpivoted block path (1e-12, or the bound (1.2) against a high-precision
oracle run: oracle/gates.py), sweep counts within one, the inertia of J kept,
V^T J V = diag(sign(lambda)) and G_out = G_in V.  Needs an MI355X."""
import numpy as np
import pytest

from paper_1008_0201_amd import workloads as W
from test_gpu_block import check_eigs, dev_colmajor

pytestmark = pytest.mark.gpu
EPS = W.DBL_EPS


@pytest.fixture(scope="module")
def solver():
    import torch
    from paper_1008_0201_amd import jevd
    assert torch.cuda.is_available()
    s = jevd.Solver()
    yield s
    s.close()


def run_sp(solver, G, J, tol, full_block, b, pivot=1):
    Gd = dev_colmajor(G)
    lam, U, V, sweeps, st = solver.evd(Gd, J, tol=tol, variant=2 if full_block else 1, block=b,
                                       check=False, pivot=pivot)
    return dict(st=st, lam=lam.cpu().numpy(), U=U.cpu().numpy(), V=V.cpu().numpy(),
                G=Gd.cpu().numpy(), sweeps=sweeps)


def check_sp(orc, G, J, tol, b, full_block, got):
    ref = orc.block_jevd(G, J, tol, b=b, full_block=full_block, sign_pivot=True)
    assert ref.status == 0 and got["st"] == 0, (ref.status, got["st"])
    check_eigs(orc, G, J, got["lam"], ref.lam)
    assert abs(got["sweeps"] - ref.sweeps) <= 1, (got["sweeps"], ref.sweeps)
    n = G.shape[1]
    jin = np.ones(n) if J is None else np.asarray(J, dtype=float)
    jout = np.sign(got["lam"])
    assert int((jout > 0).sum()) == int((jin > 0).sum())          # inertia
    U = got["U"]
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= 10 * n * EPS
    V = got["V"]
    vmax = np.max(np.sum(V * V, axis=0))
    dev = np.max(np.abs(V.T @ (jin[:, None] * V) - np.diag(jout)))
    Vr = ref.V
    dev_ref = np.max(np.abs(Vr.T @ (jin[:, None] * Vr) - np.diag(ref.J.astype(float))))
    assert dev <= max(10 * n * EPS * vmax, 4 * dev_ref), (dev, dev_ref)
    GV = (G.astype(np.longdouble) @ V.astype(np.longdouble)).astype(np.float64)
    scale = np.sqrt(np.sum((np.abs(G) @ np.abs(V)) ** 2, axis=0))
    assert np.max(np.abs(GV - got["G"]).sum(axis=0) / scale) <= 100 * n * EPS
    return ref


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("n,b", [(128, 16), (256, 32), (192, 32)])
@pytest.mark.parametrize("full_block", [False, True])
def test_sign_pivoted_hyperbolic(solver, orc, n, b, full_block, mixed):
    wl = W.graded_hyperbolic(n, k=400 + n, grade=2.0)
    J = W.random_signature(n, np.random.default_rng(n)) if mixed else wl.J
    got = run_sp(solver, wl.G, J, wl.tol, full_block, b)
    ref = check_sp(orc, wl.G, J, wl.tol, b, full_block, got)
    unp = run_sp(solver, wl.G, J, wl.tol, full_block, b, pivot=0)
    print("n=%d b=%d fb=%d mixed=%d sweeps: sign-pivoted gpu %d oracle %d, unpivoted gpu %d"
          % (n, b, full_block, mixed, got["sweeps"], ref.sweeps, unp["sweeps"]))


@pytest.mark.parametrize("full_block", [False, True])
def test_diagonal_pivoting_trig(solver, orc, full_block):
    """J = I: the diagonally pivoted Cholesky on a row-graded factor."""
    G = W.graded_rows(160, 128, k=909, decades=4.0, cond_decades=3.0)
    got = run_sp(solver, G, None, 128 * EPS, full_block, 16)
    check_sp(orc, G, None, 128 * EPS, 16, full_block, got)


def test_sign_pivot_option_rules(solver):
    from paper_1008_0201_amd import jevd
    G = dev_colmajor(np.random.default_rng(3).standard_normal((64, 64)))
    lam, U, V, sweeps, st = solver.evd(G, None, variant=0, check=False, pivot=1)
    assert st == jevd.JEVD_EINVAL          # pointwise has no Cholesky
    lam, U, V, sweeps, st = solver.evd(G, None, variant=1, block=16, check=False, pivot=2)
    assert st == jevd.JEVD_EINVAL


@pytest.mark.parametrize("full_block", [False, True])
def test_sign_pivoted_breakdown(solver, orc, full_block):
    """A zero column breaks the sign-pivoted Cholesky of its pivots down
    (Alg. 3.3 meets a zero pivot): on both sides such a pivot is processed
    on the columns of G_P with the unpivoted signs (no column moves), and the
    result meets the gates of the other sign-pivoted cases."""
    n = 128
    wl = W.graded_hyperbolic(n, k=433, grade=2.0)
    G = wl.G.copy()
    G[:, 45] = 0.0
    got = run_sp(solver, G, wl.J, wl.tol, full_block, 16)
    info = solver.info()
    ref = orc.block_jevd(G, wl.J, wl.tol, b=16, full_block=full_block, sign_pivot=True)
    assert ref.extra > 0 and info.breakdowns > 0
    assert ref.status == 0 and got["st"] == 0
    zero = np.flatnonzero(got["lam"] == 0.0)
    assert len(zero) == 1 and np.all(got["U"][:, zero[0]] == 0.0)
    nz = got["lam"] != 0.0
    nzr = ref.lam != 0.0
    Gs = np.delete(G, 45, axis=1)
    Js = np.delete(wl.J, 45)
    check_eigs(orc, Gs, Js, got["lam"][nz], ref.lam[nzr])
    assert abs(got["sweeps"] - ref.sweeps) <= 1, (got["sweeps"], ref.sweeps)
