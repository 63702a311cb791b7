"""GPU checks of the mixed-precision block path (FP32-MFMA sweeps, FP64
re-orthogonalisation of V0, G <- G V0, FP64 sweeps): the eigenvalues meet
the FP64 gate against the oracle (1e-12, or the bound (1.2) against a
high-precision oracle run: oracle/gates.py), as do those of the FP64 block
path on the same input; U and V are orthogonal to FP64 working precision
and G_out = G_in V.  Needs an MI355X."""
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


def run(solver, G, variant, b, precision, want_V=True):
    Gd = dev_colmajor(G)
    lam, U, V, sweeps, st = solver.evd(Gd, None, variant=variant, block=b, check=False,
                                       want_V=want_V, precision=precision)
    info = solver.info()
    return dict(st=st, lam=lam.cpu().numpy(), U=U.cpu().numpy(),
                V=None if V is None else V.cpu().numpy(), G=Gd.cpu().numpy(), sweeps=sweeps,
                low=info.sweeps_low)


@pytest.mark.parametrize("n,b,variant", [(256, 16, 1), (512, 32, 1), (512, 32, 2), (1024, 32, 1)])
def test_mixed_matches_oracle(solver, orc, n, b, variant):
    wl = W.graded_spd_transposed(n, k=2, lam_decades=3.0)
    got = run(solver, wl.G, variant, b, 1)
    assert got["st"] == 0 and got["low"] > 0
    ref = orc.jevd(wl.G, None, wl.tol, orc.MODMODULUS, want_v=False)
    check_eigs(orc, wl.G, None, got["lam"], ref.lam)
    U, V = got["U"], got["V"]
    assert np.max(np.abs(U.T @ U - np.eye(n))) <= 10 * n * EPS
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 10 * n * EPS
    GV = (wl.G.astype(np.longdouble) @ V.astype(np.longdouble)).astype(np.float64)
    scale = np.sqrt(np.sum((np.abs(wl.G) @ np.abs(V)) ** 2, axis=0))
    assert np.max(np.abs(GV - got["G"]).sum(axis=0) / scale) <= 100 * n * EPS
    # the FP64 block path on the same input meets the same gate
    fp64 = run(solver, wl.G, variant, b, 0, want_V=False)
    check_eigs(orc, wl.G, None, fp64["lam"], ref.lam)
    print("n=%d b=%d variant=%d: mixed %d FP32 + %d FP64 sweeps, FP64 path %d sweeps"
          % (n, b, variant, got["low"], got["sweeps"], fp64["sweeps"]))


def test_mixed_row_graded_trig(solver, orc):
    """A row-graded factor (kappa(H) huge, kappa of the scaled factor
    modest): the relative accuracy survives the FP32 preconditioning."""
    n = 256
    G = W.graded_rows(n, n, k=808, decades=4.0, cond_decades=2.0)
    got = run(solver, G, 1, 32, 1, want_V=False)
    assert got["st"] == 0
    ref = orc.jevd(G, None, n * EPS, orc.MODMODULUS, want_v=False)
    check_eigs(orc, G, None, got["lam"], ref.lam)


def test_mixed_option_rules(solver):
    from paper_1008_0201_amd import jevd
    G = dev_colmajor(np.random.default_rng(4).standard_normal((64, 64)))
    assert solver.evd(G, None, variant=0, check=False, precision=1)[4] == jevd.JEVD_EINVAL
    J = np.ones(64, dtype=np.int8)
    J[3] = -1
    assert solver.evd(G, J, variant=1, block=16, check=False, precision=1)[4] == jevd.JEVD_EINVAL
    assert solver.evd(G, None, variant=1, block=16, check=False, precision=2)[4] == jevd.JEVD_EINVAL


def test_mixed_cholesky_breakdown(solver, orc):
    """A zero column makes the pivot Cholesky break down (Sec. 2.3): in the
    FP32 sweeps such a pivot is left to the FP64 sweeps, which process it on
    the columns of G_P.  The zero column stays zero (lambda = 0, u = 0) and
    the other eigenvalues meet the gate against the oracle."""
    from paper_1008_0201_amd import jevd
    n = 256
    wl = W.graded_spd_transposed(n, k=2, lam_decades=3.0)
    G = wl.G.copy()
    G[:, 101] = 0.0
    Gd = dev_colmajor(G)
    lam, U, V, sweeps, st = solver.evd(Gd, None, variant=1, block=32, check=False, precision=1)
    info = solver.info()
    assert st == 0 and info.sweeps_low > 0 and info.breakdowns > 0
    lam, U = lam.cpu().numpy(), U.cpu().numpy()
    assert lam[101] == 0.0 and np.all(U[:, 101] == 0.0)
    ref = orc.jevd(G, None, wl.tol, orc.MODMODULUS, want_v=False)
    nz = np.arange(n) != 101
    assert ref.status == 0 and ref.lam[101] == 0.0
    check_eigs(orc, G[:, nz], None, lam[nz], ref.lam[nz])
    Vh = V.cpu().numpy()
    assert np.max(np.abs(Vh.T @ Vh - np.eye(n))) <= 10 * n * EPS
    assert jevd.JEVD_OK == 0
