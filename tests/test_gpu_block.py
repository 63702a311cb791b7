"""GPU parity of the block path (Gram and update on FP64 MFMA, Cholesky and
inner sweeps per pivot) against the block oracle, which runs the same block
ordering, inner orderings and skip rule on the same seeded inputs:
eigenvalues to a relative error of 1e-12, sweep counts within one, U
orthogonal within 10 n eps, V^T J V = J and G_out = G_in V."""
import numpy as np
import pytest

from paper_1008_0201_amd import workloads as W

pytestmark = pytest.mark.gpu
EPS = W.DBL_EPS
REL_TOL = 1e-12


@pytest.fixture(scope="module")
def solver():
    import torch
    from paper_1008_0201_amd import jevd
    assert torch.cuda.is_available()
    s = jevd.Solver()
    yield s
    s.close()


def dev_colmajor(A):
    import torch
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().T


def rel_err(a, b):
    a, b = np.sort(a), np.sort(b)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def run(solver, G, J, tol, variant, b, want_V=True, max_sweeps=50):
    Gd = dev_colmajor(G)
    lam, U, V, sweeps, st = solver.evd(Gd, J, tol=tol, variant=variant, block=b, want_V=want_V,
                                       max_sweeps=max_sweeps, check=False)
    info = solver.info()
    return dict(st=st, lam=lam.cpu().numpy(), U=U.cpu().numpy(),
                V=None if V is None else V.cpu().numpy(), G=Gd.cpu().numpy(), sweeps=sweeps,
                info=info)


def check_eigs(orc, G, J, lam_gpu, lam_ref):
    """The eigenvalue gate of oracle/gates.py, fixed in advance: 1e-12
    against the FP64 oracle; where that fails, the GPU must meet the
    relative accuracy bound (1.2), 64 n u kappa_2(B), against a binary128
    run of the oracle (80-bit above n = 192, where binary128 is too slow)."""
    from oracle import gates
    n = G.shape[1]
    prec, tiny = ("q", 1e-32) if n <= 192 else ("l", 1e-19)
    truth = lambda: orc.jevd(G, J, n * tiny, orc.MODMODULUS, want_v=False, prec=prec).lam
    res = gates.eig_gate(G, lam_gpu, lam_ref, truth)
    assert res["ok"], res
    return res


def check(orc, G, J, tol, b, full_block, got):
    ref = orc.block_jevd(G, J, tol, b=b, full_block=full_block, want_v=True, nthreads=0)
    assert ref.status == 0 and got["st"] == 0, (ref.status, got["st"])
    check_eigs(orc, G, J, got["lam"], ref.lam)
    assert abs(got["sweeps"] - ref.sweeps) <= 1, (got["sweeps"], ref.sweeps)
    n = G.shape[1]
    Uv = got["U"]
    assert np.max(np.abs(Uv.T @ Uv - np.eye(n))) <= 10 * n * EPS
    if got["V"] is not None:
        jj = np.ones(n) if J is None else np.asarray(J, dtype=float)
        V = got["V"]
        vmax = np.max(np.sum(V * V, axis=0))
        dev = np.max(np.abs(V.T @ (jj[:, None] * V) - np.diag(jj)))
        # Every rotation applied to a column of V adds rounding error, so the
        # loss of J-orthogonality grows with the number of stages (A.7), and
        # full block applies many inner sweeps per step.  Gate: 10 n eps, or
        # within 4x of the oracle's own loss on the same input.
        Vr = ref.V
        dev_ref = np.max(np.abs(Vr.T @ (jj[:, None] * Vr) - np.diag(jj)))
        assert dev <= max(10 * n * EPS * vmax, 4 * dev_ref)
        GV = (G.astype(np.longdouble) @ V.astype(np.longdouble)).astype(np.float64)
        scale = np.sqrt(np.sum((np.abs(G) @ np.abs(V)) ** 2, axis=0))
        assert np.max(np.abs(GV - got["G"]).sum(axis=0) / scale) <= 100 * n * EPS
    return ref


@pytest.mark.parametrize("n,m,b", [(64, 64, 16), (128, 128, 32), (128, 200, 16), (256, 256, 32),
                                   (320, 333, 32), (256, 256, 64), (384, 400, 64)])
@pytest.mark.parametrize("full_block", [False, True])
def test_block_trig_row_graded(solver, orc, n, m, b, full_block):
    """J = I, row-graded factor (the block workload's recipe at small size)."""
    G = W.graded_rows(m, n, k=300 + n + m, decades=4.0, cond_decades=3.0)
    got = run(solver, G, None, n * EPS, 2 if full_block else 1, b)
    ref = check(orc, G, None, n * EPS, b, full_block, got)
    print("n=%d b=%d fb=%d sweeps gpu %d oracle %d" % (n, b, full_block, got["sweeps"], ref.sweeps))


@pytest.mark.parametrize("n,b", [(128, 16), (256, 32), (512, 64)])
@pytest.mark.parametrize("full_block", [False, True])
def test_block_hyperbolic(solver, orc, n, b, full_block):
    """Block hyperbolic with unpivoted Cholesky (Alg. 3.4, HB / HF)."""
    wl = W.graded_hyperbolic(n, k=400 + n, grade=2.0)
    got = run(solver, wl.G, wl.J, wl.tol, 2 if full_block else 1, b)
    check(orc, wl.G, wl.J, wl.tol, b, full_block, got)


@pytest.mark.parametrize("variant", [1, 2])
def test_block_matches_pointwise_definition(solver, orc, variant):
    """The block workload's recipe at n = 512 (the solver receives G^T, with
    lam = 10^U(-3,0)): the block path's eigenvalues against the pointwise
    oracle, the definition of the result independent of the ordering."""
    wl = W.graded_spd_transposed(512, k=2, lam_decades=3.0)
    got = run(solver, wl.G, None, wl.tol, variant, 32, want_V=False)
    assert got["st"] == 0
    ref = orc.jevd(wl.G, None, wl.tol, orc.MODMODULUS, want_v=False)
    check_eigs(orc, wl.G, None, got["lam"], ref.lam)


@pytest.mark.parametrize("variant", [1, 2])
def test_block_literal_recipe_lam6(solver, orc, variant):
    """The block workload's recipe taken literally (lam = 10^U(-6,0), so
    kappa(Q diag(lam) Q^T) = 1e6) at n = 512, b = 64: the FP64 oracle itself
    is not within 1e-12 of the exact eigenvalues there, so the gate fixed in
    advance decides by its second test, the relative accuracy bound (1.2),
    64 n u kappa_2(B), against the 80-bit oracle."""
    wl = W.graded_spd_transposed(512, k=2, lam_decades=6.0)
    got = run(solver, wl.G, None, wl.tol, variant, 64, want_V=False)
    assert got["st"] == 0
    ref = orc.block_jevd(wl.G, None, wl.tol, b=64, full_block=variant == 2, want_v=False,
                         nthreads=0)
    res = check_eigs(orc, wl.G, None, got["lam"], ref.lam)
    print("n=512 literal recipe (lam 1e-6..1) variant %d: %s" % (variant, res))


def test_block_workload_recipe_small(solver, orc):
    """The block workload's recipe at n = 1024 against the block oracle
    (same ordering, b = 32, block-oriented)."""
    wl = W.graded_spd_transposed(1024, k=2, lam_decades=3.0)
    got = run(solver, wl.G, None, wl.tol, 1, 32)
    ref = check(orc, wl.G, None, wl.tol, 32, False, got)
    print("n=1024 block workload recipe: sweeps gpu %d oracle %d" % (got["sweeps"], ref.sweeps))


@pytest.mark.parametrize("b", [32, 64])
@pytest.mark.parametrize("full_block", [False, True])
def test_block_cholesky_breakdown_path(solver, orc, full_block, b):
    """A zero column gives a pivot Gram a zero diagonal entry, so its Cholesky
    factorisation breaks down on both sides (deterministically); that pivot
    is then processed on the columns of G_P itself, with V_P still
    accumulated for V."""
    n = 128
    G = W.graded_rows(n + 8, n, k=77, decades=2.0, cond_decades=2.0)
    G[:, 37] = 0.0
    got = run(solver, G, None, n * EPS, 2 if full_block else 1, b)
    ref = orc.block_jevd(G, None, n * EPS, b=b, full_block=full_block, want_v=True)
    assert ref.extra > 0 and got["info"].breakdowns > 0
    assert ref.status == 0 and got["st"] == 0
    assert got["lam"][37] == 0.0 and np.all(got["U"][:, 37] == 0.0)
    nz = np.arange(n) != 37
    check_eigs(orc, G[:, nz], None, got["lam"][nz], ref.lam[nz])
    V = got["V"]
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= max(10 * n * EPS, 4 * np.max(np.abs(ref.V.T @ ref.V - np.eye(n))))
    GV = (G.astype(np.longdouble) @ V.astype(np.longdouble)).astype(np.float64)
    scale = np.sqrt(np.sum((np.abs(G) @ np.abs(V)) ** 2, axis=0))
    scale[scale == 0] = 1.0
    assert np.max(np.abs(GV - got["G"]).sum(axis=0) / scale) <= 100 * n * EPS


def test_block_status_paths(solver, orc):
    G = W.graded_rows(128, 128, k=9, decades=2.0)
    got = run(solver, G, None, 0.0, 1, 32, max_sweeps=1)
    assert got["st"] == -3 and got["sweeps"] == 1
    G2 = G.copy()
    G2[3, 70] = np.inf
    got = run(solver, G2, None, 0.0, 1, 32)
    assert got["st"] == -2


@pytest.mark.parametrize("n,b,full_block", [(1000, 32, False), (1030, 64, False), (1030, 64, True),
                                            (1000, 16, True)])
def test_block_uneven_partition(solver, orc, n, b, full_block):
    """n not divisible by 2b: N = 2 ceil(n / 2b) blocks whose widths differ by
    at most one (Sec. 3), e.g. 32 blocks of 31 or 32 columns for n = 1000,
    b = 32, and 18 blocks of 57 or 58 for n = 1030, b = 64.  The GPU pads
    each block to b positions (empty ones carry identity rows of the pivot
    Gram and transform); the oracle works on the exact widths, so the inner
    orders differ and the results agree to the eigenvalue gate, not bit for
    bit."""
    wl = W.graded_spd_transposed(n, k=2, lam_decades=3.0)
    got = run(solver, wl.G, None, wl.tol, 2 if full_block else 1, b)
    ref = check(orc, wl.G, None, wl.tol, b, full_block, got)
    print("n=%d b=%d fb=%d uneven: sweeps gpu %d oracle %d" % (n, b, full_block, got["sweeps"],
                                                               ref.sweeps))


@pytest.mark.parametrize("n,m,b,full_block", [(300, 300, 32, False), (300, 317, 32, True),
                                              (70, 70, 32, False), (200, 200, 64, True)])
def test_block_uneven_hyperbolic(solver, orc, n, m, b, full_block):
    """Ragged block partitions on indefinite inputs, including blocks far
    narrower than b (n = 70, b = 32: four blocks of 17 or 18 columns)."""
    wl = W.graded_hyperbolic(n, k=450 + n, grade=2.0, m=m)
    got = run(solver, wl.G, wl.J, wl.tol, 2 if full_block else 1, b)
    check(orc, wl.G, wl.J, wl.tol, b, full_block, got)


def test_mfma_rate_diagnostic(solver):
    """jevd_mfma_f64_rate (the register-only FP64 MFMA rate the bench reports
    beside the roofline) returns a positive rate below the published peak
    of 78.6 TFLOP/s, not lower with more wavefronts per SIMD by much."""
    from paper_1008_0201_amd import jevd
    r = {w: jevd.jevd_mfma_f64_rate(solver.h, w, 512) for w in (1, 2, 4)}
    for w, t in r.items():
        assert 1.0 < t < 78.6 * 1.05, (w, t)
    assert r[4] >= 0.8 * r[1], r
