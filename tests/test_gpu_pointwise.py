"""GPU parity of the pointwise path (through the C ABI) against the oracle,
on the same seeded inputs: eigenvalues to a relative error of 1e-12, the
same sweep count within one, orthogonality of U within 10 n eps, V^T J V = J
and G_out = G_in V.  Needs an MI355X and the built libjevd.so."""
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
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    s = jevd.Solver()
    yield s
    s.close()


def dev_colmajor(A, ld=None):
    """Column-major float64 device copy of A (m x n), optionally with ld > m."""
    import torch
    m, n = A.shape
    ld = m if ld is None else ld
    buf = torch.zeros((n, ld), dtype=torch.float64, device="cuda")
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T))
    return buf.T[:m, :]


def host(t):
    return t.detach().cpu().numpy() if t is not None else None


def run_gpu(solver, G, J, tol, ordering, variant=0, want_V=True, ld=None, max_sweeps=50, **kw):
    Gd = dev_colmajor(G, ld)
    lam, U, V, sweeps, st = solver.evd(Gd, J, tol=tol, ordering=ordering, variant=variant,
                                       want_V=want_V, max_sweeps=max_sweeps, check=False, **kw)
    info = solver.info()
    return dict(st=st, lam=host(lam), U=host(U), V=host(V), G=host(Gd), sweeps=sweeps,
                rot=[info.rotations[i] for i in range(min(sweeps, 64))], info=info)


def rel_err(a, b):
    a, b = np.sort(a), np.sort(b)
    den = np.where(b != 0, np.abs(b), 1.0)
    return float(np.max(np.abs(a - b) / den))


def check_against_oracle(orc, G, J, tol, ordering, got, sweep_slack=1):
    ref = orc.jevd(G, J, tol, ordering, want_v=False)
    assert ref.status == 0
    assert got["st"] == 0, got["st"]
    assert rel_err(got["lam"], ref.lam) <= REL_TOL
    assert abs(got["sweeps"] - ref.sweeps) <= sweep_slack, (got["sweeps"], ref.sweeps)
    n = G.shape[1]
    if got["U"] is not None:
        Uv = got["U"]
        nz = np.sum(Uv * Uv, axis=0) > 0
        Uv = Uv[:, nz]
        assert np.max(np.abs(Uv.T @ Uv - np.eye(Uv.shape[1]))) <= 10 * n * EPS
    if got["V"] is not None:
        jj = np.ones(n) if J is None else np.asarray(J, dtype=float)
        V = got["V"]
        vmax = np.max(np.sum(V * V, axis=0))
        assert np.max(np.abs(V.T @ (jj[:, None] * V) - np.diag(jj))) <= 10 * n * EPS * vmax
        GV = (G.astype(np.longdouble) @ V.astype(np.longdouble)).astype(np.float64)
        scale = np.sqrt(np.sum((np.abs(G) @ np.abs(V)) ** 2, axis=0))
        assert np.max(np.abs(GV - got["G"]).sum(axis=0) / scale) <= 100 * n * EPS
    return ref


def test_small_spd_rowcyclic_n64(solver, orc):
    """H = G G^T, G 64 x 64 N(0,1), row-cyclic, tol 64 eps: the small workload."""
    wl = W.spd_gaussian(64, tol_factor=64)
    got = run_gpu(solver, wl.G, wl.J, wl.tol, W.ROWCYCLIC)
    ref = check_against_oracle(orc, wl.G, wl.J, wl.tol, W.ROWCYCLIC, got)
    print("n=64 row-cyclic sweeps gpu %d oracle %d" % (got["sweeps"], ref.sweeps))


@pytest.mark.parametrize("m,n,ld,want_V", [(1, 1, None, True), (2, 2, None, True),
                                            (3, 3, None, True), (5, 3, 9, True),
                                            (9, 8, None, True), (17, 17, None, False),
                                            (40, 33, 41, True), (64, 50, None, True),
                                            (64, 64, 70, True), (64, 64, None, False),
                                            (65, 65, None, True), (100, 90, None, True)])
@pytest.mark.parametrize("indef", [False, True])
def test_rowcyclic_small(solver, orc, m, n, ld, want_V, indef):
    """The row-cyclic ordering run as its steps of equal p + q in one
    workgroup: for m, n <= 64 four pairs per wavefront (16 lanes a pair, 1,
    2, 4 or 8 wavefronts), above that the step table of the general
    single-workgroup solve.  Graded columns, odd and ragged shapes, a padded
    leading dimension, with and without V, J = I and mixed signs;
    eigenvalues, sweep count, U, V and G V against the oracle (one pair at a
    time in row order)."""
    g = np.random.default_rng(3000 + 100 * m + n + 7 * indef)
    G = g.standard_normal((m, n)) * (10.0 ** g.uniform(-2, 2, size=n))[None, :]
    J = None
    if indef and n > 1:
        J = np.ones(n, dtype=np.int8)
        J[g.permutation(n)[: n // 2]] = -1
    got = run_gpu(solver, G, J, n * EPS, W.ROWCYCLIC, want_V=want_V, ld=ld)
    assert (got["V"] is None) == (not want_V)
    check_against_oracle(orc, G, J, n * EPS, W.ROWCYCLIC, got)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 33, 64, 100, 128])
@pytest.mark.parametrize("indef", [False, True])
def test_small_modmod_single_workgroup(solver, orc, n, indef):
    g = np.random.default_rng(n + 1000 * indef)
    m = n + (3 if n % 2 else 0)
    G = g.standard_normal((m, n)) * (10.0 ** g.uniform(-3, 3, size=n))[None, :]
    J = None
    if indef:
        J = np.ones(n, dtype=np.int8)
        J[g.permutation(n)[: n // 2]] = -1
    got = run_gpu(solver, G, J, n * EPS, W.MODMODULUS)
    check_against_oracle(orc, G, J, n * EPS, W.MODMODULUS, got)


@pytest.mark.parametrize("m,n", [(130, 130), (200, 200), (257, 257), (300, 257), (1100, 260)])
@pytest.mark.parametrize("indef", [False, True])
def test_pair_step_path(solver, orc, m, n, indef):
    """n > 128: one launch per parallel step (several tiles and a ragged tail
    of rows, odd n)."""
    wl = W.graded_hyperbolic(n, k=200 + n, m=m, grade=2.0)
    J = wl.J if indef else None
    got = run_gpu(solver, wl.G, J, wl.tol, W.MODMODULUS)
    check_against_oracle(orc, wl.G, J, wl.tol, W.MODMODULUS, got)


@pytest.mark.parametrize("ordering", [W.MODULUS, W.ROWCYCLIC])
def test_other_orderings(solver, orc, ordering):
    """n = 150 with V does not fit one workgroup's LDS: one launch per step
    (for row-cyclic the 297 steps of equal p + q)."""
    wl = W.graded_hyperbolic(150, k=31, grade=1.5)
    got = run_gpu(solver, wl.G, wl.J, wl.tol, ordering)
    check_against_oracle(orc, wl.G, wl.J, wl.tol, ordering, got)


def test_leading_dimension_and_no_v(solver, orc):
    wl = W.graded_hyperbolic(160, k=41)
    got = run_gpu(solver, wl.G, wl.J, wl.tol, W.MODMODULUS, want_V=False, ld=173)
    assert got["V"] is None
    check_against_oracle(orc, wl.G, wl.J, wl.tol, W.MODMODULUS, got)


def test_hyperbolic_graded_n1024_full_size(solver, orc):
    """The benchmark workload at full size: G = B diag(10^U(-3,3)), 1024 x 1024,
    J = diag(+1 x 512, -1 x 512), modified modulus, tol = n eps."""
    wl = W.graded_hyperbolic(1024)
    got = run_gpu(solver, wl.G, wl.J, wl.tol, W.MODMODULUS)
    # two steps of the ring per launch (n a multiple of 4, 512 < m <= 1024)
    assert got["info"].steps_per_launch == 2 and got["info"].v_deferred == 1
    ref = check_against_oracle(orc, wl.G, wl.J, wl.tol, W.MODMODULUS, got)
    print("n=1024 hyperbolic sweeps gpu %d oracle %d, rel err %.3e" %
          (got["sweeps"], ref.sweeps, rel_err(got["lam"], ref.lam)))


@pytest.mark.parametrize("m,n,want_V,spl", [(600, 520, True, 2), (1024, 516, False, 2),
                                             (514, 514, True, 1), (512, 512, True, 1),
                                             (1100, 520, True, 1), (700, 602, True, 1)])
def test_ring_two_step_launches(solver, orc, m, n, want_V, spl):
    """Two ring steps per launch where n is a multiple of 4 and 512 < m <=
    1024 (each workgroup also runs the next process of the ring and hands
    its column on through LDS; G alternates between two buffers), one step
    per launch elsewhere; against the oracle either way."""
    g = np.random.default_rng(m + 7 * n)
    G = g.standard_normal((m, n)) * (10.0 ** g.uniform(-2, 2, size=n))[None, :]
    J = np.ones(n, dtype=np.int8)
    J[g.permutation(n)[: n // 3]] = -1
    got = run_gpu(solver, G, J, n * EPS, W.MODMODULUS, want_V=want_V)
    assert got["info"].steps_per_launch == spl
    check_against_oracle(orc, G, J, n * EPS, W.MODMODULUS, got)


def test_status_paths(solver, orc):
    g = np.random.default_rng(9)
    G = g.standard_normal((40, 36))
    # not converged after one sweep: ENOCONV with the current iterate
    got = run_gpu(solver, G, None, 0.0, W.MODMODULUS, max_sweeps=1)
    assert got["st"] == -3 and got["sweeps"] == 1
    # NaN input: ENONFINITE
    G2 = G.copy()
    G2[5, 7] = np.nan
    got = run_gpu(solver, G2, None, 0.0, W.MODMODULUS)
    assert got["st"] == -2
    # zero column: lambda 0, u 0
    G3 = G.copy()
    G3[:, 4] = 0.0
    got = run_gpu(solver, G3, None, 0.0, W.MODMODULUS)
    assert got["st"] == 0 and got["lam"][4] == 0 and np.all(got["U"][:, 4] == 0)


@pytest.mark.parametrize("n", [96, 200])
def test_resume_from_iterate(solver, orc, n):
    import torch
    wl = W.graded_hyperbolic(n, k=55)
    full = run_gpu(solver, wl.G, wl.J, wl.tol, W.MODMODULUS)
    Gd = dev_colmajor(wl.G)
    _, _, V, sw1, st = solver.evd(Gd, wl.J, tol=wl.tol, max_sweeps=3, check=False)
    assert st == -3 and sw1 == 3
    lam, U, V2, sw2, st = solver.evd(Gd, wl.J, tol=wl.tol, V0=V, check=False)
    assert st == 0
    assert rel_err(host(lam), full["lam"]) <= 1e-13
    assert abs(sw1 + sw2 - full["sweeps"]) <= 1
    assert torch.allclose(V2, torch.from_numpy(full["V"]).cuda(), rtol=0, atol=1e-10 * float(np.abs(full["V"]).max()))


def test_u_aliases_g(solver, orc):
    import torch
    from paper_1008_0201_amd import jevd
    wl = W.graded_hyperbolic(140, k=61)
    Gd = dev_colmajor(wl.G)
    lam = torch.empty(140, dtype=torch.float64, device="cuda")
    st, sw = jevd.jacobi_evd(solver.h, 140, 140, Gd.data_ptr(), 140, wl.J.tobytes(), 0.0, None,
                             lam.data_ptr(), Gd.data_ptr(), 140, 0, 140)
    assert st == 0
    Uv = host(Gd)
    assert np.max(np.abs(Uv.T @ Uv - np.eye(140))) <= 10 * 140 * EPS
    ref = orc.jevd(wl.G, wl.J, wl.tol, W.MODMODULUS, want_v=False)
    assert rel_err(host(lam), ref.lam) <= REL_TOL


@pytest.mark.parametrize("n,indef", [(3000, True), (4200, False)])
def test_deferred_v_in_several_log_runs(solver, n, indef):
    """V updated from the rotation log: at n = 3000 (four rows of V per
    workgroup) a sweep's log exceeds its 64 MiB cap and is applied in two
    runs, at n = 4200 (two rows per workgroup) in three.  G's iteration must
    not depend on V (the same lambda, bit for bit, and the same rotation
    counts as without V), V^T J V = J and G_out = G_in V (products in FP64,
    whose error is within the bound)."""
    wl = W.graded_hyperbolic(n, k=300 + n, grade=1.0)
    J = wl.J if indef else None
    got = run_gpu(solver, wl.G, J, wl.tol, W.MODMODULUS)
    nov = run_gpu(solver, wl.G, J, wl.tol, W.MODMODULUS, want_V=False)
    assert got["st"] == 0 and nov["st"] == 0
    assert got["sweeps"] == nov["sweeps"] and got["rot"] == nov["rot"]
    assert np.array_equal(got["lam"], nov["lam"])
    jj = np.ones(n) if J is None else np.asarray(J, dtype=float)
    V = got["V"]
    vmax = np.max(np.sum(V * V, axis=0))
    assert np.max(np.abs(V.T @ (jj[:, None] * V) - np.diag(jj))) <= 10 * n * EPS * vmax
    scale = np.sqrt(np.sum((np.abs(wl.G) @ np.abs(V)) ** 2, axis=0))
    assert np.max(np.abs(wl.G @ V - got["G"]).sum(axis=0) / scale) <= 100 * n * EPS


def test_deferred_v_exits(solver):
    """The exits of the multi-launch path with V updated from the rotation
    log: after max_sweeps (ENOCONV) V is complete and consistent with the
    iterate (G_out = G_in V); a NaN input gives ENONFINITE; the next solve on
    the same handle is unaffected (the same result as on a fresh handle)."""
    from paper_1008_0201_amd import jevd
    n = 300
    wl = W.graded_hyperbolic(n, k=77, grade=1.5)
    got = run_gpu(solver, wl.G, wl.J, wl.tol, W.MODMODULUS, max_sweeps=2)
    assert got["st"] == -3 and got["sweeps"] == 2
    assert got["info"].v_deferred == 1
    V = got["V"]
    scale = np.sqrt(np.sum((np.abs(wl.G) @ np.abs(V)) ** 2, axis=0))
    assert np.max(np.abs(wl.G @ V - got["G"]).sum(axis=0) / scale) <= 100 * n * EPS
    bad = wl.G.copy()
    bad[7, 11] = np.nan
    assert run_gpu(solver, bad, wl.J, wl.tol, W.MODMODULUS)["st"] == -2
    again = run_gpu(solver, wl.G, wl.J, wl.tol, W.MODMODULUS)
    fresh_solver = jevd.Solver()
    try:
        fresh = run_gpu(fresh_solver, wl.G, wl.J, wl.tol, W.MODMODULUS)
    finally:
        fresh_solver.close()
    assert again["st"] == 0 and fresh["st"] == 0
    assert np.array_equal(again["lam"], fresh["lam"]) and np.array_equal(again["V"], fresh["V"])


def test_deferred_v_with_padded_leading_dimensions(solver):
    """The rotation log applied to a V with ldv > n (and G with ldg > m):
    the same V, bit for bit, as with packed buffers, and the padding rows
    untouched."""
    import torch
    from paper_1008_0201_amd import jevd
    n = 260
    wl = W.graded_hyperbolic(n, k=91, grade=1.5)
    ref = run_gpu(solver, wl.G, wl.J, wl.tol, W.MODMODULUS)
    assert ref["st"] == 0 and ref["info"].v_deferred == 1
    ldg, ldv = n + 5, n + 7
    Gd = dev_colmajor(wl.G, ldg)
    lam = torch.empty(n, dtype=torch.float64, device="cuda")
    Ub = torch.empty((n, ldg), dtype=torch.float64, device="cuda")
    Vb = torch.full((n, ldv), 7.0, dtype=torch.float64, device="cuda")
    st, sw = jevd.jacobi_evd(solver.h, n, n, Gd.data_ptr(), ldg, wl.J.tobytes(), wl.tol, None,
                             lam.data_ptr(), Ub.data_ptr(), ldg, Vb.data_ptr(), ldv)
    assert st == 0 and sw == ref["sweeps"]
    Vh = host(Vb)
    assert np.array_equal(Vh[:, :n].T, ref["V"])
    assert np.all(Vh[:, n:] == 7.0)
    assert np.array_equal(host(lam), ref["lam"])
