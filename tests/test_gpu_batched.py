"""GPU parity of the batched solver (jevd_batch_* through the C ABI) against
the oracle, instance by instance, on seeded inputs: eigenvalues to a
relative error of 1e-12, sweep count within one of the oracle's, U
orthonormal, V^T J V = J and G_out = G_in V, as for a single solve.  The
instances span the three residencies of the kernel (G and V in LDS, G only,
neither), odd n, m > n, leading dimensions above m, n = 1 and 2.  Needs an
MI355X and the built libjevd.so."""
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
    import torch
    m, n = A.shape
    ld = m if ld is None else ld
    buf = torch.zeros((n, ld), dtype=torch.float64, device="cuda")
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T))
    return buf.T[:m, :]


def rel_err(a, b):
    a, b = np.sort(a), np.sort(b)
    den = np.where(b != 0, np.abs(b), 1.0)
    return float(np.max(np.abs(a - b) / den))


def check_instance(orc, G, J, tol, ordering, lam, U, V, Gout, sweeps, st, tag):
    ref = orc.jevd(G, J, tol, ordering, want_v=False)
    assert ref.status == 0
    assert st == 0, (tag, st)
    # the eigenvalue gate of oracle/gates.py: 1e-12 against the FP64 oracle,
    # else the bound (1.2) against the 80-bit oracle
    from oracle import gates
    n = G.shape[1]
    truth = lambda: orc.jevd(G, J, n * 1e-19, ordering, want_v=False, prec="l").lam
    res = gates.eig_gate(G, lam, ref.lam, truth)
    assert res["ok"], (tag, res)
    assert abs(sweeps - ref.sweeps) <= 1, (tag, sweeps, ref.sweeps)
    n = G.shape[1]
    if U is not None:
        nz = np.sum(U * U, axis=0) > 0
        Uv = U[:, nz]
        assert np.max(np.abs(Uv.T @ Uv - np.eye(Uv.shape[1]))) <= 10 * max(n, 2) * EPS, tag
    if V is not None:
        jj = np.ones(n) if J is None else np.asarray(J, dtype=float)
        vmax = np.max(np.sum(V * V, axis=0))
        assert np.max(np.abs(V.T @ (jj[:, None] * V) - np.diag(jj))) <= 10 * max(n, 2) * EPS * vmax, tag
        GV = (G.astype(np.longdouble) @ V.astype(np.longdouble)).astype(np.float64)
        scale = np.sqrt(np.sum((np.abs(G) @ np.abs(V)) ** 2, axis=0))
        assert np.max(np.abs(GV - Gout).sum(axis=0) / scale) <= 100 * max(n, 2) * EPS, tag


def mixed_batch():
    """Instances over every residency: n <= 100 (G and V in LDS), 100 < n <=
    140 (G only), n > 140 (global), odd and even n, m > n, padded ld."""
    g = np.random.default_rng(1008)
    specs = [(1, 1), (2, 2), (3, 5), (7, 7), (16, 16), (33, 40), (64, 64), (99, 99), (100, 100),
             (101, 101), (120, 131), (140, 140), (141, 141), (160, 200), (199, 199), (256, 256),
             (257, 300), (48, 48), (90, 91), (130, 130)]
    out = []
    for i, (n, m) in enumerate(specs):
        B = g.standard_normal((m, n))
        G = B * (10.0 ** g.uniform(-2.5, 2.5, size=n))[None, :]
        J = None
        if i % 2 == 1 and n > 1:
            J = W.random_signature(n, g)
        ld = m + (i % 3) * 5
        out.append((G, J, n * EPS, ld))
    return out


def run_batch(solver, items, ordering, want_V=True, want_U=True):
    Gd = [dev_colmajor(G, ld) for (G, J, tol, ld) in items]
    Js = [J for (G, J, tol, ld) in items]
    tols = [tol for (G, J, tol, ld) in items]
    lams, Us, Vs, sweeps, stv = solver.evd_batched(Gd, Js, tols, ordering=ordering,
                                                   want_U=want_U, want_V=want_V, check=False)

    def h(t):
        return None if t is None else t.cpu().numpy()

    return [dict(lam=h(lams[i]), U=h(Us[i]), V=h(Vs[i]), G=h(Gd[i]), sweeps=sweeps[i], st=stv[i])
            for i in range(len(items))]


@pytest.mark.parametrize("ordering", [W.MODMODULUS, W.MODULUS, W.ROWCYCLIC])
def test_batched_mixed_matches_oracle(solver, orc, ordering):
    items = mixed_batch()
    if ordering == W.ROWCYCLIC:
        items = items[:12]   # row-cyclic runs one pair at a time
    res = run_batch(solver, items, ordering)
    for i, ((G, J, tol, ld), r) in enumerate(zip(items, res)):
        check_instance(orc, G, J, tol, ordering, r["lam"], r["U"], r["V"], r["G"], r["sweeps"],
                       r["st"], "instance %d n=%d" % (i, G.shape[1]))


def test_batched_workload_recipe_sample(solver, orc):
    """A slice of the uneven-batch recipe (n in 16..256, half indefinite)."""
    wls = W.batch_uneven(count=24, k=3)
    items = [(w.G, w.J, w.tol, w.m) for w in wls]
    res = run_batch(solver, items, W.MODMODULUS, want_V=False)
    for w, r in zip(wls, res):
        check_instance(orc, w.G, w.J, w.tol, W.MODMODULUS, r["lam"], r["U"], None, r["G"],
                       r["sweeps"], r["st"], w.name)


def test_batched_matches_single_solves(solver):
    """The batched kernel and the single-matrix path compute the same
    eigenvalues (both FP64 one-sided Jacobi with the same ordering)."""
    items = mixed_batch()[8:16]
    res = run_batch(solver, items, W.MODMODULUS, want_V=False)
    for (G, J, tol, ld), r in zip(items, res):
        Gd = dev_colmajor(G)
        lam, U, V, sweeps, st = solver.evd(Gd, J, tol=tol, ordering=W.MODMODULUS, want_V=False,
                                           check=False)
        assert st == 0
        assert rel_err(r["lam"], lam.cpu().numpy()) <= REL_TOL


def test_batched_status_per_instance(solver):
    """A non-finite instance reports JEVD_ENONFINITE, a capped one
    JEVD_ENOCONV; the others still converge and are unaffected."""
    from paper_1008_0201_amd import jevd
    g = np.random.default_rng(7)
    good = g.standard_normal((50, 50))
    bad = g.standard_normal((40, 40))
    bad[3, 5] = np.nan
    Gd = [dev_colmajor(good), dev_colmajor(bad), dev_colmajor(good.copy())]
    lams, Us, Vs, sweeps, stv = solver.evd_batched(Gd, None, None, check=False)
    assert stv == [jevd.JEVD_OK, jevd.JEVD_ENONFINITE, jevd.JEVD_OK]
    assert np.array_equal(lams[0].cpu().numpy(), lams[2].cpu().numpy())
    Gd = [dev_colmajor(good), dev_colmajor(np.eye(30))]
    lams, Us, Vs, sweeps, stv = solver.evd_batched(Gd, None, None, max_sweeps=1, check=False)
    assert stv == [jevd.JEVD_ENOCONV, jevd.JEVD_OK]
    assert sweeps == [1, 1]


def test_batched_invalid_arguments(solver):
    from paper_1008_0201_amd import jevd
    g = np.random.default_rng(9)
    A = dev_colmajor(g.standard_normal((20, 20)))
    with pytest.raises(jevd.JevdError) as e:
        solver.batch_plan([A], Js=[np.ones(20, dtype=np.int8) * 2])
    assert e.value.status == jevd.JEVD_EINVAL
    wide = dev_colmajor(g.standard_normal((10, 20)))
    with pytest.raises(jevd.JevdError) as e:
        solver.batch_plan([A, wide])
    assert e.value.status == jevd.JEVD_EINVAL


@pytest.mark.parametrize("split", [False, True])
def test_batched_plan_rerun_and_graph_replay(solver, split, tmp_path):
    """A plan rerun restarts from the current G_i; a captured plan replayed
    several times (with eager work between replays) gives the eager result
    bit for bit on every replay.  split: the size classes run as three
    launches (4, 8 and 16 wavefronts), two of them on the plan's second
    stream, which the capture takes in through the fork and join events."""
    import torch
    from paper_1008_0201_amd import jevd
    items = mixed_batch()[4:14]
    if split:
        # classes 0 and 1 with more instances than CUs (so they keep the
        # table's 4 and 8 wavefronts)
        g = np.random.default_rng(77)
        for n in [int(x) for x in g.integers(8, 41, size=300)] + [int(x) for x in g.integers(49, 91, size=300)]:
            items.append((g.standard_normal((n, n)), None, n * EPS, n))
    G0 = [dev_colmajor(G) for (G, J, tol, ld) in items]
    Gd = [x.clone() for x in G0]
    if split:
        assert jevd.jevd_tune_file(str(tmp_path / "tune.txt")) == jevd.JEVD_OK
        for c, w in enumerate((4, 8, 16, 16)):
            assert jevd.jevd_batch_tune_record(c, w, 1.0) == jevd.JEVD_OK
    try:
        plan = solver.batch_plan(Gd, [J for (G, J, tol, ld) in items], None, want_V=True)
    finally:
        jevd.jevd_tune_file(None)
    assert jevd.jevd_batch_waves(plan.plan) == ([4, 8, 16, 16] if split else [16, 16, 16, 16])
    try:
        plan.run()
        st, sw_ref, stv = plan.results()
        assert st == 0
        lam_ref = [t.clone() for t in plan.lams]
        V_ref = [t.clone() for t in plan.Vs]
        for a, b in zip(Gd, G0):
            a.copy_(b)
        plan.run()
        st, sw, stv = plan.results()
        assert st == 0 and sw == sw_ref
        for a, b in zip(plan.lams, lam_ref):
            assert torch.equal(a, b)

        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            for a, b in zip(Gd, G0):
                a.copy_(b)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            plan.run(stream=s)
        torch.cuda.synchronize()
        for rep in range(3):
            for a, b in zip(Gd, G0):
                a.copy_(b)
            for t in plan.lams:
                t.fill_(0.0)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            st, sw, stv = plan.results()
            assert st == 0 and sw == sw_ref, rep
            for a, b in zip(plan.lams, lam_ref):
                assert torch.equal(a, b), rep
            for a, b in zip(plan.Vs, V_ref):
                assert torch.equal(a, b), rep
        del graph
    finally:
        plan.close()


@pytest.mark.parametrize("waves", [(4, 4, 4, 4), (8, 8, 8, 8), (16, 16, 16, 16), (4, 8, 16, 16),
                                   (16, 8, 4, 16)])
def test_batched_every_workgroup_size_matches_oracle(solver, orc, waves, tmp_path):
    """The tune table's per-class workgroup sizes (class 0 .. 3) on a batch
    of 20 instances: classes with no more instances than CUs run 16
    wavefronts whatever the table says, and give the oracle's results."""
    from paper_1008_0201_amd import jevd
    path = str(tmp_path / "tune.txt")
    try:
        assert jevd.jevd_tune_file(path) == jevd.JEVD_OK
        for c in range(jevd.BATCH_CLASSES):
            assert jevd.jevd_batch_tune_record(c, waves[c], 1.0) == jevd.JEVD_OK
        items = mixed_batch()
        plan = solver.batch_plan([dev_colmajor(G, ld) for (G, J, tol, ld) in items],
                                 [J for (G, J, tol, ld) in items], [t for (G, J, t, ld) in items])
        try:
            got = jevd.jevd_batch_waves(plan.plan)
        finally:
            plan.close()
        # a class with no more instances than CUs runs 16 wavefronts (one
        # instance per CU); this batch has 20 instances
        assert got == [16, 16, 16, 16], got
        res = run_batch(solver, items, W.MODMODULUS)
    finally:
        jevd.jevd_tune_file(None)
    for i, ((G, J, tol, ld), r) in enumerate(zip(items, res)):
        check_instance(orc, G, J, tol, W.MODMODULUS, r["lam"], r["U"], r["V"], r["G"], r["sweeps"],
                       r["st"], "waves %s instance %d n=%d" % (waves, i, G.shape[1]))


def test_batched_autotune_records_a_size_per_class(solver, tmp_path):
    from paper_1008_0201_amd import jevd
    path = str(tmp_path / "tune.txt")
    try:
        assert jevd.jevd_tune_file(path) == jevd.JEVD_OK
        got = jevd.jevd_batch_autotune(solver.h)
        assert len(got) == jevd.BATCH_CLASSES and all(w in (4, 8, 16) for w in got), got
        for c, w in enumerate(got):
            st, tw, ms = jevd.jevd_batch_tune_lookup(c)
            assert st == jevd.JEVD_OK and tw == w and ms > 0.0, (c, st, tw, ms)
        assert "batch 0 " in open(path).read()
    finally:
        jevd.jevd_tune_file(None)


@pytest.mark.parametrize("waves", [4, 8])
def test_batched_small_workgroups_on_large_classes(solver, orc, waves, tmp_path):
    """Classes with more instances than CUs run the table's workgroup size:
    300 instances of class 1 (49 <= n <= 96, G and V in LDS) and 300 of
    class 3 (n > 141: G in HBM, the register step and the V log) with 4 or 8
    wavefronts per workgroup.  Every instance: U orthonormal and, J = I,
    sum(lambda) = ||G||_F^2 (orthogonal transforms keep the Frobenius norm);
    six instances per class against the oracle."""
    import torch
    from paper_1008_0201_amd import jevd
    g = np.random.default_rng(4242 + waves)
    ns = [int(x) for x in g.integers(49, 97, size=300)] + [int(x) for x in g.integers(142, 181, size=300)]
    Gs = [g.standard_normal((n, n)) * (10.0 ** g.uniform(-1.5, 1.5, size=n))[None, :] for n in ns]
    items = [(G, None, G.shape[1] * EPS, G.shape[0]) for G in Gs]
    path = str(tmp_path / "tune.txt")
    try:
        assert jevd.jevd_tune_file(path) == jevd.JEVD_OK
        for c in range(jevd.BATCH_CLASSES):
            assert jevd.jevd_batch_tune_record(c, waves, 1.0) == jevd.JEVD_OK
        plan = solver.batch_plan([dev_colmajor(G) for G in Gs], None, None)
        try:
            got = jevd.jevd_batch_waves(plan.plan)
        finally:
            plan.close()
        assert got == [0, waves, 0, waves], got
        res = run_batch(solver, items, W.MODMODULUS)
    finally:
        jevd.jevd_tune_file(None)
    for i, (G, r) in enumerate(zip(Gs, res)):
        n = G.shape[1]
        assert r["st"] == 0, (i, r["st"])
        U = r["U"]
        assert np.max(np.abs(U.T @ U - np.eye(n))) <= 10 * n * EPS, i
        fro = float(np.sum(G.astype(np.longdouble) ** 2))
        assert abs(float(np.sum(r["lam"].astype(np.longdouble))) - fro) <= 10 * n * EPS * fro, i
    for i in list(range(6)) + list(range(300, 306)):
        G = Gs[i]
        check_instance(orc, G, None, G.shape[1] * EPS, W.MODMODULUS, res[i]["lam"], res[i]["U"],
                       res[i]["V"], res[i]["G"], res[i]["sweeps"], res[i]["st"],
                       "waves %d instance %d n=%d" % (waves, i, G.shape[1]))
