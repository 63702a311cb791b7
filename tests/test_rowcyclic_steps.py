"""The row-cyclic ordering (Sec. 2.4) as the solver runs it: 2n - 3 steps of
the pairs with equal i + j.  Two checks on the CPU:
  * the library's steps hold every pair once, the pairs of a step are
    disjoint, and every column meets its partners in row order (the
    oracle's one-pair-a-step sequence);
  * one-sided Jacobi driven by the two schedules -- all pairs of a step
    computed from the state at the step's start and then applied, against
    one pair at a time in row order -- gives the same G and V to the bit
    (the oracle's 2x2 transform, J = I and indefinite J)."""
import numpy as np
import pytest

from paper_1008_0201_amd import jevd as B


def partners(order, n):
    d = {c: [] for c in range(n)}
    for i, j in order:
        d[i].append(j)
        d[j].append(i)
    return d


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 8, 17, 64, 129])
def test_rowcyclic_steps_keep_each_columns_row_order(orc, n):
    steps = B.jevd_ordering(n, B.ORD_ROWCYCLIC)
    seq = [pr for st in orc.ordering(n, orc.ROWCYCLIC) for pr in st]
    assert len(steps) == max(2 * n - 3, 0)
    flat = [pr for st in steps for pr in st]
    assert all(i < j for i, j in flat)
    assert sorted(flat) == sorted(seq) and len(flat) == n * (n - 1) // 2
    for st in steps:
        cols = [c for pr in st for c in pr]
        assert len(cols) == len(set(cols))
    assert partners(flat, n) == partners(seq, n)


def sweep(orc, G, V, J, steps, tol):
    """One sweep; the pairs of a step see the state at the step's start."""
    rot = 0
    for st in steps:
        upd = []
        for p, q in st:
            x, y = G[:, p], G[:, q]
            app, aqq, apq = float(x @ x), float(y @ y), float(x @ y)
            if app == 0.0 or aqq == 0.0 or not abs(apq) > tol * np.sqrt(app) * np.sqrt(aqq):
                continue
            same = J[p] == J[q]
            c, s, _ = orc.rotation(app, aqq, apq, same)
            upd.append((p, q, c, s, same))
        for p, q, c, s, same in upd:
            for M in (G, V):
                x, y = M[:, p].copy(), M[:, q].copy()
                M[:, p] = c * x - s * y if same else c * x + s * y
                M[:, q] = s * x + c * y
            rot += 1
    return rot


@pytest.mark.parametrize("n,indef", [(6, False), (9, False), (16, True), (23, True)])
def test_rowcyclic_steps_give_the_sequential_result_bit_for_bit(orc, n, indef):
    g = np.random.default_rng(1008 + n)
    G0 = g.standard_normal((n + 3, n)) * (10.0 ** g.uniform(-2, 2, size=n))[None, :]
    J = np.ones(n, dtype=int)
    if indef:
        J[g.permutation(n)[: n // 3]] = -1
    tol = n * np.finfo(float).eps
    seq = [[pr] for st in orc.ordering(n, orc.ROWCYCLIC) for pr in st]
    grouped = B.jevd_ordering(n, B.ORD_ROWCYCLIC)
    Ga, Va, Gb, Vb = G0.copy(), np.eye(n), G0.copy(), np.eye(n)
    for s in range(30):
        ra = sweep(orc, Ga, Va, J, seq, tol)
        rb = sweep(orc, Gb, Vb, J, grouped, tol)
        assert ra == rb, s
        assert np.array_equal(Ga, Gb) and np.array_equal(Va, Vb), s
        if ra == 0:
            break
    assert ra == 0 and s >= 3
