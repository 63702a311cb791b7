"""Pins of the oracle's pivot orderings (Sec. 2.4, Fig. 2-3, Alg. 3.1 and the
process-map description that follows it).  CPU only."""
import itertools

import pytest


def _process_map_sweep(p):
    """Simulate one sweep of the ring of p processes over 2p block columns as
    the paper describes the process map in words (Sec. 3, after Alg. 3.1):
    processes start on the antidiagonal blocks (r+1, 2p-r); each step a
    process moves down (row index + 1, same column) until it would land on a
    diagonal block; then it keeps its column and takes the one row index no
    other process occupies; from then on it keeps that row s and walks the row
    from (s, s+1), the column growing by one a step.
    Returns the list of pair sets (1-based) of the 2p steps and the final
    positions (those of the first step of the next sweep)."""
    N = 2 * p
    pos = [(r + 1, N - r) for r in range(p)]
    row = [None] * p            # fixed row s once a process has hit the diagonal
    nxt = [None] * p            # next column of a process walking its row
    steps = [set(pos)]
    for _ in range(N):
        new = [None] * p
        hit = []
        for r, (i, j) in enumerate(pos):
            if row[r] is None:
                if i + 1 == j:
                    hit.append(r)
                else:
                    new[r] = (i + 1, j)
            else:
                assert nxt[r] <= N, "a row walk never leaves the matrix in one sweep"
                new[r] = (row[r], nxt[r])
                nxt[r] += 1
        for r in hit:
            i, j = pos[r]
            used = {x for q in range(p) if new[q] is not None for x in new[q]}
            free = [x for x in range(1, N + 1) if x not in used and x != j]
            assert len(free) == 1, "exactly one row index must be unoccupied"
            s = free[0]
            assert s < j
            new[r] = (s, j)
            row[r], nxt[r] = s, s + 1
        pos = new
        steps.append(set(pos))
    return steps[:N], steps[N]


@pytest.mark.parametrize("p", list(range(2, 41)))
def test_modified_modulus_matches_process_map(orc, p):
    steps, final = _process_map_sweep(p)
    closed = orc.ordering(2 * p, orc.MODMODULUS)
    assert len(closed) == 2 * p
    for k in range(2 * p):
        got = {(i + 1, j + 1) for (i, j) in closed[k]}
        assert got == steps[k], "step %d differs" % (k + 1)
    # after a sweep the processes are back on the antidiagonal, in reverse order
    assert final == {(r + 1, 2 * p - r) for r in range(p)}


def test_first_step_of_paper_example(orc):
    # Example 1 (Sec. 3.1): with 4 columns the first step pairs (1,4) and (2,3)
    assert {(i + 1, j + 1) for i, j in orc.ordering(4, orc.MODMODULUS)[0]} == {(1, 4), (2, 3)}
    assert {(i + 1, j + 1) for i, j in orc.ordering(4, orc.MODULUS)[0]} == {(1, 4), (2, 3)}


@pytest.mark.parametrize("n", [2, 4, 6, 8, 16, 30, 64, 128])
def test_modified_modulus_structure(orc, n):
    steps = orc.ordering(n, orc.MODMODULUS)
    p = n // 2
    assert len(steps) == n
    count = {}
    for st in steps:
        assert len(st) == p                                  # every step full
        idx = [x for pr in st for x in pr]
        assert len(set(idx)) == len(idx)                     # disjoint pivots
        for pr in st:
            assert pr[0] < pr[1]
            count[pr] = count.get(pr, 0) + 1
    allpairs = set(itertools.combinations(range(n), 2))
    assert set(count) == allpairs                            # every pair
    twice = {pr for pr, c in count.items() if c == 2}
    assert twice == {(m, m + p) for m in range(p)}           # (m, m+p) twice
    assert all(c in (1, 2) for c in count.values())


@pytest.mark.parametrize("n", [2, 4, 6, 10, 32, 100])
def test_modulus_even_each_pair_once(orc, n):
    steps = orc.ordering(n, orc.MODULUS)
    p = n // 2
    seen = []
    for k, st in enumerate(steps, start=1):
        assert len(st) == (p if k % 2 else p - 1)            # Fig. 2: n/2-1 on even
        seen.extend(st)
        idx = [x for pr in st for x in pr]
        assert len(set(idx)) == len(idx)
    assert sorted(seen) == sorted(itertools.combinations(range(n), 2))
    # the modified modulus adds exactly the pair of the two idle indices
    mm = orc.ordering(n, orc.MODMODULUS)
    for k, (a, b) in enumerate(zip(steps, mm), start=1):
        extra = set(b) - set(a)
        assert len(extra) == (1 if k % 2 == 0 else 0)
        if extra:
            assert extra == {(k // 2 - 1, k // 2 - 1 + p)}


@pytest.mark.parametrize("n", [1, 3, 5, 7, 17, 255])
def test_odd_modulus_each_pair_once(orc, n):
    for kind in (orc.MODULUS, orc.MODMODULUS):
        steps = orc.ordering(n, kind)
        assert len(steps) == n
        seen = []
        for st in steps:
            assert len(st) == (n - 1) // 2
            idx = [x for pr in st for x in pr]
            assert len(set(idx)) == len(idx)
            seen.extend(st)
        assert sorted(seen) == sorted(itertools.combinations(range(n), 2))


@pytest.mark.parametrize("n", [2, 3, 7, 64])
def test_row_cyclic(orc, n):
    steps = orc.ordering(n, orc.ROWCYCLIC)
    assert [s[0] for s in steps] == list(itertools.combinations(range(n), 2))
    assert all(len(s) == 1 for s in steps)


def test_bad_arguments(orc):
    with pytest.raises(ValueError):
        orc.ordering(0, orc.MODMODULUS)
    with pytest.raises(ValueError):
        orc.ordering(8, 7)
