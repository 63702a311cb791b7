"""The property the two-steps-per-launch pointwise kernel relies on, checked
on the library's step table of the modified modulus ordering (the ring of
Alg. 3.1, pairs listed by workgroup slot; slot b runs process
(b % 8) (p / 8) + b / 8 when 8 divides p = n / 2, else process b):
  * from one step to the next, process r keeps one of its columns and takes
    the other from process r + 1 (mod p), at every step of the sweep;
  * in a launch of two steps, workgroup b (the process of slot b and the one
    after it) hands over exactly the column the first group needs, and the
    owners' final pairs cover every column once (every column is written to
    the second buffer)."""
import pytest

from paper_1008_0201_amd import jevd as B


def slot_process(b, p):
    return (b % 8) * (p // 8) + b // 8 if p % 8 == 0 else b


@pytest.mark.parametrize("n", [8, 12, 16, 20, 64, 100, 256, 1024])
def test_ring_process_receives_from_the_next(n):
    p = n // 2
    tab = B.jevd_ordering(n, B.ORD_MODMODULUS)
    assert len(tab) == n and all(len(st) == p for st in tab)
    proc_pairs = [[None] * p for _ in range(n)]
    for k in range(n):
        for b, pq in enumerate(tab[k]):
            proc_pairs[k][slot_process(b, p)] = tuple(pq)
    for k in range(n - 1):
        holder = {}
        for r, (i, j) in enumerate(proc_pairs[k]):
            holder[i] = r
            holder[j] = r
        for r, (i, j) in enumerate(proc_pairs[k + 1]):
            kept = set((i, j)) & set(proc_pairs[k][r])
            assert len(kept) == 1, (n, k, r)
            (new,) = set((i, j)) - kept
            assert holder[new] == (r + 1) % p, (n, k, r, holder[new])


@pytest.mark.parametrize("n", [8, 12, 64, 100, 1024])
def test_two_step_launch_covers_every_column(n):
    p = n // 2
    tab = B.jevd_ordering(n, B.ORD_MODMODULUS)
    proc = [[None] * p for _ in range(n)]
    for k in range(n):
        for b, pq in enumerate(tab[k]):
            proc[k][slot_process(b, p)] = tuple(pq)
    for k0 in range(0, n, 2):
        written = []
        for b in range(p):
            r = slot_process(b, p)
            own0, nxt0, own1 = proc[k0][r], proc[k0][(r + 1) % p], proc[k0 + 1][r]
            kept = set(own0) & set(own1)
            (given,) = set(nxt0) - set(proc[k0 + 1][(r + 1) % p])
            assert set(own1) == kept | {given}, (n, k0, b)
            written += list(own1)
        assert sorted(written) == list(range(n)), (n, k0)
