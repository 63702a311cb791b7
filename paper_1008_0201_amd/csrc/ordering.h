// Host-side pivot orderings of the solver.
#pragma once
#include <vector>

namespace jevd {

enum { kOrdRowCyclic = 0, kOrdModulus = 1, kOrdModModulus = 2 };

// Fills step_start (nsteps + 1 offsets) and pairs (2 ints per pair, 0-based,
// i < j).  Returns the number of steps, or -1 for bad arguments.
int build_ordering(int n, int ordering, std::vector<int> &step_start, std::vector<int> &pairs);

// Pairs of step k (1-based, 1..N) of the modulus family over N columns,
// enumerated by slot r: first the antidiagonal i + j = k (i = 1, 2, ...),
// then i + j = k + N (i = k, k+1, ...), then for the modified modulus on even
// N and even k the extra pair (k/2, k/2 + N/2).  Returns 0-based (i, j),
// i < j.  modulus_step_pairs(N, k, modified) gives the count.
#if defined(__HIPCC__)
#define JEVD_HD __host__ __device__
#else
#define JEVD_HD
#endif
JEVD_HD inline int modulus_step_pairs(int N, int k, bool modified)
{
    const int c1 = (k - 1) / 2;
    const int c2 = (k + N + 1) / 2 - k;
    return c1 + (c2 > 0 ? c2 : 0) + ((modified && N % 2 == 0 && k % 2 == 0) ? 1 : 0);
}
JEVD_HD inline void modulus_pair(int N, int k, int r, int *i0, int *j0)
{
    const int c1 = (k - 1) / 2;
    if (r < c1) {
        *i0 = r;              // i = r + 1 (1-based)
        *j0 = k - r - 2;      // j = k - i
        return;
    }
    r -= c1;
    const int c2 = (k + N + 1) / 2 - k;
    if (r < c2) {
        *i0 = k + r - 1;      // i = k + r
        *j0 = N - r - 1;      // j = k + N - i
        return;
    }
    *i0 = k / 2 - 1;          // the extra pair of the modified modulus
    *j0 = k / 2 + N / 2 - 1;
}

// Row-cyclic ordering (Sec. 2.4) as steps of disjoint pairs: step t =
// 1 .. 2N - 3 holds the pairs (i, j), i < j, with i + j == t (0-based),
// i = max(0, t - N + 1), ... .  Every pair that shares a column with (i, j)
// and precedes it in row order, (i', i) and (i', j) with i' < i or (i, j')
// with j' < j, has a smaller i + j, and every one that follows it a larger
// one, so each column meets its transforms in row order with the same
// operands; the transforms of one step touch disjoint columns and commute.
// The result is that of the pairs taken one at a time in row order.
JEVD_HD inline int rowcyclic_steps(int N) { return N >= 2 ? 2 * N - 3 : 0; }
JEVD_HD inline int rowcyclic_first(int N, int t) { return t - N + 1 > 0 ? t - N + 1 : 0; }
JEVD_HD inline int rowcyclic_step_pairs(int N, int t) { return (t + 1) / 2 - rowcyclic_first(N, t); }

}  // namespace jevd
