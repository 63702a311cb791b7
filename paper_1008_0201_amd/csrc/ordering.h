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

}  // namespace jevd
