// Pivot orderings run by the solver (host side; Sec. 2.4, Fig. 2-3, Alg. 3.1).
//
// Modulus family over N columns (or block columns), 1-based: step k = 1..N
// processes the pairs (i, j), i < j, with i + j == k (mod N), i.e. the pairs on
// the two antidiagonals i + j = k and i + j = k + N:
//   i + j = k     : i = 1 .. floor((k-1)/2),        j = k - i
//   i + j = k + N : i = k .. ceil((k+N)/2) - 1,      j = k + N - i
// For even N and even k two indices stay idle (k/2 and k/2 + N/2); the
// modified modulus ordering pairs them too, so that every step is full.
// The resulting per-step pair sets are those the ring of Alg. 3.1 visits.
// Row-cyclic: one pair per step, (1,2),(1,3),...,(1,N),(2,3),...,(N-1,N).
#include <vector>

#include "ordering.h"

namespace jevd {

int build_ordering(int n, int ordering, std::vector<int> &step_start, std::vector<int> &pairs)
{
    step_start.clear();
    pairs.clear();
    if (n < 1) return -1;
    if (ordering == kOrdRowCyclic) {
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                step_start.push_back((int)pairs.size() / 2);
                pairs.push_back(i);
                pairs.push_back(j);
            }
        step_start.push_back((int)pairs.size() / 2);
        return (int)step_start.size() - 1;
    }
    if (ordering != kOrdModulus && ordering != kOrdModModulus) return -1;
    const int N = n;
    for (int k = 1; k <= N; ++k) {
        step_start.push_back((int)pairs.size() / 2);
        for (int i = 1; i <= (k - 1) / 2; ++i) {          // antidiagonal i + j = k
            pairs.push_back(i - 1);
            pairs.push_back(k - i - 1);
        }
        const int hi = (k + N + 1) / 2 - 1;               // ceil((k+N)/2) - 1
        for (int i = k; i <= hi; ++i) {                    // antidiagonal i + j = k + N
            pairs.push_back(i - 1);
            pairs.push_back(k + N - i - 1);
        }
        if (ordering == kOrdModModulus && N % 2 == 0 && k % 2 == 0) {
            pairs.push_back(k / 2 - 1);
            pairs.push_back(k / 2 + N / 2 - 1);
        }
    }
    step_start.push_back((int)pairs.size() / 2);
    return N;
}

}  // namespace jevd
