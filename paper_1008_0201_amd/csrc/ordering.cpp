// Pivot orderings run by the solver (host side; Sec. 2.4, Fig. 2-3, Alg. 3.1).
//
// Modulus family over N columns (or block columns), 1-based: step k = 1..N
// processes the pairs (i, j), i < j, with i + j == k (mod N), i.e. the pairs on
// the two antidiagonals i + j = k and i + j = k + N:
//   i + j = k     : i = 1 .. floor((k-1)/2),        j = k - i
//   i + j = k + N : i = k .. ceil((k+N)/2) - 1,      j = k + N - i
// For even N and even k two indices stay idle (k/2 and k/2 + N/2); the
// modified modulus ordering pairs them too, so that every step is full.
// The resulting per-step pair sets are those the ring of Alg. 3.1 visits;
// for the modified modulus on even N the pairs of each step are listed in
// the order of the ring's processes (see ring_schedule), permuted to
// workgroup slots (see slot_process).
// Row-cyclic: the pairs (1,2),(1,3),...,(1,N),(2,3),...,(N-1,N), run as the
// 2N - 3 steps of equal i + j (rowcyclic_steps in ordering.h), which give the
// same result as one pair at a time.
#include <vector>

#include "ordering.h"

namespace jevd {

// The ring of Alg. 3.1 over N = 2p columns: p processes, each holding one
// pair, as in the process map described after Alg. 3.1.  A process starts on
// the antidiagonal at (r+1, N-r) (1-based).  From one step to the next it
// keeps one of its two columns:
//   - while its auxiliary position (a, c) lies below the main antidiagonal
//     (a + c > N) it moves down: a grows by one and the new first column
//     is a; if that lands on the diagonal (a == c) it instead takes the row
//     index no other process holds, a - p, as its first column and from then
//     on walks that row (both auxiliary indices become a - p);
//   - otherwise it walks right: c grows by one and the new second column is c.
// The pair sets of the N steps are the modified modulus steps (the host test
// checks this); after N steps the processes are back on the antidiagonal in
// reverse order.  Fills pairs[step][r] for one sweep, process order.
static void ring_schedule(int N, std::vector<int> &pairs)
{
    const int p = N / 2;
    std::vector<int> a(p), c(p), pi(p), pj(p);
    for (int r = 0; r < p; ++r) {
        a[r] = r + 1;
        c[r] = N - r;
        pi[r] = a[r];
        pj[r] = c[r];
    }
    pairs.assign((size_t)2 * N * p, 0);
    for (int k = 0; k < N; ++k) {
        for (int r = 0; r < p; ++r) {
            pairs[(size_t)2 * (k * p + r)] = pi[r] - 1;
            pairs[(size_t)2 * (k * p + r) + 1] = pj[r] - 1;
        }
        for (int r = 0; r < p; ++r) {
            if (a[r] + c[r] > N) {
                a[r] += 1;
                if (a[r] == c[r]) {
                    a[r] -= p;
                    c[r] = a[r];
                }
                pi[r] = a[r];
            } else {
                c[r] += 1;
                pj[r] = c[r];
            }
        }
    }
}

// Workgroup slot -> ring process.  Consecutive workgroups of a launch are
// dealt round-robin to the 8 XCDs of the MI355X; slot b runs process
// (b % 8) * (p / 8) + b / 8, so each XCD holds a contiguous run of p / 8
// neighbouring processes and a column handed to the next process usually
// stays in the same XCD's L2.  Identity when p is not a multiple of 8.
static int slot_process(int b, int p)
{
    if (p % 8) return b;
    return (b % 8) * (p / 8) + b / 8;
}

int build_ordering(int n, int ordering, std::vector<int> &step_start, std::vector<int> &pairs)
{
    step_start.clear();
    pairs.clear();
    if (n < 1) return -1;
    if (ordering == kOrdRowCyclic) {
        for (int t = 1; t <= rowcyclic_steps(n); ++t) {
            step_start.push_back((int)pairs.size() / 2);
            const int i0 = rowcyclic_first(n, t);
            for (int r = 0; r < rowcyclic_step_pairs(n, t); ++r) {
                pairs.push_back(i0 + r);
                pairs.push_back(t - i0 - r);
            }
        }
        step_start.push_back((int)pairs.size() / 2);
        return (int)step_start.size() - 1;
    }
    if (ordering != kOrdModulus && ordering != kOrdModModulus) return -1;
    const int N = n;
    if (ordering == kOrdModModulus && N % 2 == 0 && N >= 4) {
        // modified modulus on even N: the ring schedule, pairs listed by slot
        const int p = N / 2;
        std::vector<int> ring;
        ring_schedule(N, ring);
        pairs.assign((size_t)2 * N * p, 0);
        for (int k = 0; k < N; ++k) {
            step_start.push_back(k * p);
            for (int b = 0; b < p; ++b) {
                const int r = slot_process(b, p);
                pairs[(size_t)2 * (k * p + b)] = ring[(size_t)2 * (k * p + r)];
                pairs[(size_t)2 * (k * p + b) + 1] = ring[(size_t)2 * (k * p + r) + 1];
            }
        }
        step_start.push_back(N * p);
        return N;
    }
    for (int k = 1; k <= N; ++k) {
        step_start.push_back((int)pairs.size() / 2);
        const int np = modulus_step_pairs(N, k, ordering == kOrdModModulus);
        for (int r = 0; r < np; ++r) {
            int i, j;
            modulus_pair(N, k, r, &i, &j);
            pairs.push_back(i);
            pairs.push_back(j);
        }
    }
    step_start.push_back((int)pairs.size() / 2);
    return N;
}

}  // namespace jevd
