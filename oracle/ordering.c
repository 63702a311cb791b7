/*
 * Pivot orderings of the oracle.  TEST INFRASTRUCTURE ONLY: nothing in the
 * product path may link, load or call this file.
 *
 * An ordering is a sequence of steps; each step is a list of pivot pairs
 * (i, j), i < j, 0-based.  The pairs of one step are pairwise disjoint
 * (Sec. 2.4: pivots with disjoint index sets can be transformed
 * simultaneously), so processing them one after another gives bit-for-bit
 * the same result as processing them in parallel.
 *
 * Orderings (Sec. 2.4, Fig. 2 and Fig. 3, Alg. 3.1):
 *   ORC_ROWCYCLIC : (1,2),(1,3),...,(1,n),(2,3),...,(n-1,n), one pair a step.
 *   ORC_MODULUS   : step k (k = 1..n, 1-based indices) holds the pairs on the
 *                   k-th antidiagonal modulo n, i.e. i + j == k (mod n).
 *                   For even n, even k leaves two indices unpaired (the two
 *                   "diagonal" entries k/2 and k/2 + n/2).
 *   ORC_MODMODULUS: as ORC_MODULUS, and for even n and even k the extra pair
 *                   (k/2, k/2 + n/2) is processed as well, so every step is
 *                   full (n/2 pairs).  This is the per-step pair set that the
 *                   ring algorithm of Alg. 3.1 walks through.
 * For odd n both modulus orderings are the same: n steps of (n-1)/2 pairs,
 * each pair once a sweep (the paper only treats even n).
 */
#include <stdlib.h>

enum { ORC_ROWCYCLIC = 0, ORC_MODULUS = 1, ORC_MODMODULUS = 2 };

/* Fills step_start[0..nsteps] (offsets into the pair list) and pairs
 * (2 ints per pair).  Either array may be NULL to query the sizes only.
 * Returns the number of steps, or -1 for bad arguments. */
int orc_ordering(int n, int kind, int *step_start, int *pairs, int *npairs_out)
{
    if (n < 1 || kind < ORC_ROWCYCLIC || kind > ORC_MODMODULUS) return -1;
    int nsteps = 0, np = 0;
    if (kind == ORC_ROWCYCLIC) {
        for (int i = 1; i <= n; ++i)
            for (int j = i + 1; j <= n; ++j) {
                if (step_start) step_start[nsteps] = np;
                if (pairs) { pairs[2 * np] = i - 1; pairs[2 * np + 1] = j - 1; }
                ++np; ++nsteps;
            }
        if (step_start) step_start[nsteps] = np;
        if (npairs_out) *npairs_out = np;
        return nsteps;
    }
    /* modulus family: one antidiagonal (mod n) per step, 1-based indices */
    for (int k = 1; k <= n; ++k) {
        if (step_start) step_start[nsteps] = np;
        for (int i = 1; i <= n; ++i) {
            /* the unique j in 1..n with i + j == k (mod n) */
            int j = ((k - i - 1) % n + n) % n + 1;
            if (j > i) {
                if (pairs) { pairs[2 * np] = i - 1; pairs[2 * np + 1] = j - 1; }
                ++np;
            }
        }
        if (kind == ORC_MODMODULUS && n % 2 == 0 && k % 2 == 0) {
            int i = k / 2, j = k / 2 + n / 2;       /* the two unpaired indices */
            if (pairs) { pairs[2 * np] = i - 1; pairs[2 * np + 1] = j - 1; }
            ++np;
        }
        ++nsteps;
    }
    if (step_start) step_start[nsteps] = np;
    if (npairs_out) *npairs_out = np;
    return nsteps;
}
