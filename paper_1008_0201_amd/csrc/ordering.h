// Host-side pivot orderings of the solver.
#pragma once
#include <vector>

namespace jevd {

enum { kOrdRowCyclic = 0, kOrdModulus = 1, kOrdModModulus = 2 };

// Fills step_start (nsteps + 1 offsets) and pairs (2 ints per pair, 0-based,
// i < j).  Returns the number of steps, or -1 for bad arguments.
int build_ordering(int n, int ordering, std::vector<int> &step_start, std::vector<int> &pairs);

}  // namespace jevd
