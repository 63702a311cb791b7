// Internal declarations shared by the host driver and the kernel files.
#pragma once
#include <hip/hip_runtime.h>

#include "device_math.h"

namespace jevd {

// LDS of one gfx950 workgroup is 160 KiB; keep 1 KiB for static arrays.
constexpr size_t kSmallSolveLdsBytes = 160 * 1024 - 1024;

struct PairStepArgs {
    double *G;
    int m;
    long ldg;
    double *V;  // may be null
    int nv;
    long ldv;
    const int2 *pairs;  // the step's pairs (i < j), npairs of them
    int npairs;
    const signed char *J;  // device, may be null (J = I)
    double tol;
    SweepCounters *ctr;
};

struct SmallSolveArgs {
    double *G;
    int m, n;
    long ldg;
    double *V;
    long ldv;
    const signed char *J;
    double tol;
    const int2 *pairs;
    const int *step_start;
    int nsteps;
    int max_pairs_per_step;
    int max_sweeps;
    SweepCounters *ctr;  // max_sweeps slots
    int *sweeps_out;     // device
};

hipError_t launch_pair_step(const PairStepArgs &a, hipStream_t st);
hipError_t launch_small_solve(const SmallSolveArgs &a, hipStream_t st);
size_t small_solve_lds_bytes(int m, int n, bool want_v, int *lds_g, int *lds_v);
hipError_t launch_identity(double *V, int n, long ldv, hipStream_t st);
hipError_t launch_finalize(const double *G, int m, int n, long ldg, const signed char *J,
                           double *lambda, double *U, long ldu, hipStream_t st);

}  // namespace jevd
