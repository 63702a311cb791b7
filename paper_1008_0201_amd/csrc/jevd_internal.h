// Internal declarations shared by the host driver and the kernel files.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/jevd.h"

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
    SweepCounters *ctr;     // the sweep's counters (non-finite flag)
    bool prefetch_v;        // load the V pair with the G pair (most pairs rotate)
    unsigned *slot_rot;     // per workgroup slot: rotations in this sweep
    unsigned *slot_clamp;   // per workgroup slot: clamped hyperbolic transforms
    double2 *vlog;          // this step's rotation log (npairs entries): V is
                            // then left alone and updated by launch_apply_vlog;
                            // null: V is rotated in the step
};

// Deferred V update: the logged rotations of steps k0 .. k1 - 1 (entries of
// step k at vlog + (k - k0) * stride, pairs at pairs + step_start[k]).
struct VlogApplyArgs {
    double *V;
    int nv, n;   // rows and columns of V
    long ldv;
    const int2 *pairs;       // device, all steps of the ordering
    const int *step_start;   // device, nsteps + 1 offsets into pairs
    int k0, k1;
    const double2 *vlog;
    int stride;              // entries per logged step (>= pairs of any step)
    int max_pairs;           // pairs of the largest step (<= 4096)
};
// LDS for the rows of V held by one k_apply_vlog workgroup; the most log
// kept before V is brought up to date.
constexpr size_t kVlogLdsBytes = 128 * 1024;
constexpr size_t kVlogMaxBytes = (size_t)64 << 20;
// The most steps in one run of the log (their offsets also go to LDS).
constexpr int kVlogMaxSteps = 4096;
// Rows of V per k_apply_vlog workgroup for n columns (4 or 2; a column of
// them takes one more double in LDS, and there are 256 scratch columns), or
// 0 when even two rows do not fit (then V is rotated in the step).
int vlog_rows(int n);

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
    bool row_cyclic;     // the pairs are (p, q), p < q, in row order
};

// Optional kernel timing: a timed group of launches of one kernel class
// (one launch, or all launches of a sweep) is bracketed by a pair of HIP
// events on the stream; collect() (after a stream synchronisation) sums the
// durations and launch counts per class and recycles the events.
struct KernelTimer {
    bool on = false;
    hipEvent_t *ev = nullptr;  // 2 per timed launch
    int *cls = nullptr;
    int *cnt = nullptr;  // launches in each timed group
    int cap = 0, used = 0;
    double ms[4] = {0, 0, 0, 0};
    long long launches[4] = {0, 0, 0, 0};

    hipError_t begin(hipStream_t st, int c)
    {
        if (!on) return hipSuccess;
        if (used == cap) {
            const int ncap = cap ? 2 * cap : 256;
            hipEvent_t *nev = new hipEvent_t[2 * ncap];
            int *ncls = new int[ncap];
            int *ncnt = new int[ncap];
            for (int i = 0; i < 2 * cap; ++i) nev[i] = ev[i];
            for (int i = 0; i < cap; ++i) {
                ncls[i] = cls[i];
                ncnt[i] = cnt[i];
            }
            for (int i = 2 * cap; i < 2 * ncap; ++i) {
                hipError_t e = hipEventCreate(&nev[i]);
                if (e != hipSuccess) {
                    for (int j = 2 * cap; j < i; ++j) (void)hipEventDestroy(nev[j]);
                    delete[] nev;
                    delete[] ncls;
                    delete[] ncnt;
                    return e;
                }
            }
            delete[] ev;
            delete[] cls;
            delete[] cnt;
            ev = nev;
            cls = ncls;
            cnt = ncnt;
            cap = ncap;
        }
        cls[used] = c;
        return hipEventRecord(ev[2 * used], st);
    }
    hipError_t end(hipStream_t st, int nlaunch = 1)
    {
        if (!on) return hipSuccess;
        hipError_t e = hipEventRecord(ev[2 * used + 1], st);
        cnt[used] = nlaunch;
        ++used;
        return e;
    }
    hipError_t collect()
    {
        for (int i = 0; i < used; ++i) {
            float t = 0.f;
            hipError_t e = hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
            if (e != hipSuccess) return e;
            ms[cls[i]] += t;
            launches[cls[i]] += cnt[i];
        }
        used = 0;
        return hipSuccess;
    }
    void reset()
    {
        used = 0;
        for (int i = 0; i < 4; ++i) {
            ms[i] = 0;
            launches[i] = 0;
        }
    }
    void release()
    {
        for (int i = 0; i < 2 * cap; ++i) (void)hipEventDestroy(ev[i]);
        delete[] ev;
        delete[] cls;
        delete[] cnt;
        ev = nullptr;
        cls = nullptr;
        cnt = nullptr;
        cap = used = 0;
    }
};

hipError_t launch_pair_step(const PairStepArgs &a, hipStream_t st);

// `steps` (2) consecutive steps of the ring (modified modulus, even n,
// m <= 1024) in one launch of p workgroups, bit for bit the steps of
// launch_pair_step; G read from Gin, written to Gout.
struct RingStepsArgs {
    const double *Gin;
    double *Gout;
    int m;
    long ldg;
    const int2 *pairs;  // the table from the launch's first step on (p pairs per step)
    int p;              // pairs per step (n / 2)
    int steps;
    const signed char *J;
    double tol;
    SweepCounters *ctr;
    unsigned *slot_rot, *slot_clamp;
    double2 *vlog;      // null, or the log row of the first step
    int vlog_stride;    // entries between the log rows of consecutive steps
};
constexpr int kRingStepsMaxRows = 1024;
hipError_t launch_pair_steps_ring(const RingStepsArgs &a, hipStream_t st);
hipError_t launch_apply_vlog(const VlogApplyArgs &a, hipStream_t st);

struct BatchInst;
hipError_t launch_canonical(int batch, int m, int n, const double *lam, long long slam,
                            const double *U, int ldu, long long su, const double *V, int ldv,
                            long long sv, double *lam_o, double *U_o, double *V_o, hipStream_t st);
hipError_t launch_adjoint(int batch, int m, int n, const double *G, int ldg, long long sg,
                          const signed char *J, long long sj, const double *lam, long long slam,
                          const double *U, int ldu, long long su, const double *w, long long sw,
                          const double *C, int ldc, long long sc, double *dG, int ldd,
                          long long sd, double *wsK, double *wsW, double *wsM, double *wsT,
                          hipStream_t st);
constexpr int kBatchMaxN = 4096;   // largest n_i of a batched solve
hipError_t prepare_batch_kernel();
// hipFuncSetAttribute(func, MaxDynamicSharedMemorySize, bytes) on the current
// device unless a limit of at least bytes was set there already (the call
// costs about a millisecond; launches that need more than 64 KiB of dynamic
// LDS call this before every launch).
hipError_t set_lds_limit(const void *func, int bytes);  // once before the first launch (sets the LDS limit)
hipError_t launch_batch(const BatchInst *inst, const int *order, int batch, int *queue,
                        int ordering, int max_sweeps, int accumulate_v, int *sweeps, int *status,
                        int grid, int waves, hipStream_t st);
bool batch_waves_supported(int waves);
// Size classes of a batched solve: instances with kBatchClassMax[c - 1] < n
// <= kBatchClassMax[c] form class c, each launched with its own workgroup
// size (wavefronts: 4, 8 or 16, the tuned or the default one).
constexpr int kBatchClasses = JEVD_BATCH_CLASSES;
constexpr int kBatchClassMax[kBatchClasses] = {48, 96, 141, kBatchMaxN};
int batch_class_of(int n);
int default_batch_waves(int cls);
int tuned_batch_waves(int cls);           // -1: not measured
bool batch_waves_fit(int waves, int nmax);  // the step arrays of n <= nmax fit the LDS share
hipError_t launch_fill_batch(double *G, int m, int n, long count, unsigned long long seed,
                             hipStream_t st);
hipError_t launch_small_solve(const SmallSolveArgs &a, hipStream_t st);
hipError_t launch_sum_slots(unsigned *slot_rot, unsigned *slot_clamp, int nslots,
                            SweepCounters *ctr, hipStream_t st);
size_t small_solve_lds_bytes(int m, int n, bool want_v, int *lds_g, int *lds_v);
hipError_t launch_identity(double *V, int n, long ldv, hipStream_t st);
hipError_t launch_finalize(const double *G, int m, int n, long ldg, const signed char *J,
                           double *lambda, double *U, long ldu, hipStream_t st);

}  // namespace jevd
