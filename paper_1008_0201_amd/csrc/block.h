// Block one-sided Jacobi (Sec. 2.2-2.3, Alg. 3.4 with unpivoted Cholesky):
// host-side driver interface.
#pragma once
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "jevd_internal.h"

namespace jevd {

struct BlockWorkspace {
    double *partial = nullptr;  // split-K partial Grams, per pivot nsplit x (W x W)
    double *vp = nullptr;       // per pivot W x W accumulated transform, row-major
    int *flags = nullptr;       // per pivot: 1 if its transform must be applied
    double2 *vlog = nullptr;    // W = 128: per pivot the log of its inner transforms
    double *ap = nullptr;       // per pivot the W x W Gram, added up over the splits
    size_t capPartial = 0, capVp = 0, capFlags = 0, capVlog = 0, capAp = 0;
    void *tables = nullptr;     // block and inner orderings (device copies)
    // V's half of the update runs on a second stream, one step behind (two
    // parities of vp and flags); evReady: the solve's stream has reached
    // the point where the next V update may start; evVdone[p]: the V update
    // that read parity p is done; evJoin: stream hand-over
    hipStream_t vstream = nullptr;
    hipEvent_t evReady = nullptr, evVdone[2] = {nullptr, nullptr}, evJoin = nullptr;
    // mixed precision: FP32 iterate and transform, FP64 work arrays
    float *g32 = nullptr, *v32 = nullptr;
    double *t64 = nullptr, *w64 = nullptr;
    size_t capG32 = 0, capV32 = 0, capT64 = 0, capW64 = 0;
};

struct BlockRunArgs {
    int m, n;
    double *G;
    int ldg;
    signed char *dJ;         // device, may be null; rewritten by sign pivoting
    const signed char *hJ;   // host, may be null
    double tol;
    bool full_block;
    int b;
    int max_sweeps, max_inner;
    double *V;
    int ldv;
    bool sign_pivot;         // Alg. 3.3 in the pivot solve (HBSC / HFSC)
    hipStream_t stream;
    SweepCounters *dctr;  // max_sweeps slots, zeroed by run_block
    SweepCounters *hctr;  // pinned mirror
    KernelTimer *timer;
};

bool block_width_supported(int b);
bool block_shape_supported(int m, int n, int b);
bool block_partition_even(int n, int b);
bool block_options_supported(int m, int n, int b, bool sign_pivot);
// Autotuner table (tune.cpp): the block width and the variant measured
// fastest for the shape, or -1 when the shape has not been measured.
int tuned_block_width(int m, int n);
int tuned_variant(int m, int n);
int choose_block_width(int m, int n);
int auto_variant(int m, int n);
int run_block(BlockWorkspace *ws, const BlockRunArgs &a, int *sweeps_done);
// FP32-MFMA block sweeps, V0 made orthogonal in FP64, G <- G V0, then FP64
// block sweeps (a.V required; J = I).
int run_block_mixed(BlockWorkspace *ws, const BlockRunArgs &a, int max_sweeps_low, int *sweeps_low,
                    int *sweeps_done);
void block_workspace_free(BlockWorkspace *ws);

}  // namespace jevd
