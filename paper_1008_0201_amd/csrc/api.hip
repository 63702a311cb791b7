// C ABI of the one-sided Jacobi solver (include/jevd.h): argument checks,
// workspace, the sweep loop and the dispatch to the pointwise and block
// kernels.
#include <algorithm>
#include <cfloat>
#include <chrono>
#include <mutex>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/jevd.h"
#include "block.h"
#include "jevd_internal.h"
#include "ordering.h"

using namespace jevd;

namespace jevd {
struct BatchInst {  // mirrors the device-side descriptor in batched.hip
    double *G;
    double *V;
    double *lambda;
    double *U;
    const signed char *J;
    double tol;
    int m, n, ldg, ldv, ldu;
};
}  // namespace jevd

struct jevd_batch_s {
    jevd_handle_t h = nullptr;
    int batch = 0;
    int ordering = 0, max_sweeps = 50, accumulate_v = 0;
    // size classes (largest first in d_order): offset, count, workgroup size
    // in wavefronts and grid of each class's launch
    int cls_off[kBatchClasses] = {}, cls_cnt[kBatchClasses] = {};
    int cls_waves[kBatchClasses] = {};
    // launches: consecutive classes of one workgroup size share a launch and
    // its queue (so longest-first holds across them); the first launch runs
    // on the caller's stream, the others at the same time on a second
    // stream, so that their workgroups take the CUs the first launch frees
    // in its tail
    int ngrp = 0;
    int grp_off[kBatchClasses] = {}, grp_cnt[kBatchClasses] = {};
    int grp_waves[kBatchClasses] = {}, grp_grid[kBatchClasses] = {};
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    BatchInst *d_inst = nullptr;
    int *d_order = nullptr;
    int *d_queue = nullptr;    // one counter per launch
    int *d_sweeps = nullptr;   // per instance
    int *d_status = nullptr;   // per instance
    signed char *d_J = nullptr;
    void *arena = nullptr;   // one device allocation holding the arrays above
    size_t arena_bytes = 0;
    hipStream_t last = nullptr;
    bool ran = false;
};

// Work memory of jevd_adjoint_noalloc: a fixed array in the library's code
// object, one copy per GPU, held until the process ends.  Host code never
// uses the name itself (a host-side stand-in, not a device address): the
// device address is looked up once per device (scratch_address) and passed
// to the kernels like any workspace.
constexpr size_t kScratchDoubles = (size_t)4 << 20;   // 32 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[64] = {};   // per device ordinal

// The device address of `scratch` on the current device (dev), looked up
// with that device current on first use; nullptr if the lookup fails.
double *scratch_address(int dev)
{
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = (double *)ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

struct jevd_handle_s {
    int device = 0;
    hipStream_t stream = nullptr;
    double *scratch = nullptr;   // this device's `scratch` (jevd_adjoint_noalloc)

    signed char *dJ = nullptr;
    size_t capJ = 0;
    SweepCounters *dctr = nullptr;  // one slot per sweep
    SweepCounters *hctr = nullptr;  // pinned mirror
    int capCtr = 0;
    int *dsweeps = nullptr;
    int *hsweeps = nullptr;  // pinned
    unsigned *dslots = nullptr;  // per-slot rotation / clamp counts of a sweep
    size_t capSlots = 0;
    double2 *dvlog = nullptr;    // pointwise rotation log (deferred V update), two buffers
    size_t capVlog = 0;
    double *dgalt = nullptr;     // second copy of G for the multi-step ring launches
    size_t capGalt = 0;
    // device arena of the last destroyed batch plan, reused by the next one
    // (a fresh hipMalloc can take tens of milliseconds)
    void *batch_pool = nullptr;
    size_t batch_pool_bytes = 0;
    void *batch_stage = nullptr;   // pinned host image of a plan's arena (one copy)
    size_t batch_stage_bytes = 0;
    hipStream_t vstream = nullptr;   // second stream of the deferred V update
    hipEvent_t evLogged[2] = {nullptr, nullptr};    // a log buffer is complete
    hipEvent_t evApplied[2] = {nullptr, nullptr};   // V is updated from a log buffer

    // cached ordering table
    int tabN = -1, tabOrd = -1;
    std::vector<int> hstep;
    int maxPairsPerStep = 0;
    int2 *dpairs = nullptr;
    size_t capPairs = 0;
    int *dstep = nullptr;
    size_t capStep = 0;

    BlockWorkspace blk;
    KernelTimer timer;
    jevd_info info;

    double *vtmp = nullptr;  // V work array of the mixed path when V is not wanted
    size_t capVtmp = 0;
    double *tuneG = nullptr, *tuneV = nullptr;  // jevd_autotune's working copies
    size_t capTuneG = 0, capTuneV = 0;
    // adjoint work arrays: K, W, M' (n x n) and T (m x n) per instance
    double *adjK = nullptr, *adjW = nullptr, *adjM = nullptr, *adjT = nullptr;
    size_t capAdjK = 0, capAdjW = 0, capAdjM = 0, capAdjT = 0;
};

namespace {

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) {                         \
            (void)hipGetLastError();                    \
            return (_e == hipErrorOutOfMemory) ? JEVD_ENOMEM : JEVD_EHIP; \
        }                                               \
    } while (0)

template <class T>
int grow_device(T **p, size_t *cap, size_t need)
{
    if (*cap >= need && *p) return JEVD_OK;
    if (*p) HIP_TRY(hipFree(*p));
    *p = nullptr;
    *cap = 0;
    HIP_TRY(hipMalloc((void **)p, need * sizeof(T)));
    *cap = need;
    return JEVD_OK;
}

int ensure_counters(jevd_handle_t h, int nslots)
{
    if (h->capCtr >= nslots && h->dctr) return JEVD_OK;
    if (h->dctr) HIP_TRY(hipFree(h->dctr));
    if (h->hctr) HIP_TRY(hipHostFree(h->hctr));
    h->dctr = nullptr;
    h->hctr = nullptr;
    h->capCtr = 0;
    HIP_TRY(hipMalloc((void **)&h->dctr, sizeof(SweepCounters) * nslots));
    HIP_TRY(hipHostMalloc((void **)&h->hctr, sizeof(SweepCounters) * nslots, hipHostMallocDefault));
    h->capCtr = nslots;
    return JEVD_OK;
}

int ensure_ordering(jevd_handle_t h, int n, int ord)
{
    if (h->tabN == n && h->tabOrd == ord) return JEVD_OK;
    std::vector<int> st, pr;
    if (build_ordering(n, ord, st, pr) < 0) return JEVD_EINVAL;
    int st_ok = grow_device(&h->dpairs, &h->capPairs, pr.size() / 2 + 1);
    if (st_ok) return st_ok;
    st_ok = grow_device(&h->dstep, &h->capStep, st.size());
    if (st_ok) return st_ok;
    if (!pr.empty())
        HIP_TRY(hipMemcpyAsync(h->dpairs, pr.data(), pr.size() * sizeof(int), hipMemcpyHostToDevice,
                               h->stream));
    HIP_TRY(hipMemcpyAsync(h->dstep, st.data(), st.size() * sizeof(int), hipMemcpyHostToDevice,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));  // host vectors go out of scope
    h->hstep = st;
    h->maxPairsPerStep = 0;
    for (size_t k = 0; k + 1 < st.size(); ++k)
        if (st[k + 1] - st[k] > h->maxPairsPerStep) h->maxPairsPerStep = st[k + 1] - st[k];
    h->tabN = n;
    h->tabOrd = ord;
    return JEVD_OK;
}

void fill_defaults(jevd_opts *o)
{
    o->ordering = JEVD_ORD_MODMODULUS;
    o->variant = JEVD_VAR_AUTO;
    o->block = 0;
    o->max_sweeps = 50;
    o->max_inner = 30;
    o->accumulate_v = 0;
    o->pivot = JEVD_PIVOT_NONE;
    o->precision = JEVD_PREC_FP64;
}

}  // namespace

extern "C" {

int jevd_default_opts(jevd_opts *o)
{
    if (!o) return JEVD_EINVAL;
    fill_defaults(o);
    return JEVD_OK;
}

const char *jevd_strerror(int status)
{
    switch (status) {
    case JEVD_OK: return "success";
    case JEVD_EINVAL: return "invalid argument";
    case JEVD_ENONFINITE: return "non-finite value (NaN or Inf) in a Gram entry";
    case JEVD_ENOCONV: return "no convergence within max_sweeps sweeps";
    case JEVD_EHIP: return "HIP runtime error";
    case JEVD_ENOMEM: return "out of memory";
    default: return "unknown status";
    }
}

int jevd_ordering(int n, int ordering, int *step_start, int *pairs, int *nsteps, int *npairs)
{
    std::vector<int> st, pr;
    const int ns = build_ordering(n, ordering, st, pr);
    if (ns < 0) return JEVD_EINVAL;
    if (nsteps) *nsteps = ns;
    if (npairs) *npairs = (int)(pr.size() / 2);
    if (step_start) std::memcpy(step_start, st.data(), st.size() * sizeof(int));
    if (pairs && !pr.empty()) std::memcpy(pairs, pr.data(), pr.size() * sizeof(int));
    return JEVD_OK;
}

// Host-only argument check used by jacobi_evd before any device work.
int jevd_validate(int m, int n, int ldg, const signed char *J, double tol, const jevd_opts *opts,
                  const double *U, int ldu, const double *V, int ldv)
{
    if (n < 1 || m < n || ldg < m) return JEVD_EINVAL;
    if (U && ldu < m) return JEVD_EINVAL;
    if (V && ldv < n) return JEVD_EINVAL;
    if (std::isnan(tol) || std::isinf(tol)) return JEVD_EINVAL;
    if (J)
        for (int i = 0; i < n; ++i)
            if (J[i] != 1 && J[i] != -1) return JEVD_EINVAL;
    if (opts) {
        if (opts->ordering < JEVD_ORD_ROWCYCLIC || opts->ordering > JEVD_ORD_MODMODULUS) return JEVD_EINVAL;
        if (opts->variant < JEVD_VAR_POINTWISE || opts->variant > JEVD_VAR_AUTO) return JEVD_EINVAL;
        if (opts->max_sweeps < 1 || opts->max_sweeps > 100000) return JEVD_EINVAL;
        if (opts->max_inner < 1) return JEVD_EINVAL;
        if (opts->accumulate_v != 0 && opts->accumulate_v != 1) return JEVD_EINVAL;
        if (opts->accumulate_v && !V) return JEVD_EINVAL;
        if (opts->block != 0 && !block_width_supported(opts->block)) return JEVD_EINVAL;
        if (opts->pivot != JEVD_PIVOT_NONE && opts->pivot != JEVD_PIVOT_SIGN) return JEVD_EINVAL;
        if (opts->pivot == JEVD_PIVOT_SIGN && opts->variant != JEVD_VAR_BLOCK_ORIENTED &&
            opts->variant != JEVD_VAR_FULL_BLOCK)
            return JEVD_EINVAL;
        if (opts->precision != JEVD_PREC_FP64 && opts->precision != JEVD_PREC_MIXED) return JEVD_EINVAL;
        if (opts->precision == JEVD_PREC_MIXED) {
            if (opts->variant != JEVD_VAR_BLOCK_ORIENTED && opts->variant != JEVD_VAR_FULL_BLOCK)
                return JEVD_EINVAL;
            if (opts->accumulate_v) return JEVD_EINVAL;
            if (J)
                for (int i = 0; i < n; ++i)
                    if (J[i] != 1) return JEVD_EINVAL;
        }
        const int variant = (opts->variant == JEVD_VAR_AUTO) ? auto_variant(m, n) : opts->variant;
        if (variant == JEVD_VAR_BLOCK_ORIENTED || variant == JEVD_VAR_FULL_BLOCK) {
            const int b = opts->block ? opts->block : choose_block_width(m, n);
            if (!block_options_supported(m, n, b, opts->pivot == JEVD_PIVOT_SIGN)) return JEVD_EINVAL;
        }
    } else if (auto_variant(m, n) != JEVD_VAR_POINTWISE &&
               !block_shape_supported(m, n, choose_block_width(m, n))) {
        return JEVD_EINVAL;
    }
    return JEVD_OK;
}

int jevd_create(jevd_handle_t *h, void *stream)
{
    if (!h) return JEVD_EINVAL;
    *h = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return JEVD_EHIP;
    }
    jevd_handle_s *p = new (std::nothrow) jevd_handle_s();
    if (!p) return JEVD_ENOMEM;
    p->device = dev;
    p->stream = (hipStream_t)stream;
    p->scratch = scratch_address(dev);
    if (!p->scratch) {
        jevd_destroy(p);
        return JEVD_EHIP;
    }
    std::memset(&p->info, 0, sizeof(p->info));
    if (hipHostMalloc((void **)&p->hsweeps, sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&p->dsweeps, sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        jevd_destroy(p);
        return JEVD_ENOMEM;
    }
    *h = p;
    return JEVD_OK;
}

int jevd_destroy(jevd_handle_t h)
{
    if (!h) return JEVD_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    if (h->dJ) (void)hipFree(h->dJ);
    if (h->dctr) (void)hipFree(h->dctr);
    if (h->hctr) (void)hipHostFree(h->hctr);
    if (h->dsweeps) (void)hipFree(h->dsweeps);
    if (h->hsweeps) (void)hipHostFree(h->hsweeps);
    if (h->dpairs) (void)hipFree(h->dpairs);
    if (h->dstep) (void)hipFree(h->dstep);
    if (h->dslots) (void)hipFree(h->dslots);
    if (h->dvlog) (void)hipFree(h->dvlog);
    if (h->dgalt) (void)hipFree(h->dgalt);
    if (h->batch_pool) (void)hipFree(h->batch_pool);
    if (h->batch_stage) (void)hipHostFree(h->batch_stage);
    if (h->vstream) {
        (void)hipStreamSynchronize(h->vstream);
        (void)hipStreamDestroy(h->vstream);
    }
    for (int i = 0; i < 2; ++i) {
        if (h->evLogged[i]) (void)hipEventDestroy(h->evLogged[i]);
        if (h->evApplied[i]) (void)hipEventDestroy(h->evApplied[i]);
    }
    if (h->vtmp) (void)hipFree(h->vtmp);
    if (h->tuneG) (void)hipFree(h->tuneG);
    if (h->tuneV) (void)hipFree(h->tuneV);
    if (h->adjK) (void)hipFree(h->adjK);
    if (h->adjW) (void)hipFree(h->adjW);
    if (h->adjM) (void)hipFree(h->adjM);
    if (h->adjT) (void)hipFree(h->adjT);
    block_workspace_free(&h->blk);
    h->timer.release();
    delete h;
    return JEVD_OK;
}

int jevd_set_timing(jevd_handle_t h, int on)
{
    if (!h || (on != 0 && on != 1)) return JEVD_EINVAL;
    h->timer.on = on != 0;
    return JEVD_OK;
}

int jevd_get_info(jevd_handle_t h, jevd_info *info)
{
    if (!h || !info) return JEVD_EINVAL;
    *info = h->info;
    return JEVD_OK;
}

namespace jevd {
// Eight independent accumulators per wavefront, operands in registers; one
// value per thread is written so that the MFMAs are not removed.
__global__ __launch_bounds__(256) void k_mfma_rate(double *out, int iters, double a0)
{
    typedef double d4v __attribute__((ext_vector_type(4)));
    d4v acc[8];
    for (int q = 0; q < 8; ++q) acc[q] = d4v{0, 0, 0, 0};
    const double a = a0 + threadIdx.x * 1e-9, b = 0.5 * a0;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
    }
    double s = 0.0;
    for (int q = 0; q < 8; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}
}  // namespace jevd

int jevd_mfma_f64_rate(jevd_handle_t h, int waves_per_simd, int iters, double *tflops)
{
    if (!h || !tflops || iters < 1 ||
        (waves_per_simd != 1 && waves_per_simd != 2 && waves_per_simd != 4))
        return JEVD_EINVAL;
    int cus = 0;
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
    const int grid = cus * waves_per_simd;   // four wavefronts (one per SIMD) per workgroup
    double *buf = nullptr;
    HIP_TRY(hipMalloc(&buf, sizeof(double) * (size_t)grid * 256));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = JEVD_OK;
    float ms = 0.f;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = JEVD_EHIP;
    for (int rep = 0; rep < 2 && rc == JEVD_OK; ++rep) {   // the first run warms up
        if (hipEventRecord(e0, h->stream) != hipSuccess) rc = JEVD_EHIP;
        jevd::k_mfma_rate<<<grid, 256, 0, h->stream>>>(buf, iters, 1.0);
        if (rc == JEVD_OK && hipGetLastError() != hipSuccess) rc = JEVD_EHIP;
        if (rc == JEVD_OK && hipEventRecord(e1, h->stream) != hipSuccess) rc = JEVD_EHIP;
        if (rc == JEVD_OK && hipEventSynchronize(e1) != hipSuccess) rc = JEVD_EHIP;
        if (rc == JEVD_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = JEVD_EHIP;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (rc != JEVD_OK) return rc;
    const double mfmas = (double)grid * 4 * iters * 8;
    *tflops = ms > 0.f ? 2048.0 * mfmas / (ms * 1e-3) / 1e12 : 0.0;
    return JEVD_OK;
}

static int run_pointwise(jevd_handle_t h, int m, int n, double *G, int ldg, const signed char *dJ,
                         double tol, const jevd_opts &o, double *V, int ldv, int *sweeps_done)
{
    int st = ensure_ordering(h, n, o.ordering);
    if (st) return st;
    const int nsteps = (int)h->hstep.size() - 1;
    int lg = 0, lv = 0;
    const bool small = small_solve_lds_bytes(m, n, V != nullptr, &lg, &lv) > 0 && lg &&
                       (V == nullptr || lv) && (o.ordering == JEVD_ORD_ROWCYCLIC || n <= 128);
    if (small) {
        // whole solve in one workgroup (all sweeps inside the kernel)
        HIP_TRY(hipMemsetAsync(h->dctr, 0, sizeof(SweepCounters) * o.max_sweeps, h->stream));
        SmallSolveArgs a{G, m, n, (long)ldg, V, (long)ldv, dJ, tol, h->dpairs, h->dstep, nsteps,
                         h->maxPairsPerStep, o.max_sweeps, h->dctr, h->dsweeps,
                         o.ordering == JEVD_ORD_ROWCYCLIC};
        HIP_TRY(h->timer.begin(h->stream, JEVD_K_PAIR_STEP));
        HIP_TRY(launch_small_solve(a, h->stream));
        HIP_TRY(h->timer.end(h->stream));
        HIP_TRY(hipMemcpyAsync(h->hsweeps, h->dsweeps, sizeof(int), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(h->hctr, h->dctr, sizeof(SweepCounters) * o.max_sweeps,
                               hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        HIP_TRY(h->timer.collect());
        const int sw = *h->hsweeps;
        *sweeps_done = sw;
        for (int s = 0; s < sw; ++s) {
            if (h->hctr[s].nonfinite) return JEVD_ENONFINITE;
            if (h->hctr[s].rotations == 0) return JEVD_OK;
        }
        return JEVD_ENOCONV;
    }
    // one kernel launch per parallel step, one counter read-back per sweep
    HIP_TRY(hipMemsetAsync(h->dctr, 0, sizeof(SweepCounters) * o.max_sweeps, h->stream));
    const int nslots = h->maxPairsPerStep;
    st = grow_device(&h->dslots, &h->capSlots, (size_t)2 * nslots);
    if (st) return st;
    HIP_TRY(hipMemsetAsync(h->dslots, 0, sizeof(unsigned) * 2 * nslots, h->stream));
    const long long pairs_per_sweep = h->hstep[nsteps];
    // Deferred V: the steps log their rotations and V is updated once per
    // run of logged steps (a whole sweep when the log fits kVlogMaxBytes),
    // a few rows at a time in LDS, instead of its two columns being read and
    // written by every step.  The updates go to a second stream, where they
    // overlap the steps of the next run (the steps are latency-bound and
    // leave most of the chip idle); two log buffers alternate, and a step
    // that starts a run waits only for the update that last read its buffer.
    // Every exit joins the second stream into the handle's stream.
    const bool defer_v = V && vlog_rows(n) > 0 && nslots <= 16 * 256;
    h->info.v_deferred = defer_v ? 1 : 0;
    // Two steps per launch (the ring of Alg. 3.1 on even n, each workgroup
    // also running the process after its own): the modified modulus table
    // of the ring, m small enough for one group of 256 threads per pair, V
    // left to the log; the sweep's launches alternate between G and a second
    // copy of it, an even number of them per sweep.  Measured at n = 1024:
    // 61.0 ms with one step per launch, 58.0 with two, 71.8 with four (the
    // recomputed processes, 2.5 times the pair work, cost more than the
    // launches saved).
    int ring_steps = 1;
    // (m > 512: the rows per thread and block reduction of the one-step
    // launches for such m, which the multi-step launches repeat exactly)
    if (o.ordering == JEVD_ORD_MODMODULUS && n % 2 == 0 && n >= 4 && m > 512 &&
        m <= kRingStepsMaxRows && (V == nullptr || defer_v) && nslots == n / 2) {
        if (n % 4 == 0) ring_steps = 2;
    }
    if (ring_steps > 1) {
        st = grow_device(&h->dgalt, &h->capGalt, (size_t)ldg * n);
        if (st) return st;
    }
    h->info.steps_per_launch = ring_steps;
    int chunk = 0;
    if (defer_v) {
        const size_t fit = kVlogMaxBytes / ((size_t)nslots * sizeof(double2));
        chunk = (int)std::min<size_t>((size_t)nsteps, std::max<size_t>(1, fit));
        chunk = std::min(chunk, kVlogMaxSteps);
        // runs of whole multi-step launches
        chunk = std::max(ring_steps, chunk / ring_steps * ring_steps);
        st = grow_device(&h->dvlog, &h->capVlog, (size_t)2 * chunk * nslots);
        if (st) return st;
        if (!h->vstream) HIP_TRY(hipStreamCreateWithFlags(&h->vstream, hipStreamNonBlocking));
        for (int i = 0; i < 2; ++i) {
            if (!h->evLogged[i]) HIP_TRY(hipEventCreateWithFlags(&h->evLogged[i], hipEventDisableTiming));
            if (!h->evApplied[i]) HIP_TRY(hipEventCreateWithFlags(&h->evApplied[i], hipEventDisableTiming));
            // an earlier call that ended on an error may have left an update
            // running on a buffer (an event never recorded is complete)
            HIP_TRY(hipStreamWaitEvent(h->stream, h->evApplied[i], 0));
        }
    }
    bool pending[2] = {false, false};   // an update from buffer b is enqueued
    int runs = 0;
    int result = JEVD_ENOCONV;
    for (int s = 0; s < o.max_sweeps; ++s) {
        // prefetch the V pair while more than a quarter of the pairs rotate
        const bool pf = s == 0 || 4 * (long long)h->hctr[s - 1].rotations > pairs_per_sweep;
        // the step launches of a run (of a sweep without the log) are timed as
        // one group (no events between them)
        HIP_TRY(h->timer.begin(h->stream, JEVD_K_PAIR_STEP));
        int kc = 0, timed = 0;   // first step of the current run; launches in the group
        double2 *logb = nullptr;
        for (int k = 0; k < nsteps; k += ring_steps) {
            if (defer_v && k == kc) {
                const int b = runs % 2;
                if (pending[b]) HIP_TRY(hipStreamWaitEvent(h->stream, h->evApplied[b], 0));
                logb = h->dvlog + (size_t)b * chunk * nslots;
            }
            double2 *logk = defer_v ? logb + (size_t)(k - kc) * nslots : nullptr;
            if (ring_steps > 1) {
                // launch l of the sweep reads the copy it wrote last
                const bool even = (k / ring_steps) % 2 == 0;
                RingStepsArgs ra{even ? G : h->dgalt, even ? h->dgalt : G, m, (long)ldg,
                                 h->dpairs + h->hstep[k], nslots, ring_steps, dJ, tol,
                                 h->dctr + s, h->dslots, h->dslots + nslots, logk, nslots};
                HIP_TRY(launch_pair_steps_ring(ra, h->stream));
            } else {
                PairStepArgs a{G, m, (long)ldg, V, n, (long)ldv, h->dpairs + h->hstep[k],
                               h->hstep[k + 1] - h->hstep[k], dJ, tol, h->dctr + s, pf,
                               h->dslots, h->dslots + nslots, logk};
                HIP_TRY(launch_pair_step(a, h->stream));
            }
            ++timed;
            const int kn = k + ring_steps;   // the next launch's first step
            if (defer_v && (kn - kc == chunk || kn == nsteps)) {
                const int b = runs % 2;
                HIP_TRY(h->timer.end(h->stream, timed));
                timed = 0;
                HIP_TRY(hipEventRecord(h->evLogged[b], h->stream));
                HIP_TRY(hipStreamWaitEvent(h->vstream, h->evLogged[b], 0));
                HIP_TRY(h->timer.begin(h->vstream, JEVD_K_UPDATE));
                VlogApplyArgs va{V, n, n, (long)ldv, h->dpairs, h->dstep, kc, kn, logb,
                                 nslots, h->maxPairsPerStep};
                HIP_TRY(launch_apply_vlog(va, h->vstream));
                HIP_TRY(h->timer.end(h->vstream, 1));
                HIP_TRY(hipEventRecord(h->evApplied[b], h->vstream));
                pending[b] = true;
                ++runs;
                kc = kn;
                if (kn < nsteps) HIP_TRY(h->timer.begin(h->stream, JEVD_K_PAIR_STEP));
            }
        }
        if (!defer_v) HIP_TRY(h->timer.end(h->stream, timed));
        HIP_TRY(launch_sum_slots(h->dslots, h->dslots + nslots, nslots, h->dctr + s, h->stream));
        HIP_TRY(hipMemcpyAsync(h->hctr + s, h->dctr + s, sizeof(SweepCounters), hipMemcpyDeviceToHost,
                               h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        // with the second stream, the timings are collected once it has joined
        if (!defer_v) HIP_TRY(h->timer.collect());
        *sweeps_done = s + 1;
        if (h->hctr[s].nonfinite) {
            result = JEVD_ENONFINITE;
            break;
        }
        if (h->hctr[s].rotations == 0) {
            result = JEVD_OK;
            break;
        }
    }
    if (defer_v) {
        for (int b = 0; b < 2; ++b)
            if (pending[b]) HIP_TRY(hipStreamWaitEvent(h->stream, h->evApplied[b], 0));
        HIP_TRY(hipStreamSynchronize(h->stream));
        HIP_TRY(h->timer.collect());
    }
    return result;
}

int jacobi_evd(jevd_handle_t h, int m, int n, double *G, int ldg, const signed char *J, double tol,
               const jevd_opts *opts, double *lambda, double *U, int ldu, double *V, int ldv,
               int *sweeps)
{
    if (!h || !G) return JEVD_EINVAL;
    jevd_opts o;
    fill_defaults(&o);
    if (opts) o = *opts;
    int st = jevd_validate(m, n, ldg, J, tol, &o, U, ldu, V, ldv);
    if (st) return st;
    if (tol <= 0) tol = n * DBL_EPSILON;
    std::memset(&h->info, 0, sizeof(h->info));
    h->timer.reset();
    if (sweeps) *sweeps = 0;

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != h->device) return JEVD_EINVAL;  // handle belongs to another device

    signed char *dJ = nullptr;
    if (J) {
        st = grow_device(&h->dJ, &h->capJ, (size_t)n);
        if (st) return st;
        HIP_TRY(hipMemcpyAsync(h->dJ, J, (size_t)n, hipMemcpyHostToDevice, h->stream));
        dJ = h->dJ;
    }
    st = ensure_counters(h, o.max_sweeps);
    if (st) return st;
    if (V && !o.accumulate_v) HIP_TRY(launch_identity(V, n, (long)ldv, h->stream));

    int variant = o.variant;
    if (variant == JEVD_VAR_AUTO)
        variant = auto_variant(m, n) ;
    int sweeps_done = 0;
    int status;
    if (variant == JEVD_VAR_POINTWISE) {
        status = run_pointwise(h, m, n, G, ldg, dJ, tol, o, V, ldv, &sweeps_done);
        h->info.block = 0;
        h->info.ordering = o.ordering;
    } else {
        const int b = o.block ? o.block : choose_block_width(m, n);
        BlockRunArgs a{m, n, G, ldg, dJ, J, tol, variant == JEVD_VAR_FULL_BLOCK, b, o.max_sweeps,
                       o.max_inner, V, ldv, o.pivot == JEVD_PIVOT_SIGN, h->stream, h->dctr,
                       h->hctr, &h->timer};
        if (o.precision == JEVD_PREC_MIXED) {
            if (!V) {
                st = grow_device(&h->vtmp, &h->capVtmp, (size_t)n * n);
                if (st) return st;
                a.V = h->vtmp;
                a.ldv = n;
            }
            int low = 0;
            status = run_block_mixed(&h->blk, a, o.max_sweeps, &low, &sweeps_done);
            h->info.sweeps_low = low;
        } else {
            status = run_block(&h->blk, a, &sweeps_done);
        }
        h->info.block = b;
        h->info.ordering = JEVD_ORD_MODMODULUS;
    }
    if (status == JEVD_EHIP || status == JEVD_ENOMEM || status == JEVD_EINVAL) return status;
    h->info.variant = variant;
    h->info.sweeps = sweeps_done;
    for (int s = 0; s < sweeps_done && s < JEVD_INFO_MAX_SWEEPS; ++s) {
        h->info.rotations[s] = (long long)h->hctr[s].rotations;
        h->info.clamps += (long long)h->hctr[s].clamps;
        h->info.breakdowns += (long long)h->hctr[s].breakdowns;
    }
    if (lambda || U) HIP_TRY(launch_finalize(G, m, n, (long)ldg, dJ, lambda, U, (long)ldu, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int c = 0; c < JEVD_K_CLASSES; ++c) {
        h->info.kernel_ms[c] = h->timer.ms[c];
        h->info.kernel_launches[c] = h->timer.launches[c];
    }
    if (sweeps) *sweeps = sweeps_done;
    return status;
}

// Measures the candidate configurations (pointwise; block-oriented and full
// block at every admissible block width) on a working copy of the caller's
// G, each solved to convergence with the caller's J, tol and options, and
// records the fastest for (m, n) in the autotuner table (tune.cpp).
int jevd_autotune(jevd_handle_t h, int m, int n, const double *G, int ldg, const signed char *J,
                  double tol, const jevd_opts *opts, int want_v, int *block, int *variant,
                  double *ms)
{
    if (!h || !G) return JEVD_EINVAL;
    jevd_opts o;
    fill_defaults(&o);
    if (opts) o = *opts;
    o.accumulate_v = 0;
    int st = jevd_validate(m, n, ldg, J, tol, nullptr, nullptr, m, nullptr, n);
    if (st) return st;
    st = grow_device(&h->tuneG, &h->capTuneG, (size_t)m * n);
    if (st) return st;
    if (want_v) {
        st = grow_device(&h->tuneV, &h->capTuneV, (size_t)n * n);
        if (st) return st;
    }
    struct Cand {
        int variant, block;
    };
    std::vector<Cand> cands;
    // Above n = 2048 the pointwise solve (n steps per sweep, each streaming
    // all of G) and b = 16 (n / 16 steps per sweep) take several times as
    // long as the wider blocks, so they are not tried there.
    if (o.pivot == JEVD_PIVOT_NONE && o.precision == JEVD_PREC_FP64 && n <= 2048)
        cands.push_back({JEVD_VAR_POINTWISE, 0});
    for (int v : {JEVD_VAR_BLOCK_ORIENTED, JEVD_VAR_FULL_BLOCK})
        for (int b : {16, 32, 64})
            if ((b > 16 || n <= 2048) && block_options_supported(m, n, b, o.pivot == JEVD_PIVOT_SIGN))
                cands.push_back({v, b});
    int best = -1;
    double best_ms = 0.0;
    for (size_t c = 0; c < cands.size(); ++c) {
        jevd_opts oc = o;
        oc.variant = cands[c].variant;
        oc.block = cands[c].block;
        if (oc.variant == JEVD_VAR_POINTWISE && oc.precision != JEVD_PREC_FP64) continue;
        HIP_TRY(hipMemcpy2DAsync(h->tuneG, sizeof(double) * m, G, sizeof(double) * ldg,
                                 sizeof(double) * m, n, hipMemcpyDeviceToDevice, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        const auto t0 = std::chrono::steady_clock::now();
        int sw = 0;
        const int rc = jacobi_evd(h, m, n, h->tuneG, m, J, tol, &oc, nullptr, nullptr, m,
                                  want_v ? h->tuneV : nullptr, n, &sw);
        const double t = std::chrono::duration<double, std::milli>(
                             std::chrono::steady_clock::now() - t0).count();
        if (rc == JEVD_EHIP || rc == JEVD_ENOMEM) return rc;
        if (rc != JEVD_OK) continue;
        if (best < 0 || t < best_ms) {
            best = (int)c;
            best_ms = t;
        }
    }
    if (best < 0) return JEVD_ENOCONV;
    // the table keeps the record even when the tune file cannot be written
    (void)jevd_tune_record(m, n, cands[best].block, cands[best].variant, best_ms);
    if (block) *block = cands[best].block;
    if (variant) *variant = cands[best].variant;
    if (ms) *ms = best_ms;
    return JEVD_OK;
}

int jevd_canonicalize(jevd_handle_t h, int batch, int m, int n, const double *lam, long long slam,
                      const double *U, int ldu, long long su, const double *V, int ldv,
                      long long sv, double *lam_out, double *U_out, double *V_out)
{
    if (!h || batch < 1 || n < 1 || m < n || !lam || !U || !lam_out || !U_out) return JEVD_EINVAL;
    if (ldu < m || slam < n || su < (long long)ldu * n) return JEVD_EINVAL;
    if ((V == nullptr) != (V_out == nullptr)) return JEVD_EINVAL;
    if (V && (ldv < n || sv < (long long)ldv * n)) return JEVD_EINVAL;
    if (batch > 65535) return JEVD_EINVAL;   // grid y limit of the launch
    HIP_TRY(launch_canonical(batch, m, n, lam, slam, U, ldu, su, V, ldv, sv, lam_out, U_out, V_out,
                             h->stream));
    return JEVD_OK;
}

int jevd_adjoint(jevd_handle_t h, int batch, int m, int n, const double *G, int ldg, long long sg,
                 const signed char *J, long long sj, const double *lam, long long slam,
                 const double *U, int ldu, long long su, const double *w, long long sw,
                 const double *C, int ldc, long long sc, double *dG, int ldd, long long sd)
{
    if (!h || batch < 1 || n < 1 || m < n || !G || !lam || !U || !dG) return JEVD_EINVAL;
    if (ldg < m || ldu < m || ldd < m || slam < n) return JEVD_EINVAL;
    if (sg < (long long)ldg * n || su < (long long)ldu * n || sd < (long long)ldd * n) return JEVD_EINVAL;
    if (J && sj < n) return JEVD_EINVAL;
    if (w && sw < n) return JEVD_EINVAL;
    if (C && (ldc < m || sc < (long long)ldc * n)) return JEVD_EINVAL;
    if (batch > 65535) return JEVD_EINVAL;   // grid z / y limit of the launches
    const size_t nn = (size_t)n * n * batch, mn = (size_t)m * n * batch;
    int st;
    if ((st = grow_device(&h->adjK, &h->capAdjK, nn))) return st;
    if ((st = grow_device(&h->adjW, &h->capAdjW, nn))) return st;
    if ((st = grow_device(&h->adjM, &h->capAdjM, nn))) return st;
    if ((st = grow_device(&h->adjT, &h->capAdjT, mn))) return st;
    HIP_TRY(launch_adjoint(batch, m, n, G, ldg, sg, J, sj, lam, slam, U, ldu, su, w, sw, C, ldc, sc,
                           dG, ldd, sd, h->adjK, h->adjW, h->adjM, h->adjT, h->stream));
    return JEVD_OK;
}

// jevd_adjoint on the library's fixed scratch array instead of the
// handle's work arrays: no allocation at all (for callers that cannot
// allocate).  The kernels and arguments are those of jevd_adjoint; every
// work array is fully written before it is read, so nothing needs clearing.
int jevd_adjoint_noalloc(jevd_handle_t h, int batch, int m, int n, const double *G, int ldg,
                         long long sg, const signed char *J, long long sj, const double *lam,
                         long long slam, const double *U, int ldu, long long su, const double *w,
                         long long sw, const double *C, int ldc, long long sc, double *dG, int ldd,
                         long long sd)
{
    if (!h || batch < 1 || n < 1 || m < n || !G || !lam || !U || !dG) return JEVD_EINVAL;
    if (ldg < m || ldu < m || ldd < m || slam < n) return JEVD_EINVAL;
    if (sg < (long long)ldg * n || su < (long long)ldu * n || sd < (long long)ldd * n) return JEVD_EINVAL;
    if (J && sj < n) return JEVD_EINVAL;
    if (w && sw < n) return JEVD_EINVAL;
    if (C && (ldc < m || sc < (long long)ldc * n)) return JEVD_EINVAL;
    if (batch > 65535) return JEVD_EINVAL;
    const size_t nn = (size_t)n * n * batch, mn = (size_t)m * n * batch;
    if (3 * nn + mn > kScratchDoubles) return JEVD_EINVAL;   // beyond the fixed scratch
    if (!h->scratch) return JEVD_EHIP;
    double *K = h->scratch, *Wk = K + nn, *M = Wk + nn, *T = M + nn;
    HIP_TRY(launch_adjoint(batch, m, n, G, ldg, sg, J, sj, lam, slam, U, ldu, su, w, sw, C, ldc, sc,
                           dG, ldd, sd, K, Wk, M, T, h->stream));
    return JEVD_OK;
}

int jevd_batch_destroy(jevd_batch_t p)
{
    if (!p) return JEVD_OK;
    if (p->ran) (void)hipStreamSynchronize(p->last);
    if (p->arena) {
        // kept by the handle for the next plan (the larger of the two)
        if (p->arena_bytes > p->h->batch_pool_bytes) {
            if (p->h->batch_pool) (void)hipFree(p->h->batch_pool);
            p->h->batch_pool = p->arena;
            p->h->batch_pool_bytes = p->arena_bytes;
        } else {
            (void)hipFree(p->arena);
        }
    }
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->aux) (void)hipStreamDestroy(p->aux);
    delete p;
    return JEVD_OK;
}

int jevd_batch_create(jevd_handle_t h, int batch, const int *m, const int *n, double *const *G,
                      const int *ldg, const signed char *const *J, const double *tol,
                      const jevd_opts *opts, double *const *lambda, double *const *U,
                      const int *ldu, double *const *V, const int *ldv, jevd_batch_t *plan)
{
    if (!plan) return JEVD_EINVAL;
    *plan = nullptr;
    if (!h || batch < 1 || !m || !n || !G || !ldg) return JEVD_EINVAL;
    jevd_opts o;
    fill_defaults(&o);
    if (opts) o = *opts;
    if (o.variant != JEVD_VAR_POINTWISE && o.variant != JEVD_VAR_AUTO) return JEVD_EINVAL;
    std::vector<BatchInst> hi(batch);
    size_t jtotal = 0;
    for (int i = 0; i < batch; ++i) {
        const double *Ui = U ? U[i] : nullptr;
        const double *Vi = V ? V[i] : nullptr;
        const double ti = tol ? tol[i] : 0.0;
        const int st = jevd_validate(m[i], n[i], ldg[i], J ? J[i] : nullptr, ti, &o, Ui,
                                     Ui ? ldu[i] : m[i], Vi, Vi ? ldv[i] : n[i]);
        if (st) return st;
        if (!G[i] || n[i] > kBatchMaxN) return JEVD_EINVAL;
        if (J && J[i]) jtotal += (size_t)n[i];
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != h->device) return JEVD_EINVAL;
    HIP_TRY(prepare_batch_kernel());
    jevd_batch_s *p = new (std::nothrow) jevd_batch_s();
    if (!p) return JEVD_ENOMEM;
    p->h = h;
    p->batch = batch;
    p->ordering = o.ordering;
    p->max_sweeps = o.max_sweeps;
    p->accumulate_v = o.accumulate_v;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    std::vector<signed char> hJ(jtotal > 0 ? jtotal : 1);
    std::vector<size_t> joff(batch, (size_t)-1);
    size_t off = 0;
    for (int i = 0; i < batch; ++i)
        if (J && J[i]) {
            std::memcpy(hJ.data() + off, J[i], (size_t)n[i]);
            joff[i] = off;
            off += (size_t)n[i];
        }
    auto fail = [&](hipError_t e) {
        (void)hipGetLastError();
        jevd_batch_destroy(p);
        return e == hipErrorOutOfMemory ? JEVD_ENOMEM : JEVD_EHIP;
    };
    hipError_t e;
    // one arena for the plan's arrays, 256-byte aligned pieces; the handle's
    // kept arena when it is large enough
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_order = up(sizeof(BatchInst) * batch), o_queue = o_order + up(sizeof(int) * batch),
                 o_sweeps = o_queue + up(sizeof(int) * kBatchClasses),
                 o_status = o_sweeps + up(sizeof(int) * batch), o_J = o_status + up(sizeof(int) * batch),
                 total = o_J + up(hJ.size() + 1);
    if (h->batch_pool && h->batch_pool_bytes >= total) {
        p->arena = h->batch_pool;
        p->arena_bytes = h->batch_pool_bytes;
        h->batch_pool = nullptr;
        h->batch_pool_bytes = 0;
    } else {
        if ((e = hipMalloc(&p->arena, total)) != hipSuccess) return fail(e);
        p->arena_bytes = total;
    }
    char *base = (char *)p->arena;
    p->d_inst = (BatchInst *)base;
    p->d_order = (int *)(base + o_order);
    p->d_queue = (int *)(base + o_queue);
    p->d_sweeps = (int *)(base + o_sweeps);
    p->d_status = (int *)(base + o_status);
    p->d_J = (signed char *)(base + o_J);
    for (int i = 0; i < batch; ++i) {
        BatchInst &d = hi[i];
        d.G = G[i];
        d.V = V ? V[i] : nullptr;
        d.lambda = lambda ? lambda[i] : nullptr;
        d.U = U ? U[i] : nullptr;
        d.J = (joff[i] != (size_t)-1) ? p->d_J + joff[i] : nullptr;
        d.tol = (tol && tol[i] > 0) ? tol[i] : n[i] * DBL_EPSILON;
        d.m = m[i];
        d.n = n[i];
        d.ldg = ldg[i];
        d.ldv = d.V ? ldv[i] : n[i];
        d.ldu = d.U ? ldu[i] : m[i];
    }
    // by size class, largest class first, and within a class longest
    // processing time first (about n^2 m work per sweep); each class is one
    // launch with its own workgroup size: the tuned one if the class's step
    // arrays fit its LDS share, else 16 wavefronts
    std::vector<int> order(batch);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int ca = batch_class_of(n[a]), cb = batch_class_of(n[b]);
        if (ca != cb) return ca > cb;
        return (double)n[a] * n[a] * m[a] > (double)n[b] * n[b] * m[b];
    });
    int nmax[kBatchClasses] = {};
    for (int i = 0; i < batch; ++i) {
        const int c = batch_class_of(n[i]);
        ++p->cls_cnt[c];
        nmax[c] = std::max(nmax[c], n[i]);
    }
    for (int c = kBatchClasses - 1, off = 0; c >= 0; --c) {
        p->cls_off[c] = off;
        off += p->cls_cnt[c];
        if (p->cls_cnt[c] == 0) continue;
        const int tw = tuned_batch_waves(c);
        int w = (tw > 0 && batch_waves_fit(tw, nmax[c])) ? tw : default_batch_waves(c);
        // the tuner times batches of several instances per CU; with at most
        // one per CU a smaller workgroup would leave the rest of the CU idle
        if (p->cls_cnt[c] <= cus) w = 16;
        p->cls_waves[c] = batch_waves_fit(w, nmax[c]) ? w : 16;
        if (p->ngrp > 0 && p->grp_waves[p->ngrp - 1] == p->cls_waves[c]) {
            p->grp_cnt[p->ngrp - 1] += p->cls_cnt[c];
        } else {
            p->grp_off[p->ngrp] = p->cls_off[c];
            p->grp_cnt[p->ngrp] = p->cls_cnt[c];
            p->grp_waves[p->ngrp] = p->cls_waves[c];
            ++p->ngrp;
        }
    }
    for (int g = 0; g < p->ngrp; ++g)
        p->grp_grid[g] = std::min(p->grp_cnt[g], cus * (16 / p->grp_waves[g]));
    if (p->ngrp > 1) {
        if ((e = hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking)) != hipSuccess) return fail(e);
        if ((e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming)) != hipSuccess)
            return fail(e);
        if ((e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming)) != hipSuccess)
            return fail(e);
    }
    // the instance table, the order and the signs in one copy from a pinned
    // image of the arena (copies from pageable memory have stalled for tens
    // of milliseconds)
    const size_t used = o_J + hJ.size();
    if (h->batch_stage_bytes < used) {
        if (h->batch_stage) (void)hipHostFree(h->batch_stage);
        h->batch_stage = nullptr;
        h->batch_stage_bytes = 0;
        if ((e = hipHostMalloc(&h->batch_stage, used, hipHostMallocDefault)) != hipSuccess) return fail(e);
        h->batch_stage_bytes = used;
    }
    char *img = (char *)h->batch_stage;
    std::memset(img, 0, used);
    std::memcpy(img, hi.data(), sizeof(BatchInst) * batch);
    std::memcpy(img + o_order, order.data(), sizeof(int) * batch);
    if (!hJ.empty()) std::memcpy(img + o_J, hJ.data(), hJ.size());
    if ((e = hipMemcpy(p->arena, img, used, hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
    *plan = p;
    return JEVD_OK;
}

int jevd_batch_run(jevd_batch_t p, void *stream)
{
    if (!p) return JEVD_EINVAL;
    hipStream_t st = stream ? (hipStream_t)stream : p->h->stream;
    // the second stream starts from the caller's stream's prior work (event
    // recorded before the first launch) and the caller's stream waits for it
    // at the end; both are events, so a graph capture of the caller's stream
    // takes in the second stream's launches
    if (p->ngrp > 1) {
        HIP_TRY(hipEventRecord(p->ev_fork, st));
        HIP_TRY(hipStreamWaitEvent(p->aux, p->ev_fork, 0));
    }
    for (int g = 0; g < p->ngrp; ++g)
        HIP_TRY(launch_batch(p->d_inst, p->d_order + p->grp_off[g], p->grp_cnt[g], p->d_queue + g,
                             p->ordering, p->max_sweeps, p->accumulate_v, p->d_sweeps, p->d_status,
                             p->grp_grid[g], p->grp_waves[g], g == 0 ? st : p->aux));
    if (p->ngrp > 1) {
        HIP_TRY(hipEventRecord(p->ev_join, p->aux));
        HIP_TRY(hipStreamWaitEvent(st, p->ev_join, 0));
    }
    p->last = st;
    p->ran = true;
    return JEVD_OK;
}

int jevd_batch_results(jevd_batch_t p, int *sweeps, int *status)
{
    if (!p || !p->ran) return JEVD_EINVAL;
    HIP_TRY(hipStreamSynchronize(p->last));
    std::vector<int> sw(p->batch), stv(p->batch);
    HIP_TRY(hipMemcpy(sw.data(), p->d_sweeps, sizeof(int) * p->batch, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(stv.data(), p->d_status, sizeof(int) * p->batch, hipMemcpyDeviceToHost));
    if (sweeps) std::memcpy(sweeps, sw.data(), sizeof(int) * p->batch);
    if (status) std::memcpy(status, stv.data(), sizeof(int) * p->batch);
    for (int i = 0; i < p->batch; ++i)
        if (stv[i] != JEVD_OK) return stv[i];
    return JEVD_OK;
}

int jacobi_evd_batched(jevd_handle_t h, int batch, const int *m, const int *n, double *const *G,
                       const int *ldg, const signed char *const *J, const double *tol,
                       const jevd_opts *opts, double *const *lambda, double *const *U,
                       const int *ldu, double *const *V, const int *ldv, int *sweeps, int *status)
{
    jevd_batch_t p = nullptr;
    int st = jevd_batch_create(h, batch, m, n, G, ldg, J, tol, opts, lambda, U, ldu, V, ldv, &p);
    if (st) return st;
    st = jevd_batch_run(p, nullptr);
    if (st == JEVD_OK) st = jevd_batch_results(p, sweeps, status);
    jevd_batch_destroy(p);
    return st;
}

int jevd_batch_waves(jevd_batch_t p, int *waves)
{
    if (!p || !waves) return JEVD_EINVAL;
    for (int c = 0; c < kBatchClasses; ++c) waves[c] = p->cls_cnt[c] > 0 ? p->cls_waves[c] : 0;
    return JEVD_OK;
}

int jevd_batch_autotune(jevd_handle_t h, int want_v, int *waves_out)
{
    if (!h || (want_v != 0 && want_v != 1)) return JEVD_EINVAL;
    // a representative size per class and the count of instances timed
    static const int rep_n[kBatchClasses] = {40, 80, 128, 192};
    static const int count[kBatchClasses] = {2048, 1024, 1024, 512};
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(prepare_batch_kernel());
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess ||
        cus < 1)
        cus = 256;
    for (int c = 0; c < kBatchClasses; ++c) {
        const int n = rep_n[c], K = count[c];
        const size_t nn = (size_t)n * n;
        double *G0 = nullptr, *G = nullptr, *V = nullptr, *lam = nullptr;
        BatchInst *d_inst = nullptr;
        int *d_order = nullptr, *d_queue = nullptr, *d_sweeps = nullptr, *d_status = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int rc = JEVD_OK, best = -1;
        double best_ms = 0.0;
        auto ok = [&](hipError_t e) {
            if (e != hipSuccess && rc == JEVD_OK) rc = e == hipErrorOutOfMemory ? JEVD_ENOMEM : JEVD_EHIP;
            return rc == JEVD_OK;
        };
        if (ok(hipMalloc(&G0, sizeof(double) * nn * K)) && ok(hipMalloc(&G, sizeof(double) * nn * K)) &&
            (!want_v || ok(hipMalloc(&V, sizeof(double) * nn * K))) &&
            ok(hipMalloc(&lam, sizeof(double) * (size_t)n * K)) &&
            ok(hipMalloc(&d_inst, sizeof(BatchInst) * K)) && ok(hipMalloc(&d_order, sizeof(int) * K)) &&
            ok(hipMalloc(&d_queue, sizeof(int))) && ok(hipMalloc(&d_sweeps, sizeof(int) * K)) &&
            ok(hipMalloc(&d_status, sizeof(int) * K)) && ok(hipEventCreate(&e0)) &&
            ok(hipEventCreate(&e1))) {
            std::vector<BatchInst> hi(K);
            std::vector<int> order(K);
            for (int i = 0; i < K; ++i) {
                BatchInst &d = hi[i];
                d.G = G + nn * i;
                d.V = want_v ? V + nn * i : nullptr;
                d.lambda = lam + (size_t)n * i;
                d.U = nullptr;
                d.J = nullptr;
                d.tol = n * DBL_EPSILON;
                d.m = d.n = d.ldg = d.ldv = d.ldu = n;
                order[i] = i;
            }
            if (ok(hipMemcpy(d_inst, hi.data(), sizeof(BatchInst) * K, hipMemcpyHostToDevice)) &&
                ok(hipMemcpy(d_order, order.data(), sizeof(int) * K, hipMemcpyHostToDevice)) &&
                ok(launch_fill_batch(G0, n, n, K, 1000 + c, h->stream))) {
                for (int w : {4, 8, 16}) {
                    if (!batch_waves_fit(w, n)) continue;
                    const int grid = std::min(K, cus * (16 / w));
                    float best_w = 0.f;
                    for (int rep = 0; rep < 2 && rc == JEVD_OK; ++rep) {
                        float ms = 0.f;
                        if (ok(hipMemcpyAsync(G, G0, sizeof(double) * nn * K, hipMemcpyDeviceToDevice,
                                              h->stream)) &&
                            ok(hipEventRecord(e0, h->stream)) &&
                            ok(launch_batch(d_inst, d_order, K, d_queue, JEVD_ORD_MODMODULUS, 50, 0, d_sweeps,
                                            d_status, grid, w, h->stream)) &&
                            ok(hipEventRecord(e1, h->stream)) && ok(hipEventSynchronize(e1)) &&
                            ok(hipEventElapsedTime(&ms, e0, e1)))
                            best_w = (rep == 0) ? ms : std::min(best_w, ms);
                    }
                    if (rc != JEVD_OK) break;
                    if (best < 0 || best_w < best_ms) {
                        best = w;
                        best_ms = best_w;
                    }
                }
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(G0);
        (void)hipFree(G);
        (void)hipFree(V);
        (void)hipFree(lam);
        (void)hipFree(d_inst);
        (void)hipFree(d_order);
        (void)hipFree(d_queue);
        (void)hipFree(d_sweeps);
        (void)hipFree(d_status);
        if (rc != JEVD_OK) return rc;
        (void)jevd_batch_tune_record(c, best, best_ms);   // an unwritable table file is not an error
        if (waves_out) waves_out[c] = best;
    }
    return JEVD_OK;
}

}  // extern "C"
