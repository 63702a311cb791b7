// Batched pointwise one-sided Jacobi: many independent instances (each its
// own m_i x n_i factor G_i and signature J_i) in one persistent launch.
//
// Each workgroup takes instances from an atomic work queue, largest first
// (the host sorts the queue by n_i^2 m_i, a longest-processing-time order),
// and runs every sweep of an instance in-kernel, as k_small_solve does for a
// single problem: the pairs of each parallel step of the ordering (closed
// form, no tables) are dealt to the wavefronts, lanes run over rows, a
// barrier separates steps, the sweep's rotation count decides convergence.
// G_i and V_i live in LDS when they fit, otherwise they are transformed in
// place in global memory (an instance of n = 256 holds 1 MiB, which the
// 256 MiB Infinity Cache keeps on chip).  The eigenvalues lambda_i and the
// normalised columns U_i are formed at the end of the instance.
#include "../../include/jevd.h"
#include "device_math.h"
#include "jevd_internal.h"
#include "ordering.h"

namespace jevd {

struct BatchInst {
    double *G;
    double *V;
    double *lambda;
    double *U;
    const signed char *J;  // device, or null for J = I
    double tol;
    int m, n, ldg, ldv, ldu;
};

constexpr int kBatchWaves = 16;
constexpr size_t kBatchLdsBytes = 160 * 1024 - 2048;

// pairs of step st of the ordering over n columns (row-cyclic: one pair;
// modulus family: closed form)
__device__ __forceinline__ int batch_step_pairs(int ordering, int n, int st)
{
    if (ordering == kOrdRowCyclic) return 1;
    return modulus_step_pairs(n, st + 1, ordering == kOrdModModulus);
}

__global__ __launch_bounds__(kBatchWaves * 64) void k_batch_solve(
    const BatchInst *__restrict__ inst, const int *__restrict__ order, int batch,
    int *__restrict__ queue, int ordering, int max_sweeps, int accumulate_v,
    int *__restrict__ sweeps_out, int *__restrict__ status_out)
{
    constexpr int NW = kBatchWaves;
    constexpr int BS = NW * 64;
    extern __shared__ double lds[];
    __shared__ int s_idx, s_nonfinite;
    __shared__ unsigned long long s_rot[NW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (;;) {
        if (tid == 0) s_idx = atomicAdd(queue, 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= batch) break;
        const int which = order[idx];
        const BatchInst d = inst[which];
        const int m = d.m, n = d.n;
        // where the instance lives while it is transformed
        const size_t gbytes = (size_t)m * n * sizeof(double);
        const size_t vbytes = d.V ? (size_t)n * n * sizeof(double) : 0;
        const bool lg = gbytes <= kBatchLdsBytes;
        const bool lv = d.V && gbytes + vbytes <= kBatchLdsBytes;
        double *g = d.G;
        long ldg = d.ldg;
        double *v = d.V;
        long ldv = d.ldv;
        if (lg) {
            g = lds;
            ldg = m;
            for (int e = tid; e < m * n; e += BS) g[e] = d.G[(size_t)(e / m) * d.ldg + (e % m)];
        }
        if (d.V) {
            if (lv) {
                v = lds + (size_t)m * n;
                ldv = n;
            }
            for (int e = tid; e < n * n; e += BS) {
                const int r = e % n, c = e / n;
                const double x = accumulate_v ? d.V[(size_t)c * d.ldv + r] : (r == c ? 1.0 : 0.0);
                v[(size_t)c * ldv + r] = x;
            }
        }
        if (tid == 0) s_nonfinite = 0;
        __syncthreads();

        const int nsteps = ordering == kOrdRowCyclic ? n * (n - 1) / 2 : n;
        int sweep = 0, status = JEVD_ENOCONV;
        while (sweep < max_sweeps) {
            unsigned long long rot = 0;
            int rp = 0, rq = 1;  // row-cyclic state: the pair of the current step
            for (int st = 0; st < nsteps; ++st) {
                const int np = batch_step_pairs(ordering, n, st);
                for (int e = wave; e < np; e += NW) {
                    int p, q;
                    if (ordering == kOrdRowCyclic) {
                        p = rp;
                        q = rq;
                    } else {
                        modulus_pair(n, st + 1, e, &p, &q);
                    }
                    double *gp = g + (size_t)p * ldg, *gq = g + (size_t)q * ldg;
                    double app = 0.0, aqq = 0.0, apq = 0.0;
                    for (int r = lane; r < m; r += 64) {
                        const double a = gp[r], b = gq[r];
                        app = fma(a, a, app);
                        aqq = fma(b, b, aqq);
                        apq = fma(a, b, apq);
                    }
                    app = wave_sum(app);
                    aqq = wave_sum(aqq);
                    apq = wave_sum(apq);
                    if (!finite3(app, aqq, apq)) {
                        s_nonfinite = 1;
                        continue;
                    }
                    if (!needs_rotation(app, aqq, apq, d.tol)) continue;
                    const bool same = (d.J == nullptr) || (d.J[p] == d.J[q]);
                    double c, s;
                    transform_params(app, aqq, apq, same, c, s);
                    for (int r = lane; r < m; r += 64) {
                        double a = gp[r], b = gq[r];
                        rotate_elems(a, b, c, s, same);
                        gp[r] = a;
                        gq[r] = b;
                    }
                    if (v) {
                        double *vp = v + (size_t)p * ldv, *vq = v + (size_t)q * ldv;
                        for (int r = lane; r < n; r += 64) {
                            double a = vp[r], b = vq[r];
                            rotate_elems(a, b, c, s, same);
                            vp[r] = a;
                            vq[r] = b;
                        }
                    }
                    ++rot;
                }
                if (ordering == kOrdRowCyclic) {
                    if (++rq == n) {
                        ++rp;
                        rq = rp + 1;
                    }
                } else {
                    __syncthreads();
                }
            }
            if (lane == 0) s_rot[wave] = rot;
            __syncthreads();
            unsigned long long tot = 0;
            for (int w = 0; w < NW; ++w) tot += s_rot[w];
            const int nf = s_nonfinite;
            ++sweep;
            __syncthreads();
            if (nf) {
                status = JEVD_ENONFINITE;
                break;
            }
            if (tot == 0) {
                status = JEVD_OK;
                break;
            }
        }
        // the final iterate back to G (and V), then lambda_i = j_i ||g_i||^2 and
        // u_i = g_i / ||g_i|| (U may be G itself)
        if (lg)
            for (int e = tid; e < m * n; e += BS) d.G[(size_t)(e / m) * d.ldg + (e % m)] = g[e];
        if (lv)
            for (int e = tid; e < n * n; e += BS) {
                const int r = e % n, c = e / n;
                d.V[(size_t)c * d.ldv + r] = v[(size_t)c * ldv + r];
            }
        __syncthreads();
        for (int c = wave; c < n; c += NW) {
            const double *gc = g + (size_t)c * ldg;
            double s2 = 0.0;
            for (int r = lane; r < m; r += 64) s2 = fma(gc[r], gc[r], s2);
            s2 = wave_sum(s2);
            if (d.lambda && lane == 0) d.lambda[c] = (d.J && d.J[c] < 0) ? -s2 : s2;
            if (d.U) {
                const double nrm = sqrt(s2);
                double *uc = d.U + (size_t)c * d.ldu;
                for (int r = lane; r < m; r += 64) uc[r] = (s2 > 0.0) ? gc[r] / nrm : 0.0;
            }
        }
        if (tid == 0) {
            sweeps_out[which] = sweep;
            status_out[which] = status;
        }
        __syncthreads();
    }
}

__global__ void k_reset_queue(int *queue) { *queue = 0; }

hipError_t prepare_batch_kernel()
{
    return hipFuncSetAttribute((const void *)k_batch_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kBatchLdsBytes);
}

hipError_t launch_batch(const BatchInst *inst, const int *order, int batch, int *queue,
                        int ordering, int max_sweeps, int accumulate_v, int *sweeps, int *status,
                        int grid, hipStream_t st)
{
    // the queue is reset by a kernel (not a memset), so the pair of launches
    // can be captured in a graph and replayed
    k_reset_queue<<<1, 1, 0, st>>>(queue);
    k_batch_solve<<<grid, kBatchWaves * 64, kBatchLdsBytes, st>>>(inst, order, batch, queue, ordering,
                                                                  max_sweeps, accumulate_v, sweeps,
                                                                  status);
    return hipGetLastError();
}

}  // namespace jevd
