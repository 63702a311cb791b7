// Batched pointwise one-sided Jacobi: many independent instances (each its
// own m_i x n_i factor G_i and signature J_i) in one persistent launch.
//
// Each workgroup takes instances from an atomic work queue, largest first
// (the host sorts the queue by n_i^2 m_i, a longest-processing-time order),
// and runs every sweep of an instance in-kernel.  A parallel step of the
// ordering (closed form, no tables) runs in three barrier-separated phases:
// Gram sums of all the step's pairs by lane groups, the transforms with one
// lane per pair, then the rotations by the lane groups.  Handing a pair a
// whole wavefront for its scalar part would repeat that arithmetic on 64
// lanes, which made the step VALU-bound.  The sweep's rotation count decides
// convergence.  G_i and V_i live in LDS when they fit, otherwise they are
// transformed in place in global memory (an instance of n = 256 holds 1 MiB,
// which the 256 MiB Infinity Cache keeps on chip).  The eigenvalues
// lambda_i and the normalised columns U_i are formed at the end of the
// instance.
#include <mutex>

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

// A workgroup of NW wavefronts (4, 8 or 16) and NW / 16 of the LDS, so that
// 16 / NW workgroups (instances) share a CU; the wavefronts of a CU are 16
// in every configuration.
constexpr int kBatchWaves = 16;   // the most wavefronts per workgroup
constexpr size_t kBatchLdsBytes = 160 * 1024 - 256;   // the rest: static arrays
__host__ __device__ constexpr size_t batch_lds_bytes(int nw)
{
    return (kBatchLdsBytes * (size_t)nw / kBatchWaves) & ~(size_t)15;
}

// Per-instance context of one workgroup.
struct InstCtx {
    int m, n;
    double tol;
    const signed char *J;  // n signs in LDS
    double *sums;          // LDS: 3 per pair of a step (app, aqq, apq)
    double *rotcs;         // LDS: 2 per pair (c, s)
    int *flag;             // LDS: per pair: 0 none, 1 trigonometric, 2 hyperbolic
    // deferred V (G in HBM): the transforms of up to vsteps steps are logged
    // in LDS and applied to V in row blocks, so V is read and written once
    // per vsteps steps instead of once per step
    int vsteps;            // 0: V is rotated at once
    double *vlog;          // LDS: vsteps x (n/2 + 1) x (c, s)
    int *vflag;            // LDS: vsteps x (n/2 + 1) log_entry words (0: no transform)
    double *vrows;         // LDS: NW * kVRows rows of V, n each
};

constexpr int kVRows = 2;   // rows of V per wavefront in the deferred apply

// A logged transform's word: its type (1 trigonometric, 2 hyperbolic) and
// its columns p < q (n <= 4096), so that applying the log to the rows of V
// reads the pair instead of recomputing it for every row.
__device__ __forceinline__ int log_entry(int type, int p, int q) { return type | (p << 2) | (q << 17); }

// LDS bytes kept beside G and V: the signs and the per-pair step arrays.
// Rounded to 16 bytes so that the arrays at the top of LDS stay aligned.
__host__ __device__ constexpr size_t batch_aux_bytes(int n)
{
    const size_t pairs = (size_t)n / 2 + 1;
    return (pairs * 5 * sizeof(double) + pairs * sizeof(int) + (size_t)n + 15) & ~(size_t)15;
}
static_assert(kBatchLdsBytes % 16 == 0, "LDS top must stay 16-byte aligned");
static_assert(batch_aux_bytes(kBatchMaxN) <= kBatchLdsBytes, "step arrays must fit in LDS");

// Sum over groups of C consecutive lanes (C a power of two, <= 64); lane
// c = 0 of each group ends with the group's total.
__device__ __forceinline__ double group_sum(double x, int C)
{
    if (C >= 2) x += dpp_move<0xB1>(x);    // lane ^ 1
    if (C >= 4) x += dpp_move<0x4E>(x);    // lane ^ 2
    if (C >= 8) x += dpp_move<0x141>(x);   // 7 - i within 8
    if (C >= 16) x += dpp_move<0x140>(x);  // 15 - i within 16
    if (C >= 32) x += __shfl_xor(x, 16);
    if (C >= 64) x += __shfl_xor(x, 32);
    return x;
}

// One parallel step of the modulus family, in three phases separated by
// barriers:
//   1. Gram sums: each pair gets C lanes (C = 64 / pairs per wavefront),
//      lane c sums rows c, c + C, ...; the C partial sums are reduced within
//      the lane group and stored in LDS;
//   2. transforms: one lane per pair decides and computes (c, s), so the
//      scalar arithmetic of a pair runs once, not once per lane of a
//      wavefront;
//   3. rotation of the G (and V) column pairs by the same lane groups.
// g and v are LDS or global pointers of one kind each (see the callers).
template <int NW>
__device__ __forceinline__ void modulus_step(double *g, long ldg, double *v, long ldv,
                                             const InstCtx &c, int k, bool modified,
                                             unsigned &rot, int &bad)
{
    constexpr int BS = NW * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = c.n, m = c.m;
    const int np = modulus_step_pairs(n, k, modified);
    int ppw = 1;  // pairs per wavefront and pass
    while (ppw < 64 && NW * ppw < np) ppw *= 2;
    const int C = 64 / ppw, per_pass = NW * ppw;
    const int sub = lane / C, cl = lane % C;

    for (int base = 0; base < np; base += per_pass) {
        const int e = base + wave * ppw + sub;
        int p = 0, q = 0;
        const bool ok = e < np;
        if (ok) modulus_pair(n, k, e, &p, &q);
        double app = 0.0, aqq = 0.0, apq = 0.0;
        if (ok) {
            const double *gp = g + (size_t)p * ldg, *gq = g + (size_t)q * ldg;
            for (int r = cl; r < m; r += C) {
                const double x = gp[r], y = gq[r];
                app = fma(x, x, app);
                aqq = fma(y, y, aqq);
                apq = fma(x, y, apq);
            }
        }
        app = group_sum(app, C);
        aqq = group_sum(aqq, C);
        apq = group_sum(apq, C);
        if (ok && cl == 0) {
            c.sums[3 * e] = app;
            c.sums[3 * e + 1] = aqq;
            c.sums[3 * e + 2] = apq;
        }
    }
    __syncthreads();
    for (int e = tid; e < np; e += BS) {
        const double app = c.sums[3 * e], aqq = c.sums[3 * e + 1], apq = c.sums[3 * e + 2];
        int f = 0;
        if (!finite3(app, aqq, apq)) {
            bad = 1;
        } else if (needs_rotation(app, aqq, apq, c.tol)) {
            int p, q;
            modulus_pair(n, k, e, &p, &q);
            const bool same = c.J[p] == c.J[q];
            double cs, sn;
            // one lane per pair: pairs of both signs share the wavefront
            transform_params_bf(app, aqq, apq, same, cs, sn);
            c.rotcs[2 * e] = cs;
            c.rotcs[2 * e + 1] = sn;
            f = same ? 1 : 2;
            ++rot;
        }
        c.flag[e] = f;
    }
    __syncthreads();
    for (int base = 0; base < np; base += per_pass) {
        const int e = base + wave * ppw + sub;
        if (e >= np) continue;
        const int f = c.flag[e];
        if (f == 0) continue;
        int p, q;
        modulus_pair(n, k, e, &p, &q);
        const double cs = c.rotcs[2 * e], sn = c.rotcs[2 * e + 1];
        const bool same = f == 1;
        double *gp = g + (size_t)p * ldg, *gq = g + (size_t)q * ldg;
        for (int r = cl; r < m; r += C) {
            double x = gp[r], y = gq[r];
            rotate_elems(x, y, cs, sn, same);
            gp[r] = x;
            gq[r] = y;
        }
        if (v) {
            double *vp = v + (size_t)p * ldv, *vq = v + (size_t)q * ldv;
            for (int r = cl; r < n; r += C) {
                double x = vp[r], y = vq[r];
                rotate_elems(x, y, cs, sn, same);
                vp[r] = x;
                vq[r] = y;
            }
        }
    }
    __syncthreads();
}

// The step path for G in global memory: a wavefront takes one or two
// pairs (p0, q0), (p1, q1) at a time and keeps their rows in registers from
// the Gram sums to the rotation, so each element is read once per step; the
// V rows are loaded with the G rows, so their latencies overlap.  Lane l
// owns rows l, l + 64, ..., l + 64 (R - 1) (m <= 64 R).  The transform is
// computed on the whole wavefront (one useful value), which is affordable
// here because the step is bound by the global traffic.
template <int R>
__device__ __forceinline__ void two_pairs(double *g, long ldg, double *v, long ldv,
                                          const InstCtx &c, int p0, int q0, bool has1, int p1,
                                          int q1, int lane, unsigned &rot, int &bad,
                                          double *logcs = nullptr, int *logfl = nullptr,
                                          int e0 = 0, int e1 = 0)
{
    const int pp[2] = {p0, p1}, qq[2] = {q0, q1}, ee[2] = {e0, e1};
    if (logfl && lane == 0) {   // every logged pair gets an entry; rotated ones overwrite it
        logfl[e0] = 0;
        if (has1) logfl[e1] = 0;
    }
    double a[2][R], b[2][R], va[2][R], vb[2][R];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && !has1) break;
        const double *gp = g + (size_t)pp[k] * ldg, *gq = g + (size_t)qq[k] * ldg;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = lane + 64 * i;
            a[k][i] = r < c.m ? gp[r] : 0.0;
            b[k][i] = r < c.m ? gq[r] : 0.0;
        }
        if (v) {
            const double *vp = v + (size_t)pp[k] * ldv, *vq = v + (size_t)qq[k] * ldv;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = lane + 64 * i;
                va[k][i] = r < c.n ? vp[r] : 0.0;
                vb[k][i] = r < c.n ? vq[r] : 0.0;
            }
        }
    }
    double app[2] = {0.0, 0.0}, aqq[2] = {0.0, 0.0}, apq[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && !has1) break;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            app[k] = fma(a[k][i], a[k][i], app[k]);
            aqq[k] = fma(b[k][i], b[k][i], aqq[k]);
            apq[k] = fma(a[k][i], b[k][i], apq[k]);
        }
        app[k] = wave_sum(app[k]);
        aqq[k] = wave_sum(aqq[k]);
        apq[k] = wave_sum(apq[k]);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && !has1) break;
        if (!finite3(app[k], aqq[k], apq[k])) {
            bad = 1;
            continue;
        }
        if (!needs_rotation(app[k], aqq[k], apq[k], c.tol)) continue;
        const bool same = c.J[pp[k]] == c.J[qq[k]];
        double cs, sn;
        transform_params(app[k], aqq[k], apq[k], same, cs, sn);
        if (logfl && lane == 0) {
            logcs[2 * ee[k]] = cs;
            logcs[2 * ee[k] + 1] = sn;
            logfl[ee[k]] = log_entry(same ? 1 : 2, pp[k], qq[k]);
        }
        double *gp = g + (size_t)pp[k] * ldg, *gq = g + (size_t)qq[k] * ldg;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = lane + 64 * i;
            rotate_elems(a[k][i], b[k][i], cs, sn, same);
            if (r < c.m) {
                gp[r] = a[k][i];
                gq[r] = b[k][i];
            }
        }
        if (v) {
            double *vp = v + (size_t)pp[k] * ldv, *vq = v + (size_t)qq[k] * ldv;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = lane + 64 * i;
                rotate_elems(va[k][i], vb[k][i], cs, sn, same);
                if (r < c.n) {
                    vp[r] = va[k][i];
                    vq[r] = vb[k][i];
                }
            }
        }
        if (lane == 0) ++rot;
    }
}

// two_pairs without V (V logged or absent), with the scalar part of the two
// pairs in one pass: lane k (k = lane & 1) runs the threshold test and the
// transform of pair k, and lanes 0 and 1 hand the results to the wavefront.
// The step is bound by VALU issue, and the transform is most of a pair's
// instructions, so two pairs share one pass instead of running one each.
// Each lane runs the per-pair expressions of two_pairs on the same sums
// (transform_params_bf gives transform_params' values), so the results are
// the same to the bit.
template <int R>
__device__ __forceinline__ void two_pairs_nov(double *g, long ldg, const InstCtx &c, int p0, int q0,
                                              bool has1, int p1, int q1, int lane, unsigned &rot,
                                              int &bad, double *logcs, int *logfl, int e0, int e1)
{
    const int pp[2] = {p0, p1}, qq[2] = {q0, q1};
    double a[2][R], b[2][R];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && !has1) break;
        const double *gp = g + (size_t)pp[k] * ldg, *gq = g + (size_t)qq[k] * ldg;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = lane + 64 * i;
            a[k][i] = r < c.m ? gp[r] : 0.0;
            b[k][i] = r < c.m ? gq[r] : 0.0;
        }
    }
    double app[2] = {0.0, 0.0}, aqq[2] = {0.0, 0.0}, apq[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && !has1) break;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            app[k] = fma(a[k][i], a[k][i], app[k]);
            aqq[k] = fma(b[k][i], b[k][i], aqq[k]);
            apq[k] = fma(a[k][i], b[k][i], apq[k]);
        }
        app[k] = wave_sum(app[k]);
        aqq[k] = wave_sum(aqq[k]);
        apq[k] = wave_sum(apq[k]);
    }
    const bool odd = (lane & 1) != 0;
    const double sp = odd ? app[1] : app[0], sq = odd ? aqq[1] : aqq[0], spq = odd ? apq[1] : apq[0];
    const bool same = odd ? c.J[p1] == c.J[q1] : c.J[p0] == c.J[q0];
    const bool fin = finite3(sp, sq, spq);
    int f = 0;
    double cs = 0.0, sn = 0.0;
    if ((!odd || has1) && fin && needs_rotation(sp, sq, spq, c.tol)) {
        transform_params_bf(sp, sq, spq, same, cs, sn);
        f = same ? 1 : 2;
    }
    const int fk[2] = {__builtin_amdgcn_readlane(f, 0), __builtin_amdgcn_readlane(f, 1)};
    const int nonfin = __builtin_amdgcn_readlane((int)!fin, 0) | (has1 ? __builtin_amdgcn_readlane((int)!fin, 1) : 0);
    if (nonfin) bad = 1;
    const double ck[2] = {read_lane(cs, 0), read_lane(cs, 1)}, sk[2] = {read_lane(sn, 0), read_lane(sn, 1)};
    if (logfl && lane == 0) {   // every logged pair gets an entry (0: no transform)
        logfl[e0] = fk[0] ? log_entry(fk[0], p0, q0) : 0;
        if (fk[0]) {
            logcs[2 * e0] = ck[0];
            logcs[2 * e0 + 1] = sk[0];
        }
        if (has1) {
            logfl[e1] = fk[1] ? log_entry(fk[1], p1, q1) : 0;
            if (fk[1]) {
                logcs[2 * e1] = ck[1];
                logcs[2 * e1 + 1] = sk[1];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && !has1) break;
        if (!fk[k]) continue;
        const bool sm = fk[k] == 1;
        double *gp = g + (size_t)pp[k] * ldg, *gq = g + (size_t)qq[k] * ldg;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = lane + 64 * i;
            rotate_elems(a[k][i], b[k][i], ck[k], sk[k], sm);
            if (r < c.m) {
                gp[r] = a[k][i];
                gq[r] = b[k][i];
            }
        }
        if (lane == 0) ++rot;
    }
}

// One step over G in global memory by the register path (R > 0; two pairs
// per wavefront for R <= 2, one for R = 4, registers permitting).
template <int NW, int R>
__device__ __forceinline__ void global_step(double *g, long ldg, double *v, long ldv,
                                            const InstCtx &c, int k, bool modified, unsigned &rot,
                                            int &bad, double *logcs, int *logfl)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int np = modulus_step_pairs(c.n, k, modified);
    if (!v) {
        for (int e = wave; e < np; e += 2 * NW) {
            int p0, q0, p1 = 0, q1 = 0;
            modulus_pair(c.n, k, e, &p0, &q0);
            const bool has1 = e + NW < np;
            if (has1) modulus_pair(c.n, k, e + NW, &p1, &q1);
            two_pairs_nov<R>(g, ldg, c, p0, q0, has1, p1, q1, lane, rot, bad, logcs, logfl, e, e + NW);
        }
    } else if constexpr (R <= 2) {
        for (int e = wave; e < np; e += 2 * NW) {
            int p0, q0, p1 = 0, q1 = 0;
            modulus_pair(c.n, k, e, &p0, &q0);
            const bool has1 = e + NW < np;
            if (has1) modulus_pair(c.n, k, e + NW, &p1, &q1);
            two_pairs<R>(g, ldg, v, ldv, c, p0, q0, has1, p1, q1, lane, rot, bad, logcs, logfl, e,
                         e + NW);
        }
    } else {
        for (int e = wave; e < np; e += NW) {
            int p, q;
            modulus_pair(c.n, k, e, &p, &q);
            two_pairs<R>(g, ldg, v, ldv, c, p, q, false, 0, 0, lane, rot, bad, logcs, logfl, e, 0);
        }
    }
    __syncthreads();
}

// Applies the logged transforms of steps kfirst .. kfirst + nsteps - 1 to V
// (HBM, column-major): blocks of NW * kVRows rows are staged in LDS;
// a wavefront owns kVRows rows and runs every logged step on them, lanes over
// the step's pairs, each log entry (pair, type, c, s) read once for its rows.
// A row's elements meet the same transforms in the same order as by
// immediate application; each element's rotation is c x -+ s y with the
// products fused as the compiler chooses at this site, so V can differ from
// immediate application in the last bit of an element.
template <int NW>
__device__ __forceinline__ void apply_v_log(double *v, long ldv, const InstCtx &c, int kfirst,
                                            int nsteps, bool modified)
{
    constexpr int BS = NW * 64, RB = NW * kVRows;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = c.n, lp = n / 2 + 1;
    for (int r0 = 0; r0 < n; r0 += RB) {
        const int nr = min(RB, n - r0);
        for (int e = tid; e < RB * n; e += BS) {
            const int i = e % RB, col = e / RB;
            if (i < nr) c.vrows[i * n + col] = v[(size_t)col * ldv + r0 + i];
        }
        __syncthreads();
        // both rows of the wavefront in one pass over the log, each logged
        // entry read once for the two
        static_assert(kVRows == 2, "the pass below takes two rows");
        const int i0 = wave * kVRows;
        if (i0 < nr) {
            double *row0 = c.vrows + (size_t)i0 * n, *row1 = row0 + n;
            const bool has1 = i0 + 1 < nr;
            for (int st = 0; st < nsteps; ++st) {
                const int np = modulus_step_pairs(n, kfirst + st, modified);
                for (int e = lane; e < np; e += 64) {
                    const int f = c.vflag[st * lp + e];
                    if (f == 0) continue;
                    const int p = (f >> 2) & 0x7fff, q = f >> 17;
                    const double cs = c.vlog[2 * (st * lp + e)], sn = c.vlog[2 * (st * lp + e) + 1];
                    const bool same = (f & 3) == 1;
                    double x = row0[p], y = row0[q];
                    rotate_elems(x, y, cs, sn, same);
                    row0[p] = x;
                    row0[q] = y;
                    if (has1) {
                        x = row1[p];
                        y = row1[q];
                        rotate_elems(x, y, cs, sn, same);
                        row1[p] = x;
                        row1[q] = y;
                    }
                }
                // the next step's pairs read columns other lanes wrote: the
                // LDS accesses of one wavefront complete in order, and the
                // fences keep the compiler from moving them across
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        __syncthreads();
        for (int e = tid; e < RB * n; e += BS) {
            const int i = e % RB, col = e / RB;
            if (i < nr) v[(size_t)col * ldv + r0 + i] = c.vrows[i * n + col];
        }
        __syncthreads();
    }
}

// One pair with rows looped over by one wavefront (the row-cyclic path).
__device__ __forceinline__ void one_pair_loop(double *g, long ldg, double *v, long ldv,
                                              const InstCtx &c, int p, int q, int lane,
                                              unsigned &rot, int &bad)
{
    double *gp = g + (size_t)p * ldg, *gq = g + (size_t)q * ldg;
    double app = 0.0, aqq = 0.0, apq = 0.0;
    for (int r = lane; r < c.m; r += 64) {
        const double x = gp[r], y = gq[r];
        app = fma(x, x, app);
        aqq = fma(y, y, aqq);
        apq = fma(x, y, apq);
    }
    app = wave_sum(app);
    aqq = wave_sum(aqq);
    apq = wave_sum(apq);
    if (!finite3(app, aqq, apq)) {
        bad = 1;
        return;
    }
    if (!needs_rotation(app, aqq, apq, c.tol)) return;
    const bool same = c.J[p] == c.J[q];
    double cs, sn;
    transform_params(app, aqq, apq, same, cs, sn);
    for (int r = lane; r < c.m; r += 64) {
        double x = gp[r], y = gq[r];
        rotate_elems(x, y, cs, sn, same);
        gp[r] = x;
        gq[r] = y;
    }
    if (v) {
        double *vp = v + (size_t)p * ldv, *vq = v + (size_t)q * ldv;
        for (int r = lane; r < c.n; r += 64) {
            double x = vp[r], y = vq[r];
            rotate_elems(x, y, cs, sn, same);
            vp[r] = x;
            vq[r] = y;
        }
    }
    if (lane == 0) ++rot;
}

// All sweeps of one instance on (g, v); returns the status and sets sweeps.
// R = 0: the phased step (G in LDS, or m > 256); R > 0: the register step.
template <int NW, int R>
__device__ __forceinline__ int sweep_instance(double *g, long ldg, double *v, long ldv,
                                              const InstCtx &c, int ordering, int max_sweeps,
                                              int &sweeps, unsigned *s_rot, int *s_bad)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = c.n;
    int sweep = 0, status = JEVD_ENOCONV;
    int bad = 0;
    while (sweep < max_sweeps) {
        unsigned rot = 0;
        if (ordering == kOrdRowCyclic) {
            // the steps of equal p + q (the same result as one pair at a
            // time in row order), a pair per wavefront
            for (int t = 1; t <= rowcyclic_steps(n); ++t) {
                const int p0 = rowcyclic_first(n, t), np = rowcyclic_step_pairs(n, t);
                for (int e = wave; e < np; e += NW)
                    one_pair_loop(g, ldg, v, ldv, c, p0 + e, t - p0 - e, lane, rot, bad);
                __syncthreads();
            }
        } else {
            const bool modified = ordering == kOrdModModulus;
            if constexpr (R > 0) {
                const bool defer = v && c.vsteps > 0;
                const int lp = n / 2 + 1;
                int inchunk = 0, kfirst = 1;
                for (int k = 1; k <= n; ++k) {
                    global_step<NW, R>(g, ldg, defer ? nullptr : v, ldv, c, k, modified, rot, bad,
                                   defer ? c.vlog + 2 * (size_t)inchunk * lp : nullptr,
                                   defer ? c.vflag + (size_t)inchunk * lp : nullptr);
                    if (defer && (++inchunk == c.vsteps || k == n)) {
                        apply_v_log<NW>(v, ldv, c, kfirst, inchunk, modified);
                        inchunk = 0;
                        kfirst = k + 1;
                    }
                }
            } else {
                for (int k = 1; k <= n; ++k) modulus_step<NW>(g, ldg, v, ldv, c, k, modified, rot, bad);
            }
        }
        // workgroup totals: rotations and the non-finite flag
        unsigned r = rot;
        int b = bad;
        for (int off = 32; off > 0; off >>= 1) {
            r += __shfl_xor(r, off);
            b |= __shfl_xor(b, off);
        }
        if (lane == 0) {
            s_rot[wave] = r;
            s_bad[wave] = b;
        }
        __syncthreads();
        unsigned tot = 0;
        int nf = 0;
        for (int w = 0; w < NW; ++w) {
            tot += s_rot[w];
            nf |= s_bad[w];
        }
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
    sweeps = sweep;
    return status;
}

// Sixteen wavefronts per CU in every configuration (16 / NW workgroups), so
// the register budget is that of four wavefronts per SIMD.
template <int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_solve(
    const BatchInst *__restrict__ inst, const int *__restrict__ order, int batch,
    int *__restrict__ queue, int ordering, int max_sweeps, int accumulate_v,
    int *__restrict__ sweeps_out, int *__restrict__ status_out)
{
    constexpr int BS = NW * 64;
    constexpr size_t LB = batch_lds_bytes(NW);   // this workgroup's LDS
    extern __shared__ double lds[];
    __shared__ int s_idx;
    __shared__ unsigned s_rot[NW];
    __shared__ int s_bad[NW];
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
        // where the instance lives while it is transformed: G (and V) in LDS
        // when they fit beside the signs and step arrays at the top of LDS,
        // else in place in global memory
        const size_t aux = batch_aux_bytes(n);
        if (aux > LB) {
            // the step arrays do not fit this workgroup's LDS (the host
            // assigns such sizes to 16-wavefront workgroups only)
            if (tid == 0) {
                sweeps_out[which] = 0;
                status_out[which] = JEVD_EINVAL;
            }
            __syncthreads();
            continue;
        }
        const size_t gbytes = (size_t)m * n * sizeof(double);
        const size_t vbytes = d.V ? (size_t)n * n * sizeof(double) : 0;
        const bool lg = gbytes + aux <= LB;
        const bool lv = d.V && gbytes + vbytes + aux <= LB;
        const size_t pairs = (size_t)n / 2 + 1;
        char *top = (char *)lds + (LB - aux);
        InstCtx c;
        c.m = m;
        c.n = n;
        c.tol = d.tol;
        c.sums = (double *)top;
        c.rotcs = c.sums + 3 * pairs;
        c.flag = (int *)(c.rotcs + 2 * pairs);
        signed char *sJ = (signed char *)(c.flag + pairs);
        c.J = sJ;
        c.vsteps = 0;
        c.vlog = nullptr;
        c.vflag = nullptr;
        c.vrows = nullptr;
        if (!lg && d.V && m <= 256) {
            // G in HBM (the register path): LDS below the step arrays holds
            // the V row blocks and the transform log of vsteps steps
            const size_t free_bytes = LB - aux;
            const size_t rows_bytes = (size_t)NW * kVRows * n * sizeof(double);
            const size_t per_step = pairs * (2 * sizeof(double) + sizeof(int));
            if (free_bytes > rows_bytes + 4 * per_step) {
                size_t vs = (free_bytes - rows_bytes) / per_step;
                c.vsteps = (int)(vs > 32 ? 32 : vs);
                c.vrows = lds;
                c.vlog = lds + (size_t)NW * kVRows * n;
                c.vflag = (int *)(c.vlog + 2 * (size_t)c.vsteps * pairs);
            }
        }
        for (int e = tid; e < n; e += BS) sJ[e] = (d.J && d.J[e] < 0) ? -1 : 1;
        if (lg)
            for (int e = tid; e < m * n; e += BS) lds[e] = d.G[(size_t)(e / m) * d.ldg + (e % m)];
        if (d.V) {
            double *v = lv ? lds + (size_t)m * n : d.V;
            const long ldv = lv ? n : d.ldv;
            for (int e = tid; e < n * n; e += BS) {
                const int r = e % n, cc = e / n;
                const double x = accumulate_v ? d.V[(size_t)cc * d.ldv + r] : (r == cc ? 1.0 : 0.0);
                v[(size_t)cc * ldv + r] = x;
            }
        }
        __syncthreads();
        int sweep = 0, status;
        if (lg && lv)
            status = sweep_instance<NW, 0>(lds, m, lds + (size_t)m * n, n, c, ordering, max_sweeps, sweep,
                                       s_rot, s_bad);
        else if (lg)
            status = sweep_instance<NW, 0>(lds, m, d.V, d.ldv, c, ordering, max_sweeps, sweep, s_rot,
                                       s_bad);
        else if (m <= 128)
            status = sweep_instance<NW, 2>(d.G, d.ldg, d.V, d.ldv, c, ordering, max_sweeps, sweep, s_rot,
                                       s_bad);
        else if (m <= 256)
            status = sweep_instance<NW, 4>(d.G, d.ldg, d.V, d.ldv, c, ordering, max_sweeps, sweep, s_rot,
                                       s_bad);
        else
            status = sweep_instance<NW, 0>(d.G, d.ldg, d.V, d.ldv, c, ordering, max_sweeps, sweep, s_rot,
                                       s_bad);
        // the final iterate back to G (and V), then lambda_i = j_i ||g_i||^2 and
        // u_i = g_i / ||g_i|| (U may be G itself)
        if (lg)
            for (int e = tid; e < m * n; e += BS) d.G[(size_t)(e / m) * d.ldg + (e % m)] = lds[e];
        if (lv)
            for (int e = tid; e < n * n; e += BS) {
                const int r = e % n, cc = e / n;
                d.V[(size_t)cc * d.ldv + r] = lds[(size_t)m * n + (size_t)cc * n + r];
            }
        __syncthreads();
        for (int cc = wave; cc < n; cc += NW) {
            const double *gc = lg ? lds + (size_t)cc * m : d.G + (size_t)cc * d.ldg;
            double s2 = 0.0;
            for (int r = lane; r < m; r += 64) s2 = fma(gc[r], gc[r], s2);
            s2 = wave_sum(s2);
            if (d.lambda && lane == 0) d.lambda[cc] = sJ[cc] < 0 ? -s2 : s2;
            if (d.U) {
                const double nrm = sqrt(s2);
                double *uc = d.U + (size_t)cc * d.ldu;
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

// The LDS limits are set once per device (a plan is created per call by
// some callers, and the attribute calls cost about a millisecond each).
static hipError_t set_batch_lds_limits()
{
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)k_batch_solve<4>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)batch_lds_bytes(4))) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void *)k_batch_solve<8>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)batch_lds_bytes(8))) != hipSuccess)
        return e;
    return hipFuncSetAttribute((const void *)k_batch_solve<16>,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)batch_lds_bytes(16));
}

hipError_t prepare_batch_kernel()
{
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    if (dev >= 0 && dev < 64 && done[dev]) return hipSuccess;
    if ((e = set_batch_lds_limits()) != hipSuccess) return e;
    if (dev >= 0 && dev < 64) done[dev] = true;
    return hipSuccess;
}

bool batch_waves_supported(int waves) { return waves == 4 || waves == 8 || waves == 16; }

int batch_class_of(int n)
{
    for (int c = 0; c < kBatchClasses; ++c)
        if (n <= kBatchClassMax[c]) return c;
    return kBatchClasses - 1;
}

int default_batch_waves(int cls)
{
    (void)cls;
    return kBatchWaves;
}

bool batch_waves_fit(int waves, int nmax)
{
    return batch_waves_supported(waves) && batch_aux_bytes(nmax) <= batch_lds_bytes(waves);
}

// Seeded fill for the tuner's instances: x_i = (2 u_i - 1) 10^(2 w_c - 1)
// with u_i, w_c uniform from a counter hash (splitmix64) of (seed, i) and
// (seed, column c), so the columns are graded over two decades.
__device__ __forceinline__ double hash_unit(unsigned long long x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * 0x1.0p-53;
}

__global__ void k_fill_batch(double *G, int m, int n, long count, unsigned long long seed)
{
    const long total = count * (long)m * n;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total;
         i += (long)gridDim.x * blockDim.x) {
        const long col = i / m;   // column over all instances
        const double w = hash_unit(seed * 0x100000001B3ull + 2 * col + 1);
        G[i] = (2.0 * hash_unit(seed ^ (0xA5A5A5A5ull + 2 * i)) - 1.0) * exp10(2.0 * w - 1.0);
    }
}

hipError_t launch_fill_batch(double *G, int m, int n, long count, unsigned long long seed,
                             hipStream_t st)
{
    k_fill_batch<<<1024, 256, 0, st>>>(G, m, n, count, seed);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchInst *inst, const int *order, int batch, int *queue,
                        int ordering, int max_sweeps, int accumulate_v, int *sweeps, int *status,
                        int grid, int waves, hipStream_t st)
{
    // the queue is reset by a kernel (not a memset), so the pair of launches
    // can be captured in a graph and replayed
    k_reset_queue<<<1, 1, 0, st>>>(queue);
    if (waves == 4)
        k_batch_solve<4><<<grid, 4 * 64, batch_lds_bytes(4), st>>>(inst, order, batch, queue, ordering,
                                                                   max_sweeps, accumulate_v, sweeps,
                                                                   status);
    else if (waves == 8)
        k_batch_solve<8><<<grid, 8 * 64, batch_lds_bytes(8), st>>>(inst, order, batch, queue, ordering,
                                                                   max_sweeps, accumulate_v, sweeps,
                                                                   status);
    else
        k_batch_solve<16><<<grid, 16 * 64, batch_lds_bytes(16), st>>>(inst, order, batch, queue,
                                                                      ordering, max_sweeps,
                                                                      accumulate_v, sweeps, status);
    return hipGetLastError();
}

}  // namespace jevd
