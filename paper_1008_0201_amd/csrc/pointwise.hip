// Pointwise one-sided Jacobi kernels for gfx950 (Sec. 2.1).
//
//   k_pair_step        one parallel step: one workgroup per pivot pair; the
//                      pair's two columns stay in registers between the Gram
//                      pass and the rotation pass (m <= BS * CH).
//   k_pair_step_stream the same for taller columns: the columns are read
//                      twice (Gram pass, rotation pass).
//   k_apply_vlog       the deferred V update: with a rotation log the step
//                      kernels leave V alone and record each pair's (c, s);
//                      this kernel then applies a run of logged steps to a
//                      few rows of V held in LDS.
//   k_small_solve      a whole solve (all sweeps) of a small problem in one
//                      workgroup, with G and V resident in LDS; used for the
//                      row-cyclic ordering, whose pairs are strictly
//                      sequential, and for small n.
//   k_identity, k_finalize  V := I; lambda_i = j_i ||g_i||^2, u_i = g_i / ||g_i||.
#include <map>
#include <mutex>
#include "device_math.h"
#include "jevd_internal.h"
#include "ordering.h"

namespace jevd {

// Rotate the column pair (vp, vq) of length len with BS threads; loads of a
// chunk of 4 strided elements are issued before the dependent stores.
template <int BS>
__device__ __forceinline__ void rotate_columns(double *__restrict__ vp, double *__restrict__ vq,
                                               int len, double c, double s, bool same)
{
    int r = threadIdx.x;
    for (; r + 3 * BS < len; r += 4 * BS) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = vp[r + u * BS];
            b[u] = vq[r + u * BS];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            rotate_elems(a[u], b[u], c, s, same);
            vp[r + u * BS] = a[u];
            vq[r + u * BS] = b[u];
        }
    }
    for (; r < len; r += BS) {
        double a = vp[r], b = vq[r];
        rotate_elems(a, b, c, s, same);
        vp[r] = a;
        vq[r] = b;
    }
}

// One entry of the rotation log: (c, s) of the pair's transform, with c
// negated for a hyperbolic one (c = cos or cosh is positive, so the sign is
// free); (1, 0) for a pair that does not rotate (the identity, exactly).
__device__ __forceinline__ double2 log_entry(double c, double s, bool same)
{
    return make_double2(same ? c : -c, s);
}

// PF: the V pair (nv <= BS * CH rows) is loaded together with the G pair,
// before the rotation decision, so that both loads are in flight at once;
// worth it when most pairs of the sweep rotate.
template <int BS, int CH, bool PF>
__global__ __launch_bounds__(BS) void k_pair_step(double *__restrict__ G, int m, long ldg,
                                                  double *__restrict__ V, int nv, long ldv,
                                                  const int2 *__restrict__ pairs,
                                                  const signed char *__restrict__ J, double tol,
                                                  SweepCounters *__restrict__ ctr,
                                                  unsigned *__restrict__ slot_rot,
                                                  unsigned *__restrict__ slot_clamp,
                                                  double2 *__restrict__ vlog)
{
    __shared__ double sh[3 * BS / kWave];
    const int2 pq = pairs[blockIdx.x];
    double *gp = G + (size_t)pq.x * ldg;
    double *gq = G + (size_t)pq.y * ldg;
    double xp[CH], xq[CH];
    double wp[PF ? CH : 1], wq[PF ? CH : 1];
    double *vp = V ? V + (size_t)pq.x * ldv : nullptr;
    double *vq = V ? V + (size_t)pq.y * ldv : nullptr;
    double app = 0.0, aqq = 0.0, apq = 0.0;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int r = threadIdx.x + k * BS;
        xp[k] = (r < m) ? gp[r] : 0.0;
        xq[k] = (r < m) ? gq[r] : 0.0;
    }
    if constexpr (PF) {
        if (V) {
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int r = threadIdx.x + k * BS;
                wp[k] = (r < nv) ? vp[r] : 0.0;
                wq[k] = (r < nv) ? vq[r] : 0.0;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        app = fma(xp[k], xp[k], app);
        aqq = fma(xq[k], xq[k], aqq);
        apq = fma(xp[k], xq[k], apq);
    }
    block_sum3<BS>(app, aqq, apq, sh);
    if (!finite3(app, aqq, apq)) {
        if (threadIdx.x == 0) {
            ctr->nonfinite = 1u;
            if (vlog) vlog[blockIdx.x] = make_double2(1.0, 0.0);
        }
        return;
    }
    if (!needs_rotation(app, aqq, apq, tol)) {
        if (vlog && threadIdx.x == 0) vlog[blockIdx.x] = make_double2(1.0, 0.0);
        return;
    }
    const bool same = (J == nullptr) || (J[pq.x] == J[pq.y]);
    double c, s;
    const bool clamped = transform_params(app, aqq, apq, same, c, s);
    if (vlog && threadIdx.x == 0) vlog[blockIdx.x] = log_entry(c, s, same);
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int r = threadIdx.x + k * BS;
        if (r < m) {
            rotate_elems(xp[k], xq[k], c, s, same);
            gp[r] = xp[k];
            gq[r] = xq[k];
        }
    }
    if constexpr (PF) {
        if (V) {
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int r = threadIdx.x + k * BS;
                if (r < nv) {
                    rotate_elems(wp[k], wq[k], c, s, same);
                    vp[r] = wp[k];
                    vq[r] = wq[k];
                }
            }
        }
    } else {
        if (V) rotate_columns<BS>(vp, vq, nv, c, s, same);
    }
    if (threadIdx.x == 0) {
        // this slot is written by this workgroup only, and launches are
        // ordered on the stream: a plain update, no atomic
        slot_rot[blockIdx.x] += 1u;
        if (clamped) slot_clamp[blockIdx.x] += 1u;
    }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_pair_step_stream(double *__restrict__ G, int m, long ldg,
                                                         double *__restrict__ V, int nv, long ldv,
                                                         const int2 *__restrict__ pairs,
                                                         const signed char *__restrict__ J,
                                                         double tol, SweepCounters *__restrict__ ctr,
                                                         unsigned *__restrict__ slot_rot,
                                                         unsigned *__restrict__ slot_clamp,
                                                         double2 *__restrict__ vlog)
{
    __shared__ double sh[3 * BS / kWave];
    const int2 pq = pairs[blockIdx.x];
    double *gp = G + (size_t)pq.x * ldg;
    double *gq = G + (size_t)pq.y * ldg;
    double app = 0.0, aqq = 0.0, apq = 0.0;
    for (int r = threadIdx.x; r < m; r += BS) {
        const double a = gp[r], b = gq[r];
        app = fma(a, a, app);
        aqq = fma(b, b, aqq);
        apq = fma(a, b, apq);
    }
    block_sum3<BS>(app, aqq, apq, sh);
    if (!finite3(app, aqq, apq)) {
        if (threadIdx.x == 0) {
            ctr->nonfinite = 1u;
            if (vlog) vlog[blockIdx.x] = make_double2(1.0, 0.0);
        }
        return;
    }
    if (!needs_rotation(app, aqq, apq, tol)) {
        if (vlog && threadIdx.x == 0) vlog[blockIdx.x] = make_double2(1.0, 0.0);
        return;
    }
    const bool same = (J == nullptr) || (J[pq.x] == J[pq.y]);
    double c, s;
    const bool clamped = transform_params(app, aqq, apq, same, c, s);
    if (vlog && threadIdx.x == 0) vlog[blockIdx.x] = log_entry(c, s, same);
    rotate_columns<BS>(gp, gq, m, c, s, same);
    if (V) rotate_columns<BS>(V + (size_t)pq.x * ldv, V + (size_t)pq.y * ldv, nv, c, s, same);
    if (threadIdx.x == 0) {
        slot_rot[blockIdx.x] += 1u;
        if (clamped) slot_clamp[blockIdx.x] += 1u;
    }
}

// ------------------------------------------------------------ k_apply_vlog
// Rows RB b .. RB b + RB - 1 of V (all n columns, sv[col * (RB + 1) + r]:
// the padding spreads the columns that the lanes of a wavefront touch over
// the LDS banks, where a pitch of RB doubles left them on eight) go to LDS,
// with RB scratch values per thread and the run's step offsets (so that no
// scalar memory load sits on a step's path); the logged rotations of steps k0 .. k1 - 1 are applied to them in
// step order, so every element of V sees the same rotations in the same
// order (and the same arithmetic, rotate_elems) as an in-step update.  A
// thread takes pairs tid, tid + 256, ... of a step (PPT of them at most) and
// all RB rows of each, one barrier per step.  The log entries and pair
// indices of the next D steps are in flight in registers (a ring of D slots,
// refilled as each step is done; past k1 - 1 the last step is loaded again,
// so that no load is predicated): a step's LDS work is far shorter than the
// latency of the log's loads.
template <int RB, int PPT>
__global__ __launch_bounds__(256) void k_apply_vlog(double *__restrict__ V, int nv, int n, long ldv,
                                                    const int2 *__restrict__ pairs,
                                                    const int *__restrict__ step_start, int k0,
                                                    int k1, const double2 *__restrict__ vlog,
                                                    int stride)
{
    constexpr int D = PPT >= 16 ? 1 : 16 / PPT;
    // n columns of V rows, a scratch column per thread (pitch CP), the
    // offsets of steps k0 .. k1 into the pair table
    constexpr int CP = RB + 1;
    extern __shared__ double sv[];
    double *mine = sv + (size_t)(n + threadIdx.x) * CP;
    int *ss = (int *)(sv + (size_t)(n + 256) * CP);
    for (int k = k0 + (int)threadIdx.x; k <= k1; k += 256) ss[k - k0] = step_start[k];
    __syncthreads();
    const int row0 = blockIdx.x * RB;
    const int nr = min(RB, nv - row0);
    double2 cs[D][PPT];
    int2 pq[D][PPT];
    int np[D];
    auto fetch = [&](int k, double2 *c_out, int2 *p_out, int &np_out) {
        const int s0 = ss[k - k0];
        np_out = ss[k - k0 + 1] - s0;
        const double2 *lg = vlog + (size_t)(k - k0) * stride;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            // in bounds also for a step without pairs (entry 0 is read, unused)
            const int p = max(0, min((int)threadIdx.x + 256 * i, np_out - 1));
            c_out[i] = lg[p];
            p_out[i] = pairs[np_out > 0 ? s0 + p : 0];
        }
    };
#pragma unroll
    for (int j = 0; j < D; ++j) fetch(min(k0 + j, k1 - 1), cs[j], pq[j], np[j]);
    // V rows: eight loads in flight per thread (clamped indices), then LDS
    const int ne = n * RB;
    for (int e0 = 0; e0 < ne; e0 += 8 * 256) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = min(e0 + (int)threadIdx.x + 256 * u, ne - 1);
            t[u] = V[(size_t)(e / RB) * ldv + row0 + min(e % RB, nr - 1)];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + (int)threadIdx.x + 256 * u;
            if (e < ne) sv[(e / RB) * CP + e % RB] = (e % RB < nr) ? t[u] : 0.0;
        }
    }
    __syncthreads();
    for (int kb = k0; kb < k1; kb += D) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int k = kb + j;
            if (k >= k1) break;   // the same for the whole workgroup
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                // no branch: a lane without a rotation (past the step's pairs,
                // or the identity, s = 0) works on its own scratch rows, so
                // that the slot's loads are consumed on every path and the
                // compiler keeps the later slots in flight when it refills
                // this one
                const int p = (int)threadIdx.x + 256 * i;
                const bool act = p < np[j] && cs[j][i].y != 0.0;
                const bool same = cs[j][i].x > 0.0;
                const double c = fabs(cs[j][i].x), s = cs[j][i].y;
                double *a = act ? sv + pq[j][i].x * CP : mine;
                double *b = act ? sv + pq[j][i].y * CP : mine;
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    double x = a[r], y = b[r];
                    rotate_elems(x, y, c, s, same);
                    a[r] = x;
                    b[r] = y;
                }
            }
            __syncthreads();
            fetch(min(k + D, k1 - 1), cs[j], pq[j], np[j]);
        }
    }
    for (int e = threadIdx.x; e < n * RB; e += 256) {
        const int col = e / RB, r = e % RB;
        if (r < nr) V[(size_t)col * ldv + row0 + r] = sv[col * CP + r];
    }
}

// Sum the per-slot counts of a sweep into its counters and clear the slots.
__global__ __launch_bounds__(256) void k_sum_slots(unsigned *__restrict__ slot_rot,
                                                   unsigned *__restrict__ slot_clamp, int nslots,
                                                   SweepCounters *__restrict__ ctr)
{
    __shared__ unsigned long long sr[256], sc[256];
    unsigned long long r = 0, c = 0;
    for (int i = threadIdx.x; i < nslots; i += 256) {
        r += slot_rot[i];
        c += slot_clamp[i];
        slot_rot[i] = 0u;
        slot_clamp[i] = 0u;
    }
    sr[threadIdx.x] = r;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sr[threadIdx.x] += sr[threadIdx.x + h];
            sc[threadIdx.x] += sc[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ctr->rotations += sr[0];
        ctr->clamps += sc[0];
    }
}

// One pair of a step by one wavefront, lanes over the rows.  When the rows
// fit R per lane (m, n <= 64 R) they stay in registers from the dot products
// to the rotation and the V pair is loaded with the G pair; otherwise the
// rows are looped over (R = 0).
template <int R>
__device__ __forceinline__ void small_pair(double *g, long lg, double *v, long lv, int m, int n,
                                           int p, int q, const signed char *J, double tol,
                                           int lane, unsigned long long &rot,
                                           unsigned long long &ncl, int *nonfinite)
{
    double *gp = g + (size_t)p * lg, *gq = g + (size_t)q * lg;
    if constexpr (R > 0) {
        double a[R], b[R], va[R], vb[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = lane + kWave * i;
            a[i] = r < m ? gp[r] : 0.0;
            b[i] = r < m ? gq[r] : 0.0;
        }
        if (v) {
            const double *vp = v + (size_t)p * lv, *vq = v + (size_t)q * lv;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = lane + kWave * i;
                va[i] = r < n ? vp[r] : 0.0;
                vb[i] = r < n ? vq[r] : 0.0;
            }
        }
        double app = 0.0, aqq = 0.0, apq = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            app = fma(a[i], a[i], app);
            aqq = fma(b[i], b[i], aqq);
            apq = fma(a[i], b[i], apq);
        }
        app = wave_sum(app);
        aqq = wave_sum(aqq);
        apq = wave_sum(apq);
        if (!finite3(app, aqq, apq)) {
            *nonfinite = 1;
            return;
        }
        if (!needs_rotation(app, aqq, apq, tol)) return;
        const bool same = (J == nullptr) || (J[p] == J[q]);
        double c, s;
        ncl += transform_params(app, aqq, apq, same, c, s) ? 1 : 0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = lane + kWave * i;
            rotate_elems(a[i], b[i], c, s, same);
            if (r < m) {
                gp[r] = a[i];
                gq[r] = b[i];
            }
        }
        if (v) {
            double *vp = v + (size_t)p * lv, *vq = v + (size_t)q * lv;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = lane + kWave * i;
                rotate_elems(va[i], vb[i], c, s, same);
                if (r < n) {
                    vp[r] = va[i];
                    vq[r] = vb[i];
                }
            }
        }
        ++rot;
    } else {
        double app = 0.0, aqq = 0.0, apq = 0.0;
        for (int r = lane; r < m; r += kWave) {
            const double a = gp[r], b = gq[r];
            app = fma(a, a, app);
            aqq = fma(b, b, aqq);
            apq = fma(a, b, apq);
        }
        app = wave_sum(app);
        aqq = wave_sum(aqq);
        apq = wave_sum(apq);
        if (!finite3(app, aqq, apq)) {
            *nonfinite = 1;
            return;
        }
        if (!needs_rotation(app, aqq, apq, tol)) return;
        const bool same = (J == nullptr) || (J[p] == J[q]);
        double c, s;
        ncl += transform_params(app, aqq, apq, same, c, s) ? 1 : 0;
        for (int r = lane; r < m; r += kWave) {
            double a = gp[r], b = gq[r];
            rotate_elems(a, b, c, s, same);
            gp[r] = a;
            gq[r] = b;
        }
        if (v) {
            double *vp = v + (size_t)p * lv, *vq = v + (size_t)q * lv;
            for (int r = lane; r < n; r += kWave) {
                double a = vp[r], b = vq[r];
                rotate_elems(a, b, c, s, same);
                vp[r] = a;
                vq[r] = b;
            }
        }
        ++rot;
    }
}

// All sweeps on (g, v).  The caller passes pointers of one kind (LDS or
// global) for g and for v, so that the accesses compile to LDS or global
// instructions rather than generic ones.
template <int NW, int R>
__device__ __forceinline__ int small_sweeps(double *g, long lg, double *v, long lv, int m, int n,
                                            const signed char *J, double tol, const int2 *pairs,
                                            const int *step_start, int nsteps, int max_sweeps,
                                            SweepCounters *ctr, unsigned long long *red,
                                            int *nonfinite)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    int sweep = 0;
    while (sweep < max_sweeps) {
        unsigned long long rot = 0, ncl = 0;
        for (int st = 0; st < nsteps; ++st) {
            const int e0 = step_start[st], e1 = step_start[st + 1];
            for (int e = e0 + wave; e < e1; e += NW) {
                const int2 pq = pairs[e];
                small_pair<R>(g, lg, v, lv, m, n, pq.x, pq.y, J, tol, lane, rot, ncl, nonfinite);
            }
            if constexpr (NW > 1) __syncthreads();
        }
        if (lane == 0) {
            red[wave] = rot;
            red[NW + wave] = ncl;
        }
        __syncthreads();
        unsigned long long tot = 0, totc = 0;
        for (int i = 0; i < NW; ++i) {
            tot += red[i];
            totc += red[NW + i];
        }
        const int nf = *nonfinite;
        if (threadIdx.x == 0) {
            ctr[sweep].rotations = tot;
            ctr[sweep].clamps = totc;
            ctr[sweep].nonfinite = nf;
        }
        ++sweep;
        __syncthreads();
        if (tot == 0 || nf) break;
    }
    return sweep;
}

// Whole solve in one workgroup of NW wavefronts.  The pairs of each step
// are dealt round-robin to the wavefronts; lanes of a wavefront run over the
// rows.  If `lds_g` the m x n factor lives in LDS (leading dimension m), and
// if `lds_v` also V (leading dimension n); otherwise they are used in place
// in global memory.  Writes the per-sweep counters and the sweep count.
template <int NW>
__global__ __launch_bounds__(NW *kWave) void k_small_solve(
    double *__restrict__ G, int m, int n, long ldg, double *__restrict__ V, long ldv,
    const signed char *__restrict__ J, double tol, const int2 *__restrict__ pairs,
    const int *__restrict__ step_start, int nsteps, int max_sweeps, int lds_g, int lds_v,
    SweepCounters *__restrict__ ctr, int *__restrict__ sweeps_out)
{
    extern __shared__ double lds[];
    __shared__ unsigned long long red[2 * NW];
    __shared__ int nonfinite;
    constexpr int BS = NW * kWave;

    if (lds_g)
        for (int c = 0; c < n; ++c)
            for (int r = threadIdx.x; r < m; r += BS) lds[r + (size_t)c * m] = G[r + (size_t)c * ldg];
    if (V && lds_v)
        for (int c = 0; c < n; ++c)
            for (int r = threadIdx.x; r < n; r += BS)
                lds[(size_t)m * n + r + (size_t)c * n] = V[r + (size_t)c * ldv];
    if (threadIdx.x == 0) nonfinite = 0;
    __syncthreads();

    const bool regs = m <= 2 * kWave && n <= 2 * kWave;
    int sweep;
    if (lds_g && V && lds_v) {
        sweep = regs ? small_sweeps<NW, 2>(lds, m, lds + (size_t)m * n, n, m, n, J, tol, pairs,
                                           step_start, nsteps, max_sweeps, ctr, red, &nonfinite)
                     : small_sweeps<NW, 0>(lds, m, lds + (size_t)m * n, n, m, n, J, tol, pairs,
                                           step_start, nsteps, max_sweeps, ctr, red, &nonfinite);
    } else if (lds_g) {
        sweep = regs ? small_sweeps<NW, 2>(lds, m, V, ldv, m, n, J, tol, pairs, step_start, nsteps,
                                           max_sweeps, ctr, red, &nonfinite)
                     : small_sweeps<NW, 0>(lds, m, V, ldv, m, n, J, tol, pairs, step_start, nsteps,
                                           max_sweeps, ctr, red, &nonfinite);
    } else {
        sweep = small_sweeps<NW, 0>(G, ldg, V, ldv, m, n, J, tol, pairs, step_start, nsteps,
                                    max_sweeps, ctr, red, &nonfinite);
    }
    if (lds_g)
        for (int c = 0; c < n; ++c)
            for (int r = threadIdx.x; r < m; r += BS) G[r + (size_t)c * ldg] = lds[r + (size_t)c * m];
    if (V && lds_v)
        for (int c = 0; c < n; ++c)
            for (int r = threadIdx.x; r < n; r += BS)
                V[r + (size_t)c * ldv] = lds[(size_t)m * n + r + (size_t)c * n];
    if (threadIdx.x == 0) *sweeps_out = sweep;
}

// All sweeps of the row-cyclic ordering for m, n <= 64 in one workgroup.
// The ordering runs as its 2n - 3 steps of equal p + q (rowcyclic_steps in
// ordering.h: the result of one pair at a time in row order), the pairs of a
// step side by side: each 16-lane row of a wavefront takes one pair, lane l
// of the row holding rows l, l + 16, l + 32, l + 48 of its two columns of G
// (and of V), so the Gram sums end in every lane of the row after four DPP
// stages and a wavefront computes the transforms of four pairs at once.
// G and V sit in LDS column-major (pitch 64, rows past m or n zero); NW
// wavefronts cover the n / 2 pairs of the widest step.
constexpr int kRowCyclicMax = 64;
constexpr int kRcRows = 4;   // rows per lane

// A DPP move of a double for patterns that have a source lane in every lane
// (quad permutations, row mirrors): no old value is needed.
template <int CTRL>
__device__ __forceinline__ double dpp_all(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sums over the 16 lanes of each DPP row, three values with the stages
// interleaved; every lane of the row ends with the row's totals (lane ^ 1,
// lane ^ 2, then the mirrors within 8 and 16 lanes, each pairing a lane with
// one of the other half).
__device__ __forceinline__ void row_sum3(double &x, double &y, double &z)
{
    x += dpp_all<0xB1>(x);
    y += dpp_all<0xB1>(y);
    z += dpp_all<0xB1>(z);
    x += dpp_all<0x4E>(x);
    y += dpp_all<0x4E>(y);
    z += dpp_all<0x4E>(z);
    x += dpp_all<0x141>(x);
    y += dpp_all<0x141>(y);
    z += dpp_all<0x141>(z);
    x += dpp_all<0x140>(x);
    y += dpp_all<0x140>(y);
    z += dpp_all<0x140>(z);
}

template <int NW>
__global__ __launch_bounds__(NW *kWave) void k_rowcyclic_solve(
    double *__restrict__ G, int m, int n, long ldg, double *__restrict__ V, long ldv,
    const signed char *__restrict__ J, double tol, int max_sweeps,
    SweepCounters *__restrict__ ctr, int *__restrict__ sweeps_out)
{
    constexpr int P = kRowCyclicMax, BS = NW * kWave;
    __shared__ double g[P * P], v[P * P];
    __shared__ signed char js[P];
    __shared__ unsigned long long red[3 * NW];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int grp = lane >> 4, l16 = lane & 15;
    for (int e = tid; e < P * n; e += BS) {
        const int c = e / P, r = e % P;
        g[e] = r < m ? G[(size_t)c * ldg + r] : 0.0;
        if (V) v[e] = r < n ? V[(size_t)c * ldv + r] : 0.0;
    }
    if (tid < n) js[tid] = J ? J[tid] : (signed char)1;
    __syncthreads();
    int sweep = 0;
    while (sweep < max_sweeps) {
        unsigned long long rot = 0, ncl = 0, nonfinite = 0;   // counted by lane 0 of a row
        for (int t = 1; t <= rowcyclic_steps(n); ++t) {
            const int p0 = rowcyclic_first(n, t), np = rowcyclic_step_pairs(n, t);
            if (4 * wave < np) {
                const int e = 4 * wave + grp;
                const bool active = e < np;
                const int p = active ? p0 + e : p0, q = t - p;   // a valid pair when idle
                double x[kRcRows], y[kRcRows];
#pragma unroll
                for (int i = 0; i < kRcRows; ++i) {
                    x[i] = g[p * P + 16 * i + l16];
                    y[i] = g[q * P + 16 * i + l16];
                }
                double app = 0.0, aqq = 0.0, apq = 0.0;
#pragma unroll
                for (int i = 0; i < kRcRows; ++i) {
                    app = fma(x[i], x[i], app);
                    aqq = fma(y[i], y[i], aqq);
                    apq = fma(x[i], y[i], apq);
                }
                row_sum3(app, aqq, apq);
                const bool fin = finite3(app, aqq, apq);
                if (active && !fin && l16 == 0) nonfinite = 1;
                if (active && fin && needs_rotation(app, aqq, apq, tol)) {
                    // pairs of both signs may share the wavefront
                    const bool same = js[p] == js[q];
                    double c, sn;
                    const bool clamped = transform_params_bf(app, aqq, apq, same, c, sn);
#pragma unroll
                    for (int i = 0; i < kRcRows; ++i) {
                        rotate_elems(x[i], y[i], c, sn, same);
                        g[p * P + 16 * i + l16] = x[i];
                        g[q * P + 16 * i + l16] = y[i];
                    }
                    if (V) {
                        // V is read only for a pair that rotates
#pragma unroll
                        for (int i = 0; i < kRcRows; ++i) {
                            double vx = v[p * P + 16 * i + l16], vy = v[q * P + 16 * i + l16];
                            rotate_elems(vx, vy, c, sn, same);
                            v[p * P + 16 * i + l16] = vx;
                            v[q * P + 16 * i + l16] = vy;
                        }
                    }
                    if (l16 == 0) {
                        ++rot;
                        ncl += clamped ? 1 : 0;
                    }
                }
            }
            if constexpr (NW > 1) __syncthreads();
        }
        // totals over the rows of the wavefront, then over the wavefronts
        const unsigned long long wr = __shfl(rot, 0) + __shfl(rot, 16) + __shfl(rot, 32) + __shfl(rot, 48);
        const unsigned long long wc = __shfl(ncl, 0) + __shfl(ncl, 16) + __shfl(ncl, 32) + __shfl(ncl, 48);
        const unsigned long long wn = __shfl(nonfinite, 0) | __shfl(nonfinite, 16) |
                                      __shfl(nonfinite, 32) | __shfl(nonfinite, 48);
        if (lane == 0) {
            red[wave] = wr;
            red[NW + wave] = wc;
            red[2 * NW + wave] = wn;
        }
        __syncthreads();
        unsigned long long tr = 0, tc = 0, tn = 0;
        for (int w = 0; w < NW; ++w) {
            tr += red[w];
            tc += red[NW + w];
            tn |= red[2 * NW + w];
        }
        if (tid == 0) {
            ctr[sweep].rotations = tr;
            ctr[sweep].clamps = tc;
            ctr[sweep].nonfinite = (int)tn;
        }
        ++sweep;
        __syncthreads();   // red is rewritten by the next sweep
        if (tr == 0 || tn) break;
    }
    for (int e = tid; e < P * n; e += BS) {
        const int c = e / P, r = e % P;
        if (r < m) G[(size_t)c * ldg + r] = g[e];
        if (V && r < n) V[(size_t)c * ldv + r] = v[e];
    }
    if (tid == 0) *sweeps_out = sweep;
}

__global__ void k_identity(double *__restrict__ V, int n, long ldv)
{
    const int c = blockIdx.x;
    for (int r = threadIdx.x; r < n; r += blockDim.x) V[r + (size_t)c * ldv] = (r == c) ? 1.0 : 0.0;
}

template <int BS>
__global__ __launch_bounds__(BS) void k_finalize(const double *__restrict__ G, int m, long ldg,
                                                 const signed char *__restrict__ J,
                                                 double *__restrict__ lambda, double *U, long ldu)
{
    __shared__ double sh[3 * BS / kWave];
    const int c = blockIdx.x;
    const double *gc = G + (size_t)c * ldg;
    double s = 0.0, d1 = 0.0, d2 = 0.0;
    for (int r = threadIdx.x; r < m; r += BS) s = fma(gc[r], gc[r], s);
    block_sum3<BS>(s, d1, d2, sh);
    if (lambda && threadIdx.x == 0) lambda[c] = (J && J[c] < 0) ? -s : s;
    if (U) {
        const double nrm = sqrt(s);
        double *uc = U + (size_t)c * ldu;
        // U may alias G: every element is read before it is written by the same thread
        for (int r = threadIdx.x; r < m; r += BS) uc[r] = (s > 0.0) ? gc[r] / nrm : 0.0;
    }
}

// S consecutive steps of the modified modulus ordering on even n (the ring
// of Alg. 3.1) in one launch, for m <= 1024.  In the ring, process r takes
// the column it receives at step k + 1 from process r + 1 (mod p) and keeps
// the other.  Workgroup w owns process w and also runs processes w + 1 ..
// w + S - 1 (their owners run them too, with the same arithmetic): at step
// j of the launch group g (process w + g, 256 threads) is active while
// g <= S - 1 - j, and hands the column it gives up to group g - 1 through
// LDS.  Every group runs its pair as k_pair_step<256, 4> does (the same
// loads, sums, block reduction, test, transform and rotation), so the
// results are bit for bit those of one launch per step; the owner's group
// alone writes the rotation log, the slot counters and, after the last
// step, its two columns.  G is read from Gin and written to Gout (a second
// buffer), since the other workgroups still read Gin.  pairs: the table of
// step k (p pairs per step, by slot; slot b runs process slot_process(b)).
constexpr int kRingGroupThreads = 256, kRingRows = 4;

__device__ __forceinline__ int ring_slot_of(int r, int p)
{
    // the inverse of slot_process in ordering.cpp
    if (p % 8) return r;
    const int per = p / 8;
    return (r % per) * 8 + r / per;
}

template <int S>
__global__ __launch_bounds__(S *kRingGroupThreads) void k_pair_steps_ring(
    const double *__restrict__ Gin, double *__restrict__ Gout, int m, long ldg,
    const int2 *__restrict__ pairs, int p, const signed char *__restrict__ J, double tol,
    SweepCounters *__restrict__ ctr, unsigned *__restrict__ slot_rot,
    unsigned *__restrict__ slot_clamp, double2 *__restrict__ vlog, int vlog_stride)
{
    constexpr int BS = kRingGroupThreads, CH = kRingRows, NWG = BS / kWave;
    __shared__ double sh[S][3 * NWG];
    __shared__ double box[S][BS * CH];   // the column group g gives up, rows in order
    __shared__ signed char js[BS * CH];  // J (n <= m <= 1024)
    const int g = threadIdx.x / BS, t = threadIdx.x % BS, wv = t / kWave;
    // workgroup b runs the process of slot b (the XCD that ran it in the
    // one-step launches, whose L2 holds the columns it hands on)
    const int owner = (p % 8) ? (int)blockIdx.x : (int)(blockIdx.x % 8) * (p / 8) + (int)blockIdx.x / 8;
    const int proc = (owner + g) % p;
    const int slot = ring_slot_of(proc, p);
    // this process's pairs of the launch's steps, and J, read once
    int2 pqs[S];
#pragma unroll
    for (int j = 0; j < S; ++j) pqs[j] = pairs[(size_t)j * p + slot];
    if (J)
        for (int e = threadIdx.x; e < 2 * p; e += S * BS) js[e] = J[e];
    int ck = pqs[0].x, cn = pqs[0].y;   // K: kept from step to step, N: received
    double K[CH], N[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int r = t + k * BS;
        K[k] = (r < m) ? Gin[(size_t)ck * ldg + r] : 0.0;
        N[k] = (r < m) ? Gin[(size_t)cn * ldg + r] : 0.0;
    }
    __syncthreads();   // js
    for (int j = 0; j < S; ++j) {
        const bool act = g <= S - 1 - j;
        const bool kx = ck < cn;   // K holds the pair's first column
        double app = 0.0, aqq = 0.0, apq = 0.0;
        if (act) {
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const double xp = kx ? K[k] : N[k], xq = kx ? N[k] : K[k];
                app = fma(xp, xp, app);
                aqq = fma(xq, xq, aqq);
                apq = fma(xp, xq, apq);
            }
        }
        // block_sum3<256> within the group
        app = wave_sum(app);
        aqq = wave_sum(aqq);
        apq = wave_sum(apq);
        if ((t & (kWave - 1)) == 0) {
            sh[g][wv] = app;
            sh[g][NWG + wv] = aqq;
            sh[g][2 * NWG + wv] = apq;
        }
        __syncthreads();
        if (act) {
            app = sh[g][0];
            aqq = sh[g][NWG];
            apq = sh[g][2 * NWG];
#pragma unroll
            for (int i = 1; i < NWG; ++i) {
                app += sh[g][i];
                aqq += sh[g][NWG + i];
                apq += sh[g][2 * NWG + i];
            }
            const int pp = kx ? ck : cn, qq = kx ? cn : ck;
            double2 entry = make_double2(1.0, 0.0);
            if (!finite3(app, aqq, apq)) {
                if (g == 0 && t == 0) ctr->nonfinite = 1u;
            } else if (needs_rotation(app, aqq, apq, tol)) {
                const bool same = (J == nullptr) || (js[pp] == js[qq]);
                double c, sn;
                const bool clamped = transform_params(app, aqq, apq, same, c, sn);
                entry = log_entry(c, sn, same);
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    double xp = kx ? K[k] : N[k], xq = kx ? N[k] : K[k];
                    rotate_elems(xp, xq, c, sn, same);
                    K[k] = kx ? xp : xq;
                    N[k] = kx ? xq : xp;
                }
                if (g == 0 && t == 0) {
                    slot_rot[slot] += 1u;
                    if (clamped) slot_clamp[slot] += 1u;
                }
            }
            if (g == 0 && t == 0 && vlog) vlog[(size_t)j * vlog_stride + slot] = entry;
        }
        if (j + 1 == S) break;
        // the next pair of this process: keep the shared column in K, give up
        // the other (into the box, for group g - 1), receive from group g + 1
        int cnext = -1;
        if (act) {
            int2 nx = pqs[0];
#pragma unroll
            for (int i = 1; i < S; ++i)
                if (i == j + 1) nx = pqs[i];
            if (ck != nx.x && ck != nx.y) {
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const double x = K[k];
                    K[k] = N[k];
                    N[k] = x;
                }
                const int x = ck;
                ck = cn;
                cn = x;
            }
            if (g > 0)
#pragma unroll
                for (int k = 0; k < CH; ++k) box[g][t + k * BS] = N[k];
            cnext = (nx.x == ck) ? nx.y : nx.x;
        }
        __syncthreads();
        if (g <= S - 2 - j) {
            // group g + 1 gave up exactly this column (the ring hands it on)
#pragma unroll
            for (int k = 0; k < CH; ++k) N[k] = box[g + 1][t + k * BS];
            cn = cnext;
        }
        __syncthreads();   // the boxes are rewritten after the next step
    }
    if (g == 0) {
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int r = t + k * BS;
            if (r < m) {
                Gout[(size_t)ck * ldg + r] = K[k];
                Gout[(size_t)cn * ldg + r] = N[k];
            }
        }
    }
}

hipError_t launch_pair_steps_ring(const RingStepsArgs &a, hipStream_t st)
{
    if (a.m > kRingGroupThreads * kRingRows || a.p < 1) return hipErrorInvalidValue;
    switch (a.steps) {
    case 2:
        k_pair_steps_ring<2><<<a.p, 2 * kRingGroupThreads, 0, st>>>(
            a.Gin, a.Gout, a.m, a.ldg, a.pairs, a.p, a.J, a.tol, a.ctr, a.slot_rot, a.slot_clamp,
            a.vlog, a.vlog_stride);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- launchers
template <int BS, int CH>
static void launch_ch(const PairStepArgs &a, hipStream_t st)
{
    dim3 grid(a.npairs), block(BS);
    double *V = a.vlog ? nullptr : a.V;   // with a log, V is updated later
    if (a.prefetch_v && V && a.nv <= BS * CH)
        k_pair_step<BS, CH, true><<<grid, block, 0, st>>>(a.G, a.m, a.ldg, V, a.nv, a.ldv, a.pairs,
                                                          a.J, a.tol, a.ctr, a.slot_rot, a.slot_clamp,
                                                          a.vlog);
    else
        k_pair_step<BS, CH, false><<<grid, block, 0, st>>>(a.G, a.m, a.ldg, V, a.nv, a.ldv, a.pairs,
                                                           a.J, a.tol, a.ctr, a.slot_rot, a.slot_clamp,
                                                           a.vlog);
}

template <int BS>
static hipError_t launch_pair_step_bs(const PairStepArgs &a, hipStream_t st)
{
    const int ch = (a.m + BS - 1) / BS;
    if (ch <= 1)
        launch_ch<BS, 1>(a, st);
    else if (ch <= 2)
        launch_ch<BS, 2>(a, st);
    else if (ch <= 4)
        launch_ch<BS, 4>(a, st);
    else if (ch <= 8)
        launch_ch<BS, 8>(a, st);
    else if (ch <= 16)
        launch_ch<BS, 16>(a, st);
    else
        k_pair_step_stream<BS><<<dim3(a.npairs), dim3(BS), 0, st>>>(
            a.G, a.m, a.ldg, a.vlog ? nullptr : a.V, a.nv, a.ldv, a.pairs, a.J, a.tol, a.ctr,
            a.slot_rot, a.slot_clamp, a.vlog);
    return hipGetLastError();
}

hipError_t launch_pair_step(const PairStepArgs &a, hipStream_t st)
{
    if (a.npairs <= 0) return hipSuccess;
    if (a.m > 512) return launch_pair_step_bs<256>(a, st);
    if (a.m > 128) return launch_pair_step_bs<128>(a, st);
    return launch_pair_step_bs<64>(a, st);
}

size_t small_solve_lds_bytes(int m, int n, bool want_v, int *lds_g, int *lds_v)
{
    const size_t g = (size_t)m * n * sizeof(double);
    const size_t v = want_v ? (size_t)n * n * sizeof(double) : 0;
    *lds_g = *lds_v = 0;
    if (g + v <= kSmallSolveLdsBytes) {
        *lds_g = 1;
        *lds_v = want_v ? 1 : 0;
        return g + v;
    }
    if (g <= kSmallSolveLdsBytes) {
        *lds_g = 1;
        return g;
    }
    return 0;
}

hipError_t set_lds_limit(const void *func, int bytes)
{
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, int> set;   // (kernel, device) -> bytes
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = set.find({func, dev});
    if (it != set.end() && it->second >= bytes) return hipSuccess;
    if ((e = hipFuncSetAttribute(func, hipFuncAttributeMaxDynamicSharedMemorySize, bytes)) != hipSuccess)
        return e;
    set[{func, dev}] = bytes;
    return hipSuccess;
}

template <int NW>
static hipError_t launch_small_nw(const SmallSolveArgs &a, hipStream_t st)
{
    int lg = 0, lv = 0;
    const size_t bytes = small_solve_lds_bytes(a.m, a.n, a.V != nullptr, &lg, &lv);
    if (bytes > 65536) {
        hipError_t e = set_lds_limit((const void *)k_small_solve<NW>, (int)bytes);
        if (e != hipSuccess) return e;
    }
    k_small_solve<NW><<<1, NW * kWave, bytes, st>>>(a.G, a.m, a.n, a.ldg, a.V, a.ldv, a.J, a.tol,
                                                    a.pairs, a.step_start, a.nsteps, a.max_sweeps,
                                                    lg, lv, a.ctr, a.sweeps_out);
    return hipGetLastError();
}

hipError_t launch_small_solve(const SmallSolveArgs &a, hipStream_t st)
{
    if (a.row_cyclic && a.m <= kRowCyclicMax && a.n <= kRowCyclicMax) {
        // four pairs per wavefront, n / 2 pairs in the widest step
        const int waves = (a.n / 2 + 3) / 4;
        if (waves <= 1)
            k_rowcyclic_solve<1><<<1, kWave, 0, st>>>(a.G, a.m, a.n, a.ldg, a.V, a.ldv, a.J, a.tol,
                                                      a.max_sweeps, a.ctr, a.sweeps_out);
        else if (waves <= 2)
            k_rowcyclic_solve<2><<<1, 2 * kWave, 0, st>>>(a.G, a.m, a.n, a.ldg, a.V, a.ldv, a.J,
                                                          a.tol, a.max_sweeps, a.ctr, a.sweeps_out);
        else if (waves <= 4)
            k_rowcyclic_solve<4><<<1, 4 * kWave, 0, st>>>(a.G, a.m, a.n, a.ldg, a.V, a.ldv, a.J,
                                                          a.tol, a.max_sweeps, a.ctr, a.sweeps_out);
        else
            k_rowcyclic_solve<8><<<1, 8 * kWave, 0, st>>>(a.G, a.m, a.n, a.ldg, a.V, a.ldv, a.J,
                                                          a.tol, a.max_sweeps, a.ctr, a.sweeps_out);
        return hipGetLastError();
    }
    // one wavefront for strictly sequential orderings; otherwise up to 16
    if (a.max_pairs_per_step <= 1) return launch_small_nw<1>(a, st);
    if (a.max_pairs_per_step <= 4) return launch_small_nw<4>(a, st);
    if (a.max_pairs_per_step <= 8) return launch_small_nw<8>(a, st);
    return launch_small_nw<16>(a, st);
}

int vlog_rows(int n)
{
    if ((size_t)5 * (n + 256) * sizeof(double) <= kVlogLdsBytes) return 4;
    if ((size_t)3 * (n + 256) * sizeof(double) <= kVlogLdsBytes) return 2;
    return 0;
}

template <int RB, int PPT>
static hipError_t launch_apply_rb(const VlogApplyArgs &a, hipStream_t st)
{
    const size_t bytes = (size_t)(RB + 1) * (a.n + 256) * sizeof(double) +
                         (size_t)(a.k1 - a.k0 + 1) * sizeof(int);
    if (bytes > 160 * 1024) return hipErrorInvalidValue;
    if (bytes > 65536) {
        hipError_t e = set_lds_limit((const void *)k_apply_vlog<RB, PPT>, (int)bytes);
        if (e != hipSuccess) return e;
    }
    const int grid = (a.nv + RB - 1) / RB;
    k_apply_vlog<RB, PPT><<<grid, 256, bytes, st>>>(a.V, a.nv, a.n, a.ldv, a.pairs, a.step_start,
                                                    a.k0, a.k1, a.vlog, a.stride);
    return hipGetLastError();
}

template <int RB>
static hipError_t launch_apply_ppt(const VlogApplyArgs &a, hipStream_t st)
{
    const int ppt = (a.max_pairs + 255) / 256;
    if (ppt <= 1) return launch_apply_rb<RB, 1>(a, st);
    if (ppt <= 2) return launch_apply_rb<RB, 2>(a, st);
    if (ppt <= 4) return launch_apply_rb<RB, 4>(a, st);
    if (ppt <= 8) return launch_apply_rb<RB, 8>(a, st);
    return launch_apply_rb<RB, 16>(a, st);
}

hipError_t launch_apply_vlog(const VlogApplyArgs &a, hipStream_t st)
{
    if (a.k1 <= a.k0 || a.nv <= 0) return hipSuccess;
    if (a.max_pairs > 16 * 256) return hipErrorInvalidValue;
    const int rb = vlog_rows(a.n);
    if (rb == 4) return launch_apply_ppt<4>(a, st);
    if (rb == 2) return launch_apply_ppt<2>(a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_sum_slots(unsigned *slot_rot, unsigned *slot_clamp, int nslots,
                            SweepCounters *ctr, hipStream_t st)
{
    k_sum_slots<<<1, 256, 0, st>>>(slot_rot, slot_clamp, nslots, ctr);
    return hipGetLastError();
}

hipError_t launch_identity(double *V, int n, long ldv, hipStream_t st)
{
    k_identity<<<n, 256, 0, st>>>(V, n, ldv);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *G, int m, int n, long ldg, const signed char *J,
                           double *lambda, double *U, long ldu, hipStream_t st)
{
    if (m > 512)
        k_finalize<256><<<n, 256, 0, st>>>(G, m, ldg, J, lambda, U, ldu);
    else
        k_finalize<64><<<n, 64, 0, st>>>(G, m, ldg, J, lambda, U, ldu);
    return hipGetLastError();
}

}  // namespace jevd
