// Block one-sided Jacobi (Sec. 2.2-2.3; Alg. 3.4 with unpivoted Cholesky):
// block-oriented (BO) and full block (FB), trigonometric or hyperbolic.
//
// The n columns form N = n / b block columns of width b; block pairs (I, J)
// follow the modified modulus ordering over the N blocks (ring order, as in
// the pointwise path).  One outer step runs three kernels over its N/2
// pivots G_P = [G_I G_J] (m x W, W = 2b):
//   k_gram        A_P = G_P^T G_P on FP64 MFMA (v_mfma_f64_16x16x4f64), the
//                 rows split over several workgroups (split-K); only the
//                 upper 16 x 16 tiles are formed; partial sums go to a
//                 workspace and are added in split order by k_pivot_solve.
//   k_pivot_solve one workgroup per pivot: skip test, Cholesky A_P = R^T R,
//                 inner one-sided sweeps on the columns of R (trig or
//                 hyperbolic by J_P), accumulating V_P; writes V_P
//                 row-major.  After a Cholesky breakdown the inner sweeps run
//                 on the columns of G_P (and V) in place instead.
//   k_update      [G_I G_J] <- [G_I G_J] V_P and [V_I V_J] <- [V_I V_J] V_P
//                 on FP64 MFMA, in place, 64 rows per workgroup: each
//                 wavefront computes (G_P V_P)^T for 16 rows, so that both the
//                 loads of G_P and the stores of the result are 16
//                 consecutive rows per column.
#include <vector>

#include "../../include/jevd.h"
#include "block.h"
#include "device_math.h"
#include "ordering.h"

namespace jevd {

typedef double d4 __attribute__((ext_vector_type(4)));

// D += A B for a 16 x 4 A and a 4 x 16 B: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; element r of the result in lane l is
// D[l / 16 + 4 r][l % 16].
__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Global column of pivot-local column k of the block pair (I, J).
__device__ __forceinline__ int pivot_col(int k, int2 IJ, int b)
{
    return k < b ? IJ.x * b + k : IJ.y * b + (k - b);
}

// ------------------------------------------------------------------ k_gram
template <int W>
__global__ __launch_bounds__(256) void k_gram(const double *__restrict__ G, int m, long ldg, int b,
                                              const int2 *__restrict__ piv, int rows_per_split,
                                              double *__restrict__ partial)
{
    constexpr int KR = 32;                    // rows staged per iteration
    constexpr int LDC = W + 1;                // padded LDS row (doubles)
    constexpr int NT = W / 16;
    constexpr int NUP = NT * (NT + 1) / 2;    // upper tiles, diagonal included
    constexpr int TPW = (NUP + 3) / 4;        // tiles per wavefront
    __shared__ double st[KR * LDC];           // st[kr][c] = G_P[r0 + kr][c]
    const int pv = blockIdx.x, split = blockIdx.y;
    const int2 IJ = piv[pv];
    const int r_begin = split * rows_per_split;
    const int r_end = min(m, r_begin + rows_per_split);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    int ti[TPW], tj[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        int t = wave + 4 * q, it = 0;
        ti[q] = tj[q] = -1;
        if (t < NUP) {
            while (t >= NT - it) {               // row it of the upper triangle has NT - it tiles
                t -= NT - it;
                ++it;
            }
            ti[q] = it;
            tj[q] = it + t;
        }
    }
    d4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};

    for (int r0 = r_begin; r0 < r_end; r0 += KR) {
        for (int e = threadIdx.x; e < KR * W; e += 256) {
            const int kr = e % KR, c = e / KR;
            const int r = r0 + kr;
            st[kr * LDC + c] = (r < r_end) ? G[(size_t)pivot_col(c, IJ, b) * ldg + r] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KR; k += 4) {
            const double *row = st + (k + lane / 16) * LDC + (lane % 16);
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                if (ti[q] >= 0) {
                    const double a = row[ti[q] * 16];
                    const double bb = row[tj[q] * 16];
                    acc[q] = mfma16x16x4(a, bb, acc[q]);
                }
            }
        }
        __syncthreads();
    }
    double *out = partial + ((size_t)pv * gridDim.y + split) * W * W;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        if (ti[q] < 0) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = ti[q] * 16 + lane / 16 + 4 * r, col = tj[q] * 16 + lane % 16;
            out[(size_t)col * W + row] = acc[q][r];
        }
    }
}

// ---------------------------------------------------------- k_pivot_solve
// Inner sweeps on the columns of X (len rows, column c at X + c * ldx) with
// one wavefront per pair; the transform is also applied to the columns of Y
// (ylen rows, ld ldy) when Y is not null.  Returns this thread's count of
// rotations (counted by lane 0 of each wavefront only).
struct InnerTables {
    const int2 *pairs;
    const int *start;
    int nsteps;
};

template <int NW>
__device__ void inner_sweep(double *X, long ldx, int len, double *Y, long ldy, int ylen,
                            const signed char *JP, const InnerTables &tab, double tol,
                            unsigned long long &rot, unsigned long long &ncl, int *bad)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int s = 0; s < tab.nsteps; ++s) {
        for (int e = tab.start[s] + wave; e < tab.start[s + 1]; e += NW) {
            const int2 pq = tab.pairs[e];
            double *xp = X + (size_t)pq.x * ldx, *xq = X + (size_t)pq.y * ldx;
            double app = 0.0, aqq = 0.0, apq = 0.0;
            for (int r = lane; r < len; r += 64) {
                const double a = xp[r], c = xq[r];
                app = fma(a, a, app);
                aqq = fma(c, c, aqq);
                apq = fma(a, c, apq);
            }
            app = wave_sum(app);
            aqq = wave_sum(aqq);
            apq = wave_sum(apq);
            if (!finite3(app, aqq, apq)) {
                *bad = 1;
                continue;
            }
            if (!needs_rotation(app, aqq, apq, tol)) continue;
            const bool same = JP[pq.x] == JP[pq.y];
            double c, sn;
            if (transform_params(app, aqq, apq, same, c, sn) && lane == 0) ++ncl;
            for (int r = lane; r < len; r += 64) {
                double a = xp[r], d = xq[r];
                rotate_elems(a, d, c, sn, same);
                xp[r] = a;
                xq[r] = d;
            }
            if (Y) {
                double *yp = Y + (size_t)pq.x * ldy, *yq = Y + (size_t)pq.y * ldy;
                for (int r = lane; r < ylen; r += 64) {
                    double a = yp[r], d = yq[r];
                    rotate_elems(a, d, c, sn, same);
                    yp[r] = a;
                    yq[r] = d;
                }
            }
            if (lane == 0) ++rot;
        }
        __syncthreads();
    }
}

struct PivotSolveArgs {
    const double *partial;
    int nsplit;
    const signed char *J;
    const int2 *piv;
    int b;
    double tol;
    int all_pairs, full_block, max_inner;
    InnerTables full, cross;
    double *vpt;  // per pivot W x W, V_P row-major
    int *flag;    // per pivot: 1 apply V_P, 0 nothing to apply
    SweepCounters *ctr;
    // for the breakdown path: the matrices themselves
    double *G;
    int m;
    long ldg;
    double *V;
    int nv;
    long ldv;
};

template <int W>
__global__ __launch_bounds__(1024) void k_pivot_solve(PivotSolveArgs a)
{
    constexpr int NW = 16;
    extern __shared__ double lds[];
    double *A = lds;            // W x W column-major: Gram, then R
    double *VP = lds + W * W;   // W x W column-major
    __shared__ signed char JP[W];
    __shared__ int s_need, s_bad, s_broke;
    __shared__ unsigned long long s_rot[NW], s_cl[NW];
    const int pv = blockIdx.x;
    const int2 IJ = a.piv[pv];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b = a.b;

    if (tid < W) JP[tid] = a.J ? a.J[pivot_col(tid, IJ, b)] : (signed char)1;
    if (tid == 0) {
        s_need = 0;
        s_bad = 0;
        s_broke = 0;
    }
    // A_P: sum of the split partials (upper tiles), mirrored to the lower part
    for (int e = tid; e < W * W; e += 1024) {
        int r = e % W, c = e / W;
        if ((r / 16) > (c / 16) || ((r / 16) == (c / 16) && r > c)) {
            const int t = r;
            r = c;
            c = t;
        }
        const double *src = a.partial + (size_t)pv * a.nsplit * W * W + (size_t)c * W + r;
        double s = 0.0;
        for (int sp = 0; sp < a.nsplit; ++sp) s += src[(size_t)sp * W * W];
        A[e] = s;
    }
    __syncthreads();
    // skip test on the targeted off-diagonal entries; finiteness of all
    for (int e = tid; e < W * W; e += 1024) {
        const int r = e % W, c = e / W;
        const double x = A[e];
        if (!isfinite(x)) s_bad = 1;
        if (r < c && (a.all_pairs || (r < b && c >= b))) {
            const double arr = A[r * W + r], acc = A[c * W + c];
            if (arr != 0.0 && acc != 0.0 && fabs(x) > a.tol * sqrt(arr) * sqrt(acc)) s_need = 1;
        }
    }
    __syncthreads();
    if (s_bad) {
        if (tid == 0) {
            atomicOr(&a.ctr->nonfinite, 1u);
            a.flag[pv] = 0;
        }
        return;
    }
    if (!s_need) {
        if (tid == 0) a.flag[pv] = 0;
        return;
    }
    // Cholesky A_P = R^T R, right-looking, R kept in the upper triangle of A
    for (int j = 0; j < W; ++j) {
        if (tid == 0) {
            const double d = A[j * W + j];
            if (d > 0.0)
                A[j * W + j] = sqrt(d);
            else
                s_broke = 1;
        }
        __syncthreads();
        if (s_broke) break;
        const double rjj = A[j * W + j];
        for (int l = j + 1 + tid; l < W; l += 1024) A[l * W + j] /= rjj;
        __syncthreads();
        for (int e = tid; e < W * W; e += 1024) {
            const int i = e % W, l = e / W;
            if (i > j && i <= l) A[l * W + i] -= A[i * W + j] * A[l * W + j];
        }
        __syncthreads();
    }
    const bool broke = s_broke != 0;
    InnerTables tab = a.all_pairs ? a.full : a.cross;
    unsigned long long rot = 0, ncl = 0;
    int bad = 0;
    if (!broke) {
        for (int e = tid; e < W * W; e += 1024) {
            const int r = e % W, c = e / W;
            if (r > c) A[e] = 0.0;
            VP[e] = (r == c) ? 1.0 : 0.0;
        }
        __syncthreads();
    }
    const int sweeps = a.full_block ? a.max_inner : 1;
    for (int it = 0; it < sweeps; ++it) {
        unsigned long long r0 = rot;
        if (!broke) {
            inner_sweep<NW>(A, W, W, VP, W, W, JP, tab, a.tol, rot, ncl, &bad);
        } else {
            // G_P is transformed in place, and V with it: no V_P to apply
            double *gbase = a.G, *vbase = a.V;
            // columns of the pivot are not contiguous: run on the two blocks
            // through a column map by transforming pivot-local pair indices
            // into global ones
            for (int s = 0; s < tab.nsteps; ++s) {
                for (int e = tab.start[s] + wave; e < tab.start[s + 1]; e += NW) {
                    const int2 pq = tab.pairs[e];
                    double *xp = gbase + (size_t)pivot_col(pq.x, IJ, b) * a.ldg;
                    double *xq = gbase + (size_t)pivot_col(pq.y, IJ, b) * a.ldg;
                    double app = 0.0, aqq = 0.0, apq = 0.0;
                    for (int r = lane; r < a.m; r += 64) {
                        const double x = xp[r], y = xq[r];
                        app = fma(x, x, app);
                        aqq = fma(y, y, aqq);
                        apq = fma(x, y, apq);
                    }
                    app = wave_sum(app);
                    aqq = wave_sum(aqq);
                    apq = wave_sum(apq);
                    if (!finite3(app, aqq, apq)) {
                        bad = 1;
                        continue;
                    }
                    if (!needs_rotation(app, aqq, apq, a.tol)) continue;
                    const bool same = JP[pq.x] == JP[pq.y];
                    double c, sn;
                    if (transform_params(app, aqq, apq, same, c, sn) && lane == 0) ++ncl;
                    for (int r = lane; r < a.m; r += 64) {
                        double x = xp[r], y = xq[r];
                        rotate_elems(x, y, c, sn, same);
                        xp[r] = x;
                        xq[r] = y;
                    }
                    if (vbase) {
                        double *yp = vbase + (size_t)pivot_col(pq.x, IJ, b) * a.ldv;
                        double *yq = vbase + (size_t)pivot_col(pq.y, IJ, b) * a.ldv;
                        for (int r = lane; r < a.nv; r += 64) {
                            double x = yp[r], y = yq[r];
                            rotate_elems(x, y, c, sn, same);
                            yp[r] = x;
                            yq[r] = y;
                        }
                    }
                    if (lane == 0) ++rot;
                }
                __syncthreads();
            }
        }
        // rotations of this inner sweep, summed over the workgroup
        if (lane == 0) s_rot[wave] = rot - r0;
        __syncthreads();
        unsigned long long tot = 0;
        for (int w = 0; w < NW; ++w) tot += s_rot[w];
        __syncthreads();
        if (tot == 0) break;
    }
    if (lane == 0) {
        s_rot[wave] = rot;
        s_cl[wave] = ncl;
    }
    if (bad) s_bad = 1;
    __syncthreads();
    unsigned long long tot = 0, totc = 0;
    for (int w = 0; w < NW; ++w) {
        tot += s_rot[w];
        totc += s_cl[w];
    }
    if (tid == 0) {
        if (tot) atomicAdd(&a.ctr->rotations, tot);
        if (totc) atomicAdd(&a.ctr->clamps, totc);
        if (broke) atomicAdd(&a.ctr->breakdowns, 1ull);
        if (s_bad) atomicOr(&a.ctr->nonfinite, 1u);
        a.flag[pv] = (!broke && tot > 0 && !s_bad) ? 1 : 0;
    }
    if (!broke && tot > 0) {
        double *out = a.vpt + (size_t)pv * W * W;
        for (int e = tid; e < W * W; e += 1024) {
            const int r = e / W, c = e % W;
            out[e] = VP[c * W + r];
        }
    }
}

// ---------------------------------------------------------------- k_update
template <int W>
__global__ __launch_bounds__(256) void k_update(double *__restrict__ G, int m, long ldg,
                                                double *__restrict__ V, int nv, long ldv, int b,
                                                const int2 *__restrict__ piv,
                                                const double *__restrict__ vpt,
                                                const int *__restrict__ flag, int tiles_g)
{
    constexpr int KS = W / 4;   // k-steps of the MFMA
    constexpr int NT = W / 16;  // output column tiles
    __shared__ double S[W * W]; // V_P row-major
    const int pv = blockIdx.y;
    if (flag[pv] != 1) return;
    const int2 IJ = piv[pv];
    const bool isV = (int)blockIdx.x >= tiles_g;
    double *X = isV ? V : G;
    const long ld = isV ? ldv : ldg;
    const int rows = isV ? nv : m;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = ((isV ? (int)blockIdx.x - tiles_g : (int)blockIdx.x) * 64) + wave * 16 + lane % 16;

    const double *src = vpt + (size_t)pv * W * W;
    for (int e = threadIdx.x; e < W * W; e += 256) S[e] = src[e];
    double bf[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + lane / 16;
        bf[ks] = (row < rows) ? X[(size_t)pivot_col(k, IJ, b) * ld + row] : 0.0;
    }
    __syncthreads();
    d4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const double *srow = S + (4 * ks + lane / 16) * W + (lane % 16);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma16x16x4(srow[t * 16], bf[ks], acc[t]);
    }
    if (row < rows) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int col = t * 16 + lane / 16 + 4 * r;
                X[(size_t)pivot_col(col, IJ, b) * ld + row] = acc[t][r];
            }
    }
}

// ------------------------------------------------------------ host driver
bool block_width_supported(int b) { return b == 16 || b == 32; }

bool block_shape_supported(int m, int n, int b)
{
    return block_width_supported(b) && n % (2 * b) == 0 && m >= n;
}

int choose_block_width(int m, int n)
{
    (void)m;
    if (n % 64 == 0) return 32;
    if (n % 32 == 0) return 16;
    return 32;   // rejected later by block_shape_supported
}

int auto_variant(int m, int n)
{
    (void)m;
    (void)n;
    return JEVD_VAR_POINTWISE;
}

namespace {

#define HIP_TRY(expr)                                                      \
    do {                                                                   \
        hipError_t _e = (expr);                                            \
        if (_e != hipSuccess) {                                            \
            (void)hipGetLastError();                                       \
            return (_e == hipErrorOutOfMemory) ? JEVD_ENOMEM : JEVD_EHIP;  \
        }                                                                  \
    } while (0)

template <class T>
int grow(T **p, size_t *cap, size_t need)
{
    if (*cap >= need && *p) return JEVD_OK;
    if (*p) HIP_TRY(hipFree(*p));
    *p = nullptr;
    *cap = 0;
    HIP_TRY(hipMalloc((void **)p, need * sizeof(T)));
    *cap = need;
    return JEVD_OK;
}

}  // namespace

struct BlockTables {
    int b = -1, N = -1;
    std::vector<int> outer_start;
    int2 *d_outer = nullptr;
    size_t cap_outer = 0;
    int2 *d_inner = nullptr;      // full table, then cross table
    int *d_inner_start = nullptr; // full starts, then cross starts
    size_t cap_inner = 0, cap_inner_start = 0;
    int nfull = 0, ncross = 0, full_pairs = 0;
};

static BlockTables *tables_of(BlockWorkspace *ws)
{
    if (!ws->tables) ws->tables = new BlockTables();
    return (BlockTables *)ws->tables;
}

static int prepare_tables(BlockWorkspace *ws, int N, int b, hipStream_t st)
{
    BlockTables *t = tables_of(ws);
    if (t->N == N && t->b == b) return JEVD_OK;
    std::vector<int> os, op, fs, fp;
    build_ordering(N, kOrdModModulus, os, op);
    const int W = 2 * b;
    build_ordering(W, kOrdModModulus, fs, fp);
    // cross pairs: step s = 0..b-1 holds (k, b + (k + s) mod b), k = 0..b-1
    std::vector<int> cs, cp;
    for (int s = 0; s < b; ++s) {
        cs.push_back((int)cp.size() / 2);
        for (int k = 0; k < b; ++k) {
            cp.push_back(k);
            cp.push_back(b + (k + s) % b);
        }
    }
    cs.push_back((int)cp.size() / 2);
    int rc = grow(&t->d_outer, &t->cap_outer, op.size() / 2 + 1);
    if (rc) return rc;
    std::vector<int> pairs(fp);
    pairs.insert(pairs.end(), cp.begin(), cp.end());
    std::vector<int> starts(fs);
    for (int x : cs) starts.push_back(x + (int)fp.size() / 2);
    rc = grow(&t->d_inner, &t->cap_inner, pairs.size() / 2 + 1);
    if (rc) return rc;
    rc = grow(&t->d_inner_start, &t->cap_inner_start, starts.size());
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(t->d_outer, op.data(), op.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(t->d_inner, pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(t->d_inner_start, starts.data(), starts.size() * sizeof(int),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    t->outer_start = os;
    t->nfull = (int)fs.size() - 1;
    t->ncross = (int)cs.size() - 1;
    t->full_pairs = (int)fp.size() / 2;
    t->N = N;
    t->b = b;
    return JEVD_OK;
}

template <int W>
static hipError_t launch_step(BlockWorkspace *ws, const BlockRunArgs &a, BlockTables *t, int k,
                              int nsplit, int rows_per_split, SweepCounters *ctr)
{
    const int npiv = t->N / 2;
    const int2 *piv = t->d_outer + t->outer_start[k];
    hipStream_t st = a.stream;
    hipError_t e;
    if ((e = a.timer->begin(st, JEVD_K_GRAM)) != hipSuccess) return e;
    k_gram<W><<<dim3(npiv, nsplit), 256, 0, st>>>(a.G, a.m, (long)a.ldg, a.b, piv, rows_per_split,
                                                   ws->partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = a.timer->end(st)) != hipSuccess) return e;

    PivotSolveArgs p;
    p.partial = ws->partial;
    p.nsplit = nsplit;
    p.J = a.dJ;
    p.piv = piv;
    p.b = a.b;
    p.tol = a.tol;
    p.all_pairs = (a.full_block || k == 0) ? 1 : 0;
    p.full_block = a.full_block ? 1 : 0;
    p.max_inner = a.max_inner;
    p.full = InnerTables{t->d_inner, t->d_inner_start, t->nfull};
    // the cross starts follow the nfull + 1 offsets of the full table
    p.cross = InnerTables{t->d_inner, t->d_inner_start + t->nfull + 1, t->ncross};
    p.vpt = ws->vp;
    p.flag = ws->flags;
    p.ctr = ctr;
    p.G = a.G;
    p.m = a.m;
    p.ldg = a.ldg;
    p.V = a.V;
    p.nv = a.n;
    p.ldv = a.ldv;
    const size_t lds = 2 * (size_t)W * W * sizeof(double);
    if ((e = a.timer->begin(st, JEVD_K_PIVOT_SOLVE)) != hipSuccess) return e;
    k_pivot_solve<W><<<npiv, 1024, lds, st>>>(p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = a.timer->end(st)) != hipSuccess) return e;

    const int tiles_g = (a.m + 63) / 64;
    const int tiles_v = a.V ? (a.n + 63) / 64 : 0;
    if ((e = a.timer->begin(st, JEVD_K_UPDATE)) != hipSuccess) return e;
    k_update<W><<<dim3(tiles_g + tiles_v, npiv), 256, 0, st>>>(a.G, a.m, (long)a.ldg, a.V, a.n,
                                                               (long)a.ldv, a.b, piv, ws->vp,
                                                               ws->flags, tiles_g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return a.timer->end(st);
}

int run_block(BlockWorkspace *ws, const BlockRunArgs &a, int *sweeps_done)
{
    *sweeps_done = 0;
    if (!block_shape_supported(a.m, a.n, a.b)) return JEVD_EINVAL;
    const int b = a.b, W = 2 * b, N = a.n / b, npiv = N / 2;
    int rc = prepare_tables(ws, N, b, a.stream);
    if (rc) return rc;
    BlockTables *t = tables_of(ws);
    // split the rows of each Gram so that a step has about 2048 workgroups
    int nsplit = 2048 / npiv;
    if (nsplit < 1) nsplit = 1;
    int maxsplit = (a.m + 255) / 256;
    if (nsplit > maxsplit) nsplit = maxsplit;
    int rows_per_split = (a.m + nsplit - 1) / nsplit;
    rows_per_split = (rows_per_split + 31) / 32 * 32;
    nsplit = (a.m + rows_per_split - 1) / rows_per_split;
    rc = grow(&ws->partial, &ws->capPartial, (size_t)npiv * nsplit * W * W);
    if (rc) return rc;
    rc = grow(&ws->vp, &ws->capVp, (size_t)npiv * W * W);
    if (rc) return rc;
    rc = grow(&ws->flags, &ws->capFlags, (size_t)npiv);
    if (rc) return rc;
    if (W == 64 && 2 * (size_t)W * W * sizeof(double) > 65536)
        HIP_TRY(hipFuncSetAttribute((const void *)k_pivot_solve<64>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(2 * W * W * sizeof(double))));
    HIP_TRY(hipMemsetAsync(a.dctr, 0, sizeof(SweepCounters) * a.max_sweeps, a.stream));
    for (int s = 0; s < a.max_sweeps; ++s) {
        for (int k = 0; k < N; ++k) {
            hipError_t e = (W == 32) ? launch_step<32>(ws, a, t, k, nsplit, rows_per_split, a.dctr + s)
                                     : launch_step<64>(ws, a, t, k, nsplit, rows_per_split, a.dctr + s);
            HIP_TRY(e);
        }
        HIP_TRY(hipMemcpyAsync(a.hctr + s, a.dctr + s, sizeof(SweepCounters), hipMemcpyDeviceToHost,
                               a.stream));
        HIP_TRY(hipStreamSynchronize(a.stream));
        HIP_TRY(a.timer->collect());
        *sweeps_done = s + 1;
        if (a.hctr[s].nonfinite) return JEVD_ENONFINITE;
        if (a.hctr[s].rotations == 0) return JEVD_OK;
    }
    return JEVD_ENOCONV;
}

void block_workspace_free(BlockWorkspace *ws)
{
    if (ws->partial) (void)hipFree(ws->partial);
    if (ws->vp) (void)hipFree(ws->vp);
    if (ws->flags) (void)hipFree(ws->flags);
    if (ws->tables) {
        BlockTables *t = (BlockTables *)ws->tables;
        if (t->d_outer) (void)hipFree(t->d_outer);
        if (t->d_inner) (void)hipFree(t->d_inner);
        if (t->d_inner_start) (void)hipFree(t->d_inner_start);
        delete t;
    }
    *ws = BlockWorkspace();
}

}  // namespace jevd
