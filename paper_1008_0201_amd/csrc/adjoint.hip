// Canonical outputs and the adjoint of the one-sided Jacobi eigen-
// decomposition, batched over instances of one shape (m x n, m >= n).
//
// The solver leaves G V = U Sigma with V^T J V = J, so H = G J G^T has the
// orthonormal eigenvectors U and the eigenvalues lambda_i = j_i sigma_i^2
// (Sec. 1, Sec. 2.1).  For the loss L = sum_i w_i lambda_i + <C, U>, first-
// order perturbation theory of the symmetric H (simple nonzero spectrum),
// pulled back through dH = dG J G^T + G J dG^T, gives
//   dL/dG = [ U M' + [m > n] C Lambda^{-1} ] W J,   W = U^T G,  K = U^T C,
//   M'_ki = (K_ki - K_ik) / (lambda_i - lambda_k)   (k != i),
//   M'_ii = 2 w_i,
//   minus [m > n] K_ki / lambda_i in every entry (the m - n zero eigenvalues
//   of H; their term (I - U U^T) C Lambda^{-1} U^T G J is formed as
//   (C - U K) Lambda^{-1} W J).
// W is taken from G itself rather than from Sigma V^{-1}: a hyperbolic V can
// be far from orthogonal, and V^{-1} = J V^T J holds only to eps |V|^2.
// Four dense contractions (U^T C, U^T G, U M', T W) run on FP64 MFMA; M' is
// one elementwise pass.
#include "../../include/jevd.h"
#include "jevd_internal.h"

#include <hip/hip_runtime.h>

namespace jevd {

typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- canonical
// One wavefront per (instance, input column i): the rank of column i in the
// order of decreasing lambda (ties, and non-finite values mapped to -inf,
// by position, so the ranks always form a permutation), the sign that makes
// the entry of largest magnitude of u_i (the first such) positive, then
// u_i, v_i and lambda_i are written to slot rank.
__global__ __launch_bounds__(64) void k_canonical(
    int m, int n, const double *__restrict__ lam, long long slam, const double *__restrict__ U,
    int ldu, long long su, const double *__restrict__ V, int ldv, long long sv,
    double *__restrict__ lam_o, double *__restrict__ U_o, double *__restrict__ V_o)
{
    const int i = blockIdx.x, b = blockIdx.y, lane = threadIdx.x;
    const double *lb = lam + b * slam;
    auto key = [](double x) { return (x == x && x > -INFINITY) ? x : -INFINITY; };
    const double li = key(lb[i]);
    int rank = 0;
    for (int k = lane; k < n; k += 64) {
        const double lk = key(lb[k]);
        rank += (lk > li || (lk == li && k < i)) ? 1 : 0;
    }
    for (int off = 32; off > 0; off >>= 1) rank += __shfl_xor(rank, off);
    const double *ui = U + b * su + (size_t)i * ldu;
    double best = -1.0;
    int bidx = 0x7fffffff;
    for (int r = lane; r < m; r += 64) {
        const double a = fabs(ui[r]);
        if (a > best) {   // first maximum of this lane's rows
            best = a;
            bidx = r;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bidx, off);
        if (ob > best || (ob == best && oi < bidx)) {
            best = ob;
            bidx = oi;
        }
    }
    const double s = (bidx < m && ui[bidx] < 0.0) ? -1.0 : 1.0;
    double *uo = U_o + b * su + (size_t)rank * ldu;
    for (int r = lane; r < m; r += 64) uo[r] = s * ui[r];
    if (V) {
        const double *vi = V + b * sv + (size_t)i * ldv;
        double *vo = V_o + b * sv + (size_t)rank * ldv;
        for (int r = lane; r < n; r += 64) vo[r] = s * vi[r];
    }
    if (lane == 0) lam_o[b * slam + rank] = lb[i];
}

// ------------------------------------------------------------ batched GEMM
// D_b = [op(A_b) op(B_b) + E_b diag(1 / e_b)] diag(sgn_b) for column-major
// FP64 operands (the addend and the signs optional),
// op(A) M x K, op(B) K x N.  A 64 x 64 tile of D per workgroup of four
// wavefronts (2 x 2, each 32 x 32 as 2 x 2 MFMA tiles of 16 x 16); K in
// chunks of 16 staged through LDS.  Tails in M, N, K are zero-filled.
struct GemmArgs {
    int M, N, K;
    const double *A;
    int lda;
    long long sa;
    const double *B;
    int ldb;
    long long sb;
    double *D;
    int ldd;
    long long sd;
    const double *E;   // optional addend E diag(1 / e)
    int lde;
    long long se;
    const double *e;   // divisors of the columns of E (length N per instance)
    long long ses;
    const signed char *sgn;   // optional signs of the columns of D (length N)
    long long ssg;
};

constexpr int kTile = 64, kKc = 16, kPitch = kTile + 1;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_bgemm(GemmArgs g)
{
    __shared__ double As[kKc][kPitch];   // As[k][i] = op(A)[i0 + i][k0 + k]
    __shared__ double Bs[kKc][kPitch];   // Bs[k][j] = op(B)[k0 + k][j0 + j]
    const int b = blockIdx.z;
    const int i0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wi = (wave & 1) * 32, wj = (wave >> 1) * 32;
    const double *A = g.A + b * g.sa;
    const double *B = g.B + b * g.sb;
    d4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < g.K; k0 += kKc) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int i, k;
            if (!TA) {   // op(A)[i][k] = A[i + k lda]: consecutive threads, consecutive i
                i = tid & 63;
                k = (tid >> 6) + 4 * r;
            } else {     // op(A)[i][k] = A[k + i lda]: consecutive threads, consecutive k
                k = tid & 15;
                i = (tid >> 4) + 16 * r;
            }
            const int gi = i0 + i, gk = k0 + k;
            double x = 0.0;
            if (gi < g.M && gk < g.K) x = TA ? A[gk + (size_t)gi * g.lda] : A[gi + (size_t)gk * g.lda];
            As[k][i] = x;
            int j, kb;
            if (!TB) {   // op(B)[k][j] = B[k + j ldb]
                kb = tid & 15;
                j = (tid >> 4) + 16 * r;
            } else {     // op(B)[k][j] = B[j + k ldb]
                j = tid & 63;
                kb = (tid >> 6) + 4 * r;
            }
            const int gj = j0 + j, gkb = k0 + kb;
            double y = 0.0;
            if (gj < g.N && gkb < g.K) y = TB ? B[gj + (size_t)gkb * g.ldb] : B[gkb + (size_t)gj * g.ldb];
            Bs[kb][j] = y;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKc; kk += 4) {
            const int kr = kk + lane / 16;
            const double a0 = As[kr][wi + (lane & 15)];
            const double a1 = As[kr][wi + 16 + (lane & 15)];
            const double b0 = Bs[kr][wj + (lane & 15)];
            const double b1 = Bs[kr][wj + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
    double *D = g.D + b * g.sd;
    const double *E = g.E ? g.E + b * g.se : nullptr;
    const double *e = g.e ? g.e + b * g.ses : nullptr;
    const signed char *sg = g.sgn ? g.sgn + b * g.ssg : nullptr;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int col = j0 + wj + 16 * y + (lane & 15);
            if (col >= g.N) continue;
            const double ediv = (E && e) ? e[col] : 1.0;
            const bool neg = sg && sg[col] < 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i0 + wi + 16 * x + lane / 16 + 4 * r;
                if (row >= g.M) continue;
                double v = acc[x][y][r];
                if (E) v += E[row + (size_t)col * g.lde] / ediv;
                D[row + (size_t)col * g.ldd] = neg ? -v : v;
            }
        }
}

// ------------------------------------------------------------- middle step
// M'_ki from K (n x n, null for C = 0), lambda and w (null for w = 0).
__global__ __launch_bounds__(256) void k_adj_mid(int m, int n, const double *__restrict__ lam,
                                                 long long slam, const double *__restrict__ w,
                                                 long long sw, const double *__restrict__ K,
                                                 double *__restrict__ Mp)
{
    const int b = blockIdx.y;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long long)n * n) return;
    const int k = (int)(e % n), i = (int)(e / n);
    const double *lb = lam + b * slam;
    const double li = lb[i];
    const double *Kb = K ? K + (size_t)b * n * n : nullptr;
    double v;
    if (k == i) {
        v = w ? 2.0 * w[b * sw + i] : 0.0;
    } else {
        v = Kb ? (Kb[k + (size_t)i * n] - Kb[i + (size_t)k * n]) / (li - lb[k]) : 0.0;
    }
    if (Kb && m > n) v -= Kb[k + (size_t)i * n] / li;
    Mp[(size_t)b * n * n + e] = v;
}

// ------------------------------------------------------------------- host
hipError_t launch_canonical(int batch, int m, int n, const double *lam, long long slam,
                            const double *U, int ldu, long long su, const double *V, int ldv,
                            long long sv, double *lam_o, double *U_o, double *V_o, hipStream_t st)
{
    k_canonical<<<dim3(n, batch), 64, 0, st>>>(m, n, lam, slam, U, ldu, su, V, ldv, sv, lam_o, U_o,
                                              V_o);
    return hipGetLastError();
}

static void launch_gemm(bool ta, bool tb, const GemmArgs &g, int batch, hipStream_t st)
{
    dim3 grid((g.M + kTile - 1) / kTile, (g.N + kTile - 1) / kTile, batch);
    if (ta && !tb) k_bgemm<true, false><<<grid, 256, 0, st>>>(g);
    else if (!ta && !tb) k_bgemm<false, false><<<grid, 256, 0, st>>>(g);
    else if (!ta && tb) k_bgemm<false, true><<<grid, 256, 0, st>>>(g);
    else k_bgemm<true, true><<<grid, 256, 0, st>>>(g);
}

hipError_t launch_adjoint(int batch, int m, int n, const double *G, int ldg, long long sg,
                          const signed char *J, long long sj, const double *lam, long long slam,
                          const double *U, int ldu, long long su, const double *w, long long sw,
                          const double *C, int ldc, long long sc, double *dG, int ldd,
                          long long sd, double *wsK, double *wsW, double *wsM, double *wsT,
                          hipStream_t st)
{
    const long long nn = (long long)n * n, mn = (long long)m * n;
    if (C) {   // K = U^T C
        GemmArgs g{};
        g.M = n; g.N = n; g.K = m;
        g.A = U; g.lda = ldu; g.sa = su;
        g.B = C; g.ldb = ldc; g.sb = sc;
        g.D = wsK; g.ldd = n; g.sd = nn;
        launch_gemm(true, false, g, batch, st);
    }
    {   // W = U^T G
        GemmArgs g{};
        g.M = n; g.N = n; g.K = m;
        g.A = U; g.lda = ldu; g.sa = su;
        g.B = G; g.ldb = ldg; g.sb = sg;
        g.D = wsW; g.ldd = n; g.sd = nn;
        launch_gemm(true, false, g, batch, st);
    }
    {
        dim3 grid((unsigned)((nn + 255) / 256), batch);
        k_adj_mid<<<grid, 256, 0, st>>>(m, n, lam, slam, w, sw, C ? wsK : nullptr, wsM);
    }
    {   // T = U M' [+ C Lambda^{-1} when m > n]
        GemmArgs g{};
        g.M = m; g.N = n; g.K = n;
        g.A = U; g.lda = ldu; g.sa = su;
        g.B = wsM; g.ldb = n; g.sb = nn;
        g.D = wsT; g.ldd = m; g.sd = mn;
        if (C && m > n) {
            g.E = C; g.lde = ldc; g.se = sc;
            g.e = lam; g.ses = slam;
        }
        launch_gemm(false, false, g, batch, st);
    }
    {   // dG = T W J
        GemmArgs g{};
        g.M = m; g.N = n; g.K = n;
        g.A = wsT; g.lda = m; g.sa = mn;
        g.B = wsW; g.ldb = n; g.sb = nn;
        g.D = dG; g.ldd = ldd; g.sd = sd;
        g.sgn = J; g.ssg = sj;
        launch_gemm(false, false, g, batch, st);
    }
    return hipGetLastError();
}

}  // namespace jevd
