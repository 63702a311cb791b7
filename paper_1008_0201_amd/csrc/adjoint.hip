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
#include "gemm.h"
#include "jevd_internal.h"

#include <hip/hip_runtime.h>

namespace jevd {

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

// ------------------------------------------------------------- middle step
// M'_ki from K (n x n, null for C = 0), lambda and w (null for w = 0).  A
// 32 x 32 tile of M' per workgroup: the matching tiles of K and of K^T are
// read with consecutive threads on consecutive rows and staged in LDS, so
// neither read is strided.
constexpr int kMidTile = 32;
__global__ __launch_bounds__(256) void k_adj_mid(int m, int n, const double *__restrict__ lam,
                                                 long long slam, const double *__restrict__ w,
                                                 long long sw, const double *__restrict__ K,
                                                 double *__restrict__ Mp)
{
    __shared__ double t1[kMidTile][kMidTile + 1];   // t1[c][r] = K[k0 + r, i0 + c]
    __shared__ double t2[kMidTile][kMidTile + 1];   // t2[c][r] = K[i0 + r, k0 + c]
    const int b = blockIdx.z;
    const int k0 = blockIdx.x * kMidTile, i0 = blockIdx.y * kMidTile;
    const int tx = threadIdx.x % kMidTile, ty = threadIdx.x / kMidTile;
    constexpr int kRowsPerPass = 256 / kMidTile;
    const double *Kb = K ? K + (size_t)b * n * n : nullptr;
    if (Kb) {
        for (int c = ty; c < kMidTile; c += kRowsPerPass) {
            const int i = i0 + c, k = k0 + tx;
            t1[c][tx] = (i < n && k < n) ? Kb[k + (size_t)i * n] : 0.0;
            const int kc = k0 + c, ir = i0 + tx;
            t2[c][tx] = (kc < n && ir < n) ? Kb[ir + (size_t)kc * n] : 0.0;
        }
    }
    __syncthreads();
    const double *lb = lam + b * slam;
    for (int c = ty; c < kMidTile; c += kRowsPerPass) {
        const int i = i0 + c, k = k0 + tx;
        if (i >= n || k >= n) continue;
        const double li = lb[i];
        const double kki = Kb ? t1[c][tx] : 0.0;   // K[k, i]
        const double kik = Kb ? t2[tx][c] : 0.0;   // K[i, k]
        double v;
        if (k == i) {
            v = w ? 2.0 * w[b * sw + i] : 0.0;
        } else {
            v = Kb ? (kki - kik) / (li - lb[k]) : 0.0;
        }
        if (Kb && m > n) v -= kki / li;
        Mp[(size_t)b * n * n + k + (size_t)i * n] = v;
    }
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
        const unsigned tiles = (unsigned)((n + kMidTile - 1) / kMidTile);
        dim3 grid(tiles, tiles, batch);
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
