// Batched FP64 GEMM on MFMA (v_mfma_f64_16x16x4f64) with a fused epilogue.
#include "gemm.h"

namespace jevd {

typedef double d4 __attribute__((ext_vector_type(4)));

// D_b = [op(A_b) op(B_b) + E_b diag(1 / e_b)] diag(sgn_b) for column-major
// FP64 operands (the addend and the signs optional),
// op(A) M x K, op(B) K x N.  A 64 x 64 tile of D per workgroup of four
// wavefronts (2 x 2, each 32 x 32 as 2 x 2 MFMA tiles of 16 x 16); K in
// chunks of 32 staged through LDS, the next chunk loaded into registers
// while the MFMAs run on the current one.  Tails in M, N, K are
// zero-filled.  The MFMAs accumulate over k in increasing order whatever
// the chunking.
constexpr int kTile = 64, kKc = 32, kPitch = kTile + 1;
constexpr int kPer = kKc * kTile / 256;   // elements of each operand per thread and chunk

// Thread tid's share of a chunk: op(A)[i][k] and op(B)[kb][j], with
// consecutive threads on consecutive addresses of the column-major operands.
template <bool TA, bool TB>
__device__ __forceinline__ void chunk_index(int tid, int r, int &i, int &k, int &j, int &kb)
{
    if (!TA) {   // op(A)[i][k] = A[i + k lda]
        i = tid & 63;
        k = (tid >> 6) + 4 * r;
    } else {     // op(A)[i][k] = A[k + i lda]
        k = tid & 31;
        i = (tid >> 5) + 8 * r;
    }
    if (!TB) {   // op(B)[k][j] = B[k + j ldb]
        kb = tid & 31;
        j = (tid >> 5) + 8 * r;
    } else {     // op(B)[k][j] = B[j + k ldb]
        j = tid & 63;
        kb = (tid >> 6) + 4 * r;
    }
}

template <bool TA, bool TB>
__device__ __forceinline__ void load_chunk(const GemmArgs &g, const double *A, const double *B, int i0,
                                           int j0, int k0, int tid, double (&xa)[kPer],
                                           double (&xb)[kPer])
{
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        int i, k, j, kb;
        chunk_index<TA, TB>(tid, r, i, k, j, kb);
        const int gi = i0 + i, gk = k0 + k, gj = j0 + j, gkb = k0 + kb;
        xa[r] = (gi < g.M && gk < g.K) ? (TA ? A[gk + (size_t)gi * g.lda] : A[gi + (size_t)gk * g.lda])
                                       : 0.0;
        xb[r] = (gj < g.N && gkb < g.K) ? (TB ? B[gj + (size_t)gkb * g.ldb] : B[gkb + (size_t)gj * g.ldb])
                                        : 0.0;
    }
}

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

    double xa[kPer], xb[kPer];
    load_chunk<TA, TB>(g, A, B, i0, j0, 0, tid, xa, xb);
    for (int k0 = 0; k0 < g.K; k0 += kKc) {
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            int i, k, j, kb;
            chunk_index<TA, TB>(tid, r, i, k, j, kb);
            As[k][i] = xa[r];
            Bs[kb][j] = xb[r];
        }
        __syncthreads();
        // the next chunk's loads are in flight during this chunk's MFMAs
        if (k0 + kKc < g.K) load_chunk<TA, TB>(g, A, B, i0, j0, k0 + kKc, tid, xa, xb);
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

void launch_gemm(bool ta, bool tb, const GemmArgs &g, int batch, hipStream_t st)
{
    dim3 grid((g.M + kTile - 1) / kTile, (g.N + kTile - 1) / kTile, batch);
    if (ta && !tb) k_bgemm<true, false><<<grid, 256, 0, st>>>(g);
    else if (!ta && !tb) k_bgemm<false, false><<<grid, 256, 0, st>>>(g);
    else if (!ta && tb) k_bgemm<false, true><<<grid, 256, 0, st>>>(g);
    else k_bgemm<true, true><<<grid, 256, 0, st>>>(g);
}

}  // namespace jevd
