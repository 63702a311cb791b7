// Batched FP64 GEMM on MFMA with a fused epilogue, shared by the adjoint
// and the re-orthogonalisation of the mixed-precision path.
#pragma once
#include <hip/hip_runtime.h>

namespace jevd {

// D_b = [op(A_b) op(B_b) + E_b diag(1 / e_b)] diag(sgn_b) for column-major
// FP64 operands (the addend and the signs optional), op(A) M x K, op(B)
// K x N, instance b at the given batch strides.
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

// Enqueues the GEMM of `batch` instances on st (op = transpose when ta / tb).
void launch_gemm(bool ta, bool tb, const GemmArgs &g, int batch, hipStream_t st);

}  // namespace jevd
