// Device-side arithmetic shared by the Jacobi kernels: 2x2 transform
// parameters, the rotation threshold and wavefront / workgroup reductions.
// gfx950 (CDNA4): 64-lane wavefronts.
#pragma once
#include <hip/hip_runtime.h>

namespace jevd {

constexpr int kWave = 64;

// Parameters of the 2x2 transform that diagonalises the pivot Gram
// [[app, apq], [apq, aqq]] of a column pair (Sec. 2.1, step 2).
//
// Equal signs in J (trigonometric rotation, the real case of (2.1) with the
// sign convention of (A.1)): new columns (c g_p - s g_q, s g_p + c g_q).
// The new off-diagonal entry cs(app - aqq) + (c^2 - s^2) apq vanishes for
// t = s / c solving t^2 + 2 z t - 1 = 0, z = (aqq - app) / (2 apq); the
// smaller root is t = sgn(z) / (|z| + sqrt(1 + z^2)), c = 1 / sqrt(1 + t^2).
//
// Opposite signs (hyperbolic transform, Sec. 2.1): new columns
// (ch g_p + sh g_q, sh g_p + ch g_q).  The new off-diagonal entry
// ch sh (app + aqq) + (ch^2 + sh^2) apq vanishes for t = sh / ch solving
// t^2 + 2 z t + 1 = 0, z = (app + aqq) / (2 apq); the smaller root is
// t = -sgn(z) / (|z| + sqrt((|z| - 1)(|z| + 1))), ch = 1 / sqrt((1 - t)(1 + t)).
// |z| >= 1 holds in exact arithmetic (the Gram is positive semidefinite);
// if rounding gives |z| <= 1 the transform would be singular and |tanh| is
// clamped to 0.9 (Sec. 3.2).
//
// sgn(z) = +1 for z >= 0 (also for -0).  For |z| > 1e150, t takes its limit
// 1 / (2 z) (trig) or -1 / (2 z) (hyperbolic) so that z^2 cannot overflow.
// Returns true if the hyperbolic clamp was used.
__device__ __forceinline__ bool transform_params(double app, double aqq, double apq,
                                                 bool same_sign, double &c, double &s)
{
    double t;
    bool clamped = false;
    if (same_sign) {
        const double z = (aqq - app) / (2.0 * apq);
        const double az = fabs(z);
        if (az > 1e150) {
            t = 1.0 / (2.0 * z);
        } else {
            const double sg = (z >= 0.0) ? 1.0 : -1.0;
            t = sg / (az + sqrt(1.0 + z * z));
        }
        c = 1.0 / sqrt(1.0 + t * t);
    } else {
        const double z = (app + aqq) / (2.0 * apq);
        const double sg = (z >= 0.0) ? 1.0 : -1.0;
        const double az = fabs(z);
        if (az <= 1.0) {
            t = -sg * 0.9;
            clamped = true;
        } else if (az > 1e150) {
            t = -1.0 / (2.0 * z);
        } else {
            t = -sg / (az + sqrt((az - 1.0) * (az + 1.0)));
        }
        c = 1.0 / sqrt((1.0 - t) * (1.0 + t));
    }
    s = c * t;
    return clamped;
}

// The rotation decision of one pair: rotate iff both columns are nonzero and
// |apq| > tol * sqrt(app) * sqrt(aqq).
__device__ __forceinline__ bool needs_rotation(double app, double aqq, double apq, double tol)
{
    if (app == 0.0 || aqq == 0.0) return false;
    return fabs(apq) > tol * sqrt(app) * sqrt(aqq);
}

__device__ __forceinline__ bool finite3(double a, double b, double c)
{
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// New values of one element pair under the transform.
__device__ __forceinline__ void rotate_elems(double &x, double &y, double c, double s, bool same_sign)
{
    const double xo = x, yo = y;
    if (same_sign) {
        x = c * xo - s * yo;
        y = s * xo + c * yo;
    } else {
        x = c * xo + s * yo;
        y = s * xo + c * yo;
    }
}

// Butterfly sum over the 64 lanes of a wavefront; every lane ends with the
// total, summed in the same order on every lane (deterministic).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum of three values over a workgroup of BS threads; every thread gets the
// totals.  sh must hold 3 * BS / 64 doubles of LDS.  Contains a barrier.
template <int BS>
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *sh)
{
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    if constexpr (BS > kWave) {
        constexpr int NW = BS / kWave;
        const int w = threadIdx.x / kWave;
        if ((threadIdx.x & (kWave - 1)) == 0) {
            sh[w] = a;
            sh[NW + w] = b;
            sh[2 * NW + w] = c;
        }
        __syncthreads();
        a = sh[0];
        b = sh[NW];
        c = sh[2 * NW];
#pragma unroll
        for (int i = 1; i < NW; ++i) {
            a += sh[i];
            b += sh[NW + i];
            c += sh[2 * NW + i];
        }
    }
}

// Per-sweep counters kept in device memory (one slot per sweep).
struct SweepCounters {
    unsigned long long rotations;  // pairs (or inner pairs) rotated in the sweep
    unsigned long long clamps;     // hyperbolic transforms clamped
    unsigned long long breakdowns; // block pivots whose Cholesky broke down
    unsigned int nonfinite;        // set when a Gram entry is NaN or Inf
    unsigned int pad;
};

}  // namespace jevd
