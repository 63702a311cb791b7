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

// transform_params as one branch-free chain, for wavefronts whose lanes
// take different cases (trigonometric and hyperbolic pairs, |zeta| past
// 1e150, the clamp): each case's expression is selected as an operand
// instead of run as a branch of its own, so the wavefront runs one division
// -> square root -> division -> square root -> division chain instead of
// one per case.  The values are those of transform_params (the same
// expressions, chosen by the same conditions).  Callers test needs_rotation
// first and skip this when no lane of the wavefront needs a transform.
__device__ __forceinline__ bool transform_params_bf(double app, double aqq, double apq,
                                                    bool same_sign, double &c, double &s)
{
    const double z = (same_sign ? aqq - app : app + aqq) / (2.0 * apq);
    const double az = fabs(z);
    const double sg = (z >= 0.0) ? 1.0 : -1.0;
    const double rad = same_sign ? 1.0 + z * z : (az - 1.0) * (az + 1.0);
    double t = (same_sign ? sg : -sg) / (az + sqrt(rad));
    t = (az > 1e150) ? (same_sign ? 1.0 : -1.0) / (2.0 * z) : t;
    const bool clamped = !same_sign && az <= 1.0;
    t = clamped ? -sg * 0.9 : t;
    c = 1.0 / sqrt(same_sign ? 1.0 + t * t : (1.0 - t) * (1.0 + t));
    s = c * t;
    return clamped;
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

// DPP lane permutation of a double (both 32-bit halves moved alike).
// CTRL: 0xB1 quad_perm [1,0,3,2] (lane ^ 1), 0x4E quad_perm [2,3,0,1]
// (lane ^ 2), 0x141 row_half_mirror (i <-> 7-i within 8 lanes), 0x140
// row_mirror (i <-> 15-i within 16 lanes).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront; every lane ends with the same total.
// Within each row of 16 lanes a butterfly of DPP moves (xor 1, xor 2, then
// the half-mirror and mirror, which pair the two quads and the two halves);
// the four row sums are then read from lanes 0, 16, 32, 48 and added as
// (r0 + r1) + (r2 + r3).  Every lane adds the same operands in the same
// order, so the result is identical on all lanes and from run to run.
// All 64 lanes must be active.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_move<0xB1>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0x141>(v);
    v += dpp_move<0x140>(v);
    const double r0 = read_lane(v, 0), r1 = read_lane(v, 16);
    const double r2 = read_lane(v, 32), r3 = read_lane(v, 48);
    return (r0 + r1) + (r2 + r3);
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
