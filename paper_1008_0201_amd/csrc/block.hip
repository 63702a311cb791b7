// Block one-sided Jacobi (Sec. 2.2-2.3; Alg. 3.4 with unpivoted Cholesky,
// or the sign-pivoted Cholesky of Alg. 3.3): block-oriented (BO) and full
// block (FB), trigonometric or hyperbolic.
//
// The n columns form N = 2 ceil(n / 2b) block columns whose widths differ by
// at most one and are at most b (Sec. 3); block pairs (I, J) follow the
// modified modulus ordering over the N blocks (ring order, as in the
// pointwise path).  A pivot G_P = [G_I G_J] has W = 2b positions, block I
// in positions [0, b) and block J in [b, 2b); a block narrower than b leaves
// its last positions empty (they load as zero columns, get an identity row
// and column in the pivot Gram and transform, and are never stored).  One
// outer step runs three kernels over its N/2 pivots:
//   k_gram        A_P = G_P^T G_P on FP64 MFMA (v_mfma_f64_16x16x4f64), the
//                 rows split over several workgroups (split-K); only the
//                 upper 16 x 16 tiles are formed; partial sums go to a
//                 workspace and are added in split order by the pivot solve.
//   k_pivot_solve one workgroup per pivot: skip test, Cholesky A_P = R^T R,
//                 inner one-sided sweeps on the columns of R (trig or
//                 hyperbolic by J_P), accumulating V_P; writes V_P
//                 row-major.  After a Cholesky breakdown the inner sweeps run
//                 on the columns of G_P in place instead, still accumulating
//                 V_P, which is then applied to V only.  For W = 128 (b = 64)
//                 R alone fills the LDS: the inner transforms are logged and
//                 V_P is formed from the log once R is no longer needed.
//   k_update      [G_I G_J] <- [G_I G_J] V_P and [V_I V_J] <- [V_I V_J] V_P
//                 on FP64 MFMA, in place, four row tiles per workgroup: each
//                 wavefront computes (G_P V_P)^T for 16 rows of a tile, so
//                 that both the loads of G_P and the stores of the result are
//                 16 consecutive rows per column.
#include <utility>
#include <vector>

#include "../../include/jevd.h"
#include "block.h"
#include "gemm.h"
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

// The same product for FP32 operands (v_mfma_f32_16x16x4f32): the operand
// layout is that of the FP64 instruction, but element r of the result in
// lane l is D[4 (l / 16) + r][l % 16].
typedef float f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4 mfma16x16x4(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Accumulator type and result row of the 16 x 16 x 4 product per element type.
template <class T> struct Mfma;
template <> struct Mfma<double> {
    typedef d4 acc;
    __device__ static int row(int lane, int r) { return lane / 16 + 4 * r; }
};
template <> struct Mfma<float> {
    typedef f4 acc;
    __device__ static int row(int lane, int r) { return 4 * (lane / 16) + r; }
};

// A pivot: the first column and the width of its two blocks (x, y: block
// I; z, w: block J).  Position k (0 <= k < 2b) of the pivot is column x + k
// for k < y, column z + k - b for b <= k < b + w, and empty otherwise.
__device__ __forceinline__ int pivot_col(int k, int4 d, int b)
{
    if (k < b) return k < d.y ? d.x + k : -1;
    return (k - b) < d.w ? d.z + (k - b) : -1;
}
__device__ __forceinline__ bool pivot_real(int k, int4 d, int b)
{
    return k < b ? k < d.y : (k - b) < d.w;
}

// Orders the LDS accesses of one wavefront across lanes: one wavefront's
// LDS operations complete in issue order, and the fences keep the compiler
// from moving them across this point.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ k_gram
// Tile t of the upper triangle of NT x NT tiles, row-major: row and column.
__host__ __device__ constexpr int upper_tile_i(int NT, int t)
{
    int it = 0;
    while (t >= NT - it) {   // row it of the upper triangle has NT - it tiles
        t -= NT - it;
        ++it;
    }
    return it;
}
__host__ __device__ constexpr int upper_tile_j(int NT, int t)
{
    int it = 0;
    while (t >= NT - it) {
        t -= NT - it;
        ++it;
    }
    return it + t;
}

// x, or +0 when !keep, without a branch (an all-ones or all-zeros mask on
// the bits).
__device__ __forceinline__ double zero_unless(double x, bool keep)
{
    const long long m = -(long long)keep;
    return __longlong_as_double(__double_as_longlong(x) & m);
}
__device__ __forceinline__ float zero_unless(float x, bool keep)
{
    const int m = -(int)keep;
    return __int_as_float(__float_as_int(x) & m);
}

// Tile WV + 4 Q of the upper triangle (past the last tile: tile 0 again,
// computed but not stored), known at compile time.
template <int NT, int WV, int Q>
struct GramTile {
    static constexpr int t = (WV + 4 * Q < NT * (NT + 1) / 2) ? WV + 4 * Q : 0;
    static constexpr int i = upper_tile_i(NT, t);
    static constexpr int j = upper_tile_j(NT, t);
};

template <int NT, int WV, class T, class Acc, size_t... Q>
__device__ __forceinline__ void gram_mfmas(const T *cur, Acc *acc, std::index_sequence<Q...>)
{
    ((acc[Q] = mfma16x16x4(cur[GramTile<NT, WV, Q>::i], cur[GramTile<NT, WV, Q>::j], acc[Q])), ...);
}

// The MFMAs of one staged slab for wavefront WV: tiles WV, WV + 4, ... of
// the upper triangle, all indices known at compile time.  Each k-step reads
// the NT column-block operands once; the reads of step k + 1 are issued
// before the MFMAs of step k.
template <int W, class T, int KR, int LDC, int WV>
__device__ __forceinline__ void gram_slab(const T *st, int lane, typename Mfma<T>::acc *acc)
{
    constexpr int NT = W / 16;
    constexpr int NUP = NT * (NT + 1) / 2;
    constexpr int TPW = (NUP + 3) / 4;
    const T *row = st + (lane / 16) * LDC + (lane % 16);
    T cur[NT], nxt[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) cur[c] = row[c * 16];
#pragma unroll
    for (int k = 0; k < KR; k += 4) {
        if (k + 4 < KR) {
#pragma unroll
            for (int c = 0; c < NT; ++c) nxt[c] = row[(k + 4) * LDC + c * 16];
        }
        gram_mfmas<NT, WV>(cur, acc, std::make_index_sequence<TPW>());
#pragma unroll
        for (int c = 0; c < NT; ++c) cur[c] = nxt[c];
    }
}

// Slabs of 32 rows of G_P (16 at W = 128, whose nine tiles per wavefront
// take the registers) are staged transposed in LDS (row pitch W+1), double
// buffered: the loads of slabs s+1 and s+2 are in flight in registers while
// the MFMAs of slab s run, with one barrier per slab.  Every wavefront runs the
// same number of tiles (the upper tiles padded with repeats that are not
// stored) and the tile indices are wave-uniform, so the k-loop has no
// branches and the LDS reads of a slab overlap its MFMAs.  Empty pivot
// positions load column 0 of their block and are stored to LDS as zeros.
template <int W, class T>
__device__ __forceinline__ void gram_body(const T *__restrict__ G, int m, long ldg,
                                          const int4 *__restrict__ piv, int rows_per_split,
                                          double *__restrict__ partial)
{
    constexpr int KR = W <= 64 ? 32 : 16;     // rows staged per slab
    constexpr int LDC = W + 1;                // padded LDS row (elements)
    constexpr int NT = W / 16;
    constexpr int NUP = NT * (NT + 1) / 2;    // upper tiles, diagonal included
    constexpr int TPW = (NUP + 3) / 4;        // tiles per wavefront
    constexpr int EPT = KR * W / 256;         // staged elements per thread
    static_assert(EPT <= 32, "one mask bit per staged element");
    __shared__ T st[2][KR * LDC];             // st[buf][kr][c] = G_P[r0 + kr][c]
    const int pv = blockIdx.x, split = blockIdx.y;
    const int4 d = piv[pv];
    const int r_begin = split * rows_per_split;
    const int r_end = min(m, r_begin + rows_per_split);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    typename Mfma<T>::acc acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = typename Mfma<T>::acc{0, 0, 0, 0};

    // element u of this thread's slab share: row kr = tid % KR of pivot
    // position c0 + CS u, c0 = tid / KR.  CS divides b = W / 2, so positions
    // CS u .. CS u + CS - 1 lie in one block: a wave-uniform block base per
    // u and a 32-bit per-lane column offset (0 for an empty position).
    constexpr int CS = 256 / KR;
    constexpr int HB = W / 2;
    static_assert(HB % CS == 0, "slab columns must not straddle the blocks");
    const int kr = threadIdx.x % KR, c0 = threadIdx.x / KR;
    const T *colb[EPT];
    unsigned coff[EPT];
    unsigned live_cols = 0;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int c = CS * u;
        const bool in_i = c < HB;
        const int o = (in_i ? c : c - HB) + c0, w = in_i ? d.y : d.w;
        const bool real = o < w;
        colb[u] = G + (size_t)(in_i ? d.x : d.z) * ldg;
        coff[u] = (unsigned)(real ? o : 0) * (unsigned)ldg;
        live_cols |= (unsigned)real << u;
    }
    const int st_off = kr * LDC + c0;
    // Two slabs of loads in flight: register sets ra and rb take alternate
    // slabs, and a set is refilled with the slab two ahead as soon as it has
    // gone to LDS.  Rows past r_end load row r_end - 1 (no predicated load:
    // every lane of a column then reads one line) and are stored to LDS as
    // zeros; the select sits at the store, so that the loads stay in flight
    // across the MFMAs.
    auto load_slab = [&](T *reg, int r0) {
        const unsigned rr = (unsigned)min(r0 + kr, r_end - 1);
#pragma unroll
        for (int u = 0; u < EPT; ++u) reg[u] = colb[u][coff[u] + rr];
    };
    auto run_slab = [&](T *reg, int r0, int buf) {
        // zeroing by a bit mask: a select here was turned into a branch
        // around the store, which left the loads counted as in flight
        const bool live = r0 + kr < r_end;
#pragma unroll
        for (int u = 0; u < EPT; ++u)
            st[buf][st_off + CS * u] = zero_unless(reg[u], live && ((live_cols >> u) & 1u));
        __syncthreads();
        load_slab(reg, r0 + 2 * KR);
        switch (wv) {
        case 0: gram_slab<W, T, KR, LDC, 0>(st[buf], lane, acc); break;
        case 1: gram_slab<W, T, KR, LDC, 1>(st[buf], lane, acc); break;
        case 2: gram_slab<W, T, KR, LDC, 2>(st[buf], lane, acc); break;
        default: gram_slab<W, T, KR, LDC, 3>(st[buf], lane, acc); break;
        }
    };
    T ra[EPT], rb[EPT];
    load_slab(ra, r_begin);
    load_slab(rb, r_begin + KR);
    for (int r0 = r_begin; r0 < r_end; r0 += 2 * KR) {
        run_slab(ra, r0, 0);
        if (r0 + KR >= r_end) break;   // the same for the whole workgroup
        run_slab(rb, r0 + KR, 1);
    }
    double *out = partial + ((size_t)pv * gridDim.y + split) * W * W;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int t = wv + 4 * q;
        if (t >= NUP) continue;
        const int ti = upper_tile_i(NT, t), tj = upper_tile_j(NT, t);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = ti * 16 + Mfma<T>::row(lane, r), col = tj * 16 + lane % 16;
            out[(size_t)col * W + row] = (double)acc[q][r];
        }
    }
}

// The step's workgroups (about 1024) are resident at once with four per CU
// for W <= 64, hence the register budget of four wavefronts per SIMD; at
// W = 128 two workgroups fit a CU (66 KiB of LDS each) and the wavefronts
// hold nine upper tiles each, so the budget is two per SIMD.
template <int W, class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_gram(
    const T *__restrict__ G, int m, long ldg, const int4 *__restrict__ piv, int rows_per_split,
    double *__restrict__ partial)
{
    gram_body<W, T>(G, m, ldg, piv, rows_per_split, partial);
}

template <class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gram128(
    const T *__restrict__ G, int m, long ldg, const int4 *__restrict__ piv, int rows_per_split,
    double *__restrict__ partial)
{
    gram_body<128, T>(G, m, ldg, piv, rows_per_split, partial);
}

// The Gram of the W = 128 pivots without LDS staging.  Wavefront w owns
// half h = w % 2 of the 36 upper tiles (18 each) and takes the chunks of 8
// rows c = w / 2, w / 2 + 2, ... of the split, so there is no barrier in the
// row loop.  The operands come straight from G: for column block c a lane
// holds column c 16 + lane % 16 at rows 2 g and 2 g + 1 of the chunk,
// g = lane / 16, read as one 16-byte load (the 64 lanes of a block cover its
// 16 columns x 8 rows).  The chunk's two k-steps take the first and the
// second element of each pair: the Gram sums over the rows, so which row
// feeds which k-slot of an MFMA only has to be the same for both operands.
// Four register sets rotate, the operands of the next three chunks in
// flight while a chunk's MFMAs run.  At the end the two row halves of each
// tile half are added in LDS (in a fixed order).  For even partitions (no
// empty position) and an even ldg (16-byte aligned row pairs); the last
// chunk of a split may be partial (rows past r_end are zero).
constexpr int kGramRowsChunk = 8;

__device__ __forceinline__ void gram_rows_load(const char *const *colb, unsigned off, double2 *o)
{
#pragma unroll
    for (int c = 0; c < 8; ++c) o[c] = *(const double2 *)(colb[c] + off);
}

// Row and column of upper tile T of 8 x 8 tiles, as compile-time constants.
template <int T> struct UpperTile8 {
    static constexpr int i = upper_tile_i(8, T);
    static constexpr int j = upper_tile_j(8, T);
};

template <int H, size_t... Q>
__device__ __forceinline__ void gram_rows_mfmas(const double *op, d4 *acc, std::index_sequence<Q...>)
{
    ((acc[Q] = mfma16x16x4(op[UpperTile8<18 * H + (int)Q>::i], op[UpperTile8<18 * H + (int)Q>::j],
                           acc[Q])),
     ...);
}

template <int H>
__device__ __forceinline__ void gram_rows_chunk(const double2 *o, d4 *acc)
{
    double op[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) op[c] = o[c].x;
    gram_rows_mfmas<H>(op, acc, std::make_index_sequence<18>());
#pragma unroll
    for (int c = 0; c < 8; ++c) op[c] = o[c].y;
    gram_rows_mfmas<H>(op, acc, std::make_index_sequence<18>());
}

// The row loop of one wavefront over the chunks c0, c0 + 2, ... (n of
// them); off: the byte offset of this lane's first row pair.  Chunk j + 3
// is loaded into the set chunk j - 1 used.  The main loop takes four chunks
// per pass without a branch (so that the count of loads in flight is the
// same on every path and the waits stay exact); the last n mod 4 chunks
// follow.  Loads past the last chunk reload it (in bounds, never used).
template <int H>
__device__ __forceinline__ void gram_rows_loop(const char *const *colb, unsigned off, int n, d4 *acc)
{
    constexpr unsigned step = 2 * kGramRowsChunk * sizeof(double);   // to the wavefront's next chunk
    double2 b0[8], b1[8], b2[8], b3[8];
    auto at = [&](int j) { return off + (unsigned)min(j, n - 1) * step; };
    gram_rows_load(colb, at(0), b0);
    gram_rows_load(colb, at(1), b1);
    gram_rows_load(colb, at(2), b2);
    int j = 0;
    for (; j + 4 <= n; j += 4) {
        gram_rows_load(colb, at(j + 3), b3);
        gram_rows_chunk<H>(b0, acc);
        gram_rows_load(colb, at(j + 4), b0);
        gram_rows_chunk<H>(b1, acc);
        gram_rows_load(colb, at(j + 5), b1);
        gram_rows_chunk<H>(b2, acc);
        gram_rows_load(colb, at(j + 6), b2);
        gram_rows_chunk<H>(b3, acc);
    }
    const int rem = n - j;   // chunks j, j + 1, j + 2 are in b0, b1, b2
    if (rem > 0) gram_rows_chunk<H>(b0, acc);
    if (rem > 1) gram_rows_chunk<H>(b1, acc);
    if (rem > 2) gram_rows_chunk<H>(b2, acc);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_gram128_rows(
    const double *__restrict__ G, int m, long ldg, const int4 *__restrict__ piv, int rows_per_split,
    double *__restrict__ partial)
{
    constexpr int W = 128, NT = 8, NH = 18;
    __shared__ double red[2 * NH * 256];   // the tiles of wavefronts 2 and 3, element-major
    const int pv = blockIdx.x, split = blockIdx.y;
    const int4 d = piv[pv];
    const int lane = threadIdx.x & 63, g = lane / 16;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int half = wave & 1, c0 = wave >> 1;
    const int r_begin = split * rows_per_split;
    const int r_end = min(m, r_begin + rows_per_split);
    // block c: uniform first column (of block I for c < 4, of block J after)
    // at the split's first row; this lane's column lane % 16 of it and its
    // row pair in chunk c0 as a byte offset
    const char *colb[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c)
        colb[c] = (const char *)(G + (size_t)(c < 4 ? d.x + 16 * c : d.z + 16 * (c - 4)) * ldg + r_begin);
    const unsigned off = ((unsigned)(lane % 16) * (unsigned)ldg + (unsigned)(kGramRowsChunk * c0 + 2 * g)) *
                         (unsigned)sizeof(double);
    d4 acc[NH];
#pragma unroll
    for (int q = 0; q < NH; ++q) acc[q] = d4{0, 0, 0, 0};
    const int nchunks = (r_end - r_begin) / kGramRowsChunk;   // all full (8 | m, 8 | rows_per_split)
    const int n = (nchunks - c0 + 1) / 2;                     // chunks of this wavefront
    if (n > 0) {
        if (half == 0)
            gram_rows_loop<0>(colb, off, n, acc);
        else
            gram_rows_loop<1>(colb, off, n, acc);
    }
    // the second row half (wavefronts 2, 3) to LDS, added by the first (0, 1)
    double *rh = red + half * NH * 256;
    if (c0 == 1) {
#pragma unroll
        for (int q = 0; q < NH; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) rh[q * 256 + r * 64 + lane] = acc[q][r];
    }
    __syncthreads();
    if (c0 == 0) {
        double *out = partial + ((size_t)pv * gridDim.y + split) * W * W;
#pragma unroll
        for (int q = 0; q < NH; ++q) {
            const int t = NH * half + q;
            const int ti = upper_tile_i(NT, t), tj = upper_tile_j(NT, t);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = ti * 16 + Mfma<double>::row(lane, r), col = tj * 16 + lane % 16;
                out[(size_t)col * W + row] = acc[q][r] + rh[q * 256 + r * 64 + lane];
            }
        }
    }
}

// ----------------------------------------------------------- k_gram_reduce
// Adds the split-K partial Grams of every pivot in split order (the same
// order for every entry, so the sum is deterministic) and writes the full
// symmetric A_P (W x W, column-major) for the pivot solve.  The partials
// hold the upper 16 x 16 tiles (diagonal tiles whole); an entry of a lower
// tile is its transpose.  An empty pivot position (a block narrower than b)
// has a zero row and column, and gets 1 on the diagonal: an identity row and
// column of A_P.  Spread over the whole chip, so the pivot solve (one
// workgroup per pivot) copies a finished matrix instead of waiting on nsplit
// scattered loads per entry.
template <int W>
__global__ __launch_bounds__(256) void k_gram_reduce(const double *__restrict__ partial,
                                                     int nsplit, const int4 *__restrict__ piv,
                                                     int b, double *__restrict__ ap)
{
    const int pv = blockIdx.y;
    const int e = blockIdx.x * 256 + threadIdx.x;   // entry (r, c) of the upper storage
    if (e >= W * W) return;
    const int r = e % W, c = e / W;
    if ((r / 16) > (c / 16) || ((r / 16) == (c / 16) && r > c)) return;   // lower: written below
    const double *src = partial + (size_t)pv * nsplit * W * W + e;
    double v[8];
    double acc = 0.0;
    for (int s0 = 0; s0 < nsplit; s0 += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = (s0 + u < nsplit) ? src[(size_t)(s0 + u) * W * W] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (s0 + u < nsplit) acc += v[u];
    }
    if (r == c && !pivot_real(r, piv[pv], b)) acc = 1.0;
    double *out = ap + (size_t)pv * W * W;
    out[(size_t)c * W + r] = acc;
    out[(size_t)r * W + c] = acc;
}

// ---------------------------------------------------------- k_pivot_solve
// Inner orderings over the W = 2b columns of a pivot, in closed form (no
// table reads on the critical path of an inner step):
//   all pairs : the modified modulus ordering over W columns, W steps of
//               W/2 pairs (modulus_pair);
//   I x J     : the bipartite shift, b steps; step s holds (k, b + (k+s) mod b).
__device__ __forceinline__ int inner_steps(int all_pairs, int W) { return all_pairs ? W : W / 2; }
__device__ __forceinline__ int inner_step_pairs(int all_pairs, int W) { return W / 2; }
__device__ __forceinline__ int2 inner_pair(int all_pairs, int W, int s, int r)
{
    if (all_pairs) {
        int i, j;
        modulus_pair(W, s + 1, r, &i, &j);
        return make_int2(i, j);
    }
    const int b = W / 2;
    return make_int2(r, b + (r + s) % b);
}

// inner_pair with the ordering fixed at compile time (no branch on it in
// the step loops).
template <bool ALL>
__device__ __forceinline__ int2 inner_pair_t(int W, int s, int r)
{
    if constexpr (ALL) {
        int i, j;
        modulus_pair(W, s + 1, r, &i, &j);
        return make_int2(i, j);
    } else {
        const int b = W / 2;
        return make_int2(r, b + (r + s) % b);
    }
}

// Breakdown path: one inner sweep directly on the columns of G_P (len rows,
// pivot-local column k at X + pivot_col(k) * ldx), one wavefront per pair,
// lanes over rows; the transforms are accumulated in V_P (Y: W x W, pitch
// ldy), which is later applied to V only.  rot / ncl count on lane 0.
template <int NW>
__device__ void inner_sweep_global(double *X, long ldx, int len, double *Y, long ldy, int ylen,
                                   const signed char *JP, int all_pairs, int W, double tol,
                                   int4 d, int b, unsigned long long &rot,
                                   unsigned long long &ncl, int *bad)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nsteps = inner_steps(all_pairs, W), npairs = inner_step_pairs(all_pairs, W);
    for (int s = 0; s < nsteps; ++s) {
        for (int e = wave; e < npairs; e += NW) {
            const int2 pq = inner_pair(all_pairs, W, s, e);
            const int cp = pivot_col(pq.x, d, b), cq = pivot_col(pq.y, d, b);
            if (cp < 0 || cq < 0) continue;   // an empty position: nothing to rotate
            double *xp = X + (size_t)cp * ldx;
            double *xq = X + (size_t)cq * ldx;
            double app = 0.0, aqq = 0.0, apq = 0.0;
            for (int r = lane; r < len; r += 64) {
                const double x = xp[r], y = xq[r];
                app = fma(x, x, app);
                aqq = fma(y, y, aqq);
                apq = fma(x, y, apq);
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
                double x = xp[r], y = xq[r];
                rotate_elems(x, y, c, sn, same);
                xp[r] = x;
                xq[r] = y;
            }
            {
                double *yp = Y + (size_t)pq.x * ldy;
                double *yq = Y + (size_t)pq.y * ldy;
                for (int r = lane; r < ylen; r += 64) {
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

struct PivotSolveArgs {
    const double *ap;   // per pivot the W x W Gram A_P (column-major), from k_gram_reduce
    signed char *J;  // device signs (null: J = I); rewritten by the sign pivoting
    const int4 *piv;
    int b;
    double tol;
    int all_pairs, full_block, max_inner;
    double *vpt;  // per pivot W x W, V_P row-major
    int *flag;    // per pivot: 1 apply V_P to G and V, 2 to V only (G_P was
                  // transformed in place after a Cholesky breakdown), 0 none
    SweepCounters *ctr;
    // for the breakdown path: G itself
    double *G;
    int m;
    long ldg;
    int sign_pivot;  // Alg. 3.3 instead of the unpivoted Cholesky
    // W = 128: the inner transforms of each pivot, (c, s) per pair and step
    // (c negated for a hyperbolic transform; (1, 0): none), log_stride
    // entries per pivot
    double2 *vlog;
    long log_stride;
};

// LDS pitch of the factor R: one more than W (bank spread when the lanes of
// a wavefront read different columns at the same row).
template <int W>
constexpr int gram_pitch() { return W + 1; }

// Workgroup of the pivot solve: 4 wavefronts; the inner sweeps run as
// ring_sweep (each pair on 8 or 16 lanes of one wavefront).
constexpr int kPivotThreads = 256;

// Sum over groups of L consecutive lanes (L = 8 or 16); every lane of a
// group ends with the group's total (lane ^ 1, lane ^ 2, then the mirrors
// within 8 and 16 lanes, each pairing a lane with one of the other half).
template <int L>
__device__ __forceinline__ void group_sum3_all(double &x, double &y, double &z)
{
    static_assert(L == 8 || L == 16, "DPP groups of 8 or 16 lanes");
    x += dpp_move<0xB1>(x);
    y += dpp_move<0xB1>(y);
    z += dpp_move<0xB1>(z);
    x += dpp_move<0x4E>(x);
    y += dpp_move<0x4E>(y);
    z += dpp_move<0x4E>(z);
    x += dpp_move<0x141>(x);
    y += dpp_move<0x141>(y);
    z += dpp_move<0x141>(z);
    if constexpr (L == 16) {
        x += dpp_move<0x140>(x);
        y += dpp_move<0x140>(y);
        z += dpp_move<0x140>(z);
    }
}

// The products x_i y_i of RL rows added as a pairwise tree (t_i += t_{i+h},
// h = RL/2, ..., 1), rounded at every operation (no contraction), so that
// ring_converged forms bit for bit the sums of a ring_sweep step.
template <int RL>
__device__ __forceinline__ double lane_dot(const double (&x)[RL], const double (&y)[RL])
{
    double t[RL];
#pragma unroll
    for (int i = 0; i < RL; ++i) t[i] = __dmul_rn(x[i], y[i]);
#pragma unroll
    for (int h = RL / 2; h > 0; h /= 2)
#pragma unroll
        for (int i = 0; i < h; ++i) t[i] = __dadd_rn(t[i], t[i + h]);
    return t[0];
}

// One inner sweep over the W columns of R (A) and V_P (VP), both in LDS at
// pitch gram_pitch<W>, for W = 32 or 64 in the kPivotThreads workgroup.
// The W/2 pairs of a step go to W/2 processes, PPW per wavefront, L lanes a
// process; lane l of a process holds rows l, l + L, ... of the pair's two
// columns of R and of V_P in registers.  From one step to the next a
// process keeps one of its columns: in the ring of Alg. 3.1 (all pairs: the
// modified modulus steps, process k starting on (k, W - 1 - k) and moving
// by the process map) and in the bipartite shift (process k: column k of
// block I, the J column moving on).  Only the column it gives up goes
// through LDS: written after the step, read by the process that takes it
// after the barrier, so a step moves half the columns and has one barrier.
// The kept column stays in K (id ck), the received one in N (id cn); the
// pair is (min, max) of the two ids.  On entry and exit every column is in
// LDS.  Returns the rotations of the sweep counted once per pair (on lane 0
// of each process).
template <int W, bool ALL>
__device__ __forceinline__ unsigned long long ring_sweep(double *A, double *VP,
                                                         const signed char *JI, double tol,
                                                         unsigned long long &ncl, int &bad)
{
    constexpr int P = gram_pitch<W>(), NW = kPivotThreads / 64, NP = W / 2;
    constexpr int PPW = NP / NW, L = 64 / PPW, RL = W / L;
    static_assert(PPW * NW == NP && L * RL == W, "pairs dealt evenly");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int k = wave * PPW + lane / L, lg = lane % L;
    const int nsteps = inner_steps(ALL, W);
    // ring state in the 1-based terms of the process map
    int ra = k + 1, rc = W - k;
    int ck = k, cn = ALL ? W - 1 - k : NP + k;
    double K[RL], N[RL], VK[RL], VN[RL];
#pragma unroll
    for (int i = 0; i < RL; ++i) {
        K[i] = A[ck * P + lg + L * i];
        N[i] = A[cn * P + lg + L * i];
        VK[i] = VP[ck * P + lg + L * i];
        VN[i] = VP[cn * P + lg + L * i];
    }
    unsigned long long rot = 0;
    for (int s = 0; s < nsteps; ++s) {
        const bool kx = ck < cn;   // K holds the pair's first column
        // this lane's products added as a pairwise tree (rounding grows with
        // log2(RL), not RL), then over the lanes of the process
        double skk = lane_dot<RL>(K, K), snn = lane_dot<RL>(N, N), skn = lane_dot<RL>(K, N);
        group_sum3_all<L>(skk, snn, skn);
        const double app = kx ? skk : snn, aqq = kx ? snn : skk, apq = skn;
        const int p = kx ? ck : cn, q = kx ? cn : ck;
        bool act = false;
        if (!finite3(app, aqq, apq))
            bad = 1;
        else
            act = needs_rotation(app, aqq, apq, tol);
        if (act) {
            // pairs of both signs may share the wavefront (sign pivoting)
            const bool same = JI[p] == JI[q];
            double c, sn;
            const bool cl = transform_params_bf(app, aqq, apq, same, c, sn);
            // rotate_elems on (x, y) = (K, N) or (N, K): K' = c K + al N,
            // N' = c N + be K
            const double al = same ? (kx ? -sn : sn) : sn;
            const double be = same ? -al : sn;
#pragma unroll
            for (int i = 0; i < RL; ++i) {
                const double k0 = K[i], n0 = N[i], vk0 = VK[i], vn0 = VN[i];
                K[i] = c * k0 + al * n0;
                N[i] = c * n0 + be * k0;
                VK[i] = c * vk0 + al * vn0;
                VN[i] = c * vn0 + be * vk0;
            }
            if (lg == 0) {
                ++rot;
                ncl += cl ? 1 : 0;
            }
        }
        if (s + 1 == nsteps) break;
        // the next pair of this process, the column it keeps and the one it
        // receives
        int pn, qn;
        if constexpr (ALL) {
            // moving down the first column becomes a (after the diagonal:
            // the row no other process holds); walking right the second c
            if (ra + rc > W) {
                ++ra;
                if (ra == rc) {
                    ra -= NP;
                    rc = ra;
                }
                pn = ra - 1;
                qn = q;
            } else {
                ++rc;
                pn = p;
                qn = rc - 1;
            }
        } else {
            pn = k;
            qn = NP + (k + s + 1) % NP;
        }
        if (ck != pn && ck != qn) {
            // N is the column kept: swap the roles
#pragma unroll
            for (int i = 0; i < RL; ++i) {
                const double t = K[i], vt = VK[i];
                K[i] = N[i];
                VK[i] = VN[i];
                N[i] = t;
                VN[i] = vt;
            }
            const int t = ck;
            ck = cn;
            cn = t;
        }
#pragma unroll
        for (int i = 0; i < RL; ++i) {
            A[cn * P + lg + L * i] = N[i];
            VP[cn * P + lg + L * i] = VN[i];
        }
        cn = (pn == ck) ? qn : pn;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RL; ++i) {
            N[i] = A[cn * P + lg + L * i];
            VN[i] = VP[cn * P + lg + L * i];
        }
    }
#pragma unroll
    for (int i = 0; i < RL; ++i) {
        A[ck * P + lg + L * i] = K[i];
        A[cn * P + lg + L * i] = N[i];
        VP[ck * P + lg + L * i] = VK[i];
        VP[cn * P + lg + L * i] = VN[i];
    }
    __syncthreads();
    return rot;
}

// Whether an inner sweep run now would rotate nothing (full block: the
// sweep that ends a pivot's inner iteration).  While no pair rotates the
// columns do not change, so that sweep rotates nothing exactly when no pair
// passes the threshold with the columns as they are; this tests all W (W-1)
// / 2 pairs at once, one thread per pair, with the sums of a ring_sweep
// step formed in the same order: lane l of a process (L lanes) holds rows l,
// l + L, ... and adds its products by lane_dot; the DPP butterfly of
// group_sum3_all then gives every lane the balanced tree over the lanes in
// order, ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7)) (and the same for
// lanes 8..15 added to it when L = 16), since a + b == b + a exactly.
// Returns false as well when a sum is not finite (the sweep reports it).
// Called by the whole workgroup; flag is a shared int.
template <int W>
__device__ bool ring_converged(const double *A, double tol, int *flag)
{
    constexpr int P = gram_pitch<W>(), NW = kPivotThreads / 64, NP = W / 2;
    constexpr int PPW = NP / NW, L = 64 / PPW, RL = W / L;
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < W * (W - 1) / 2; e += kPivotThreads) {
        // pair e -> (p, q), p < q, by rows of the strict upper triangle
        int p = 0, rem = e;
        while (rem >= W - 1 - p) {
            rem -= W - 1 - p;
            ++p;
        }
        const int q = p + 1 + rem;
        const double *cp = A + p * P, *cq = A + q * P;
        double xpp[L], xqq[L], xpq[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            double vp[RL], vq[RL];
#pragma unroll
            for (int i = 0; i < RL; ++i) {
                vp[i] = cp[l + L * i];
                vq[i] = cq[l + L * i];
            }
            xpp[l] = lane_dot<RL>(vp, vp);
            xqq[l] = lane_dot<RL>(vq, vq);
            xpq[l] = lane_dot<RL>(vp, vq);
        }
#pragma unroll
        for (int h = 1; h < L; h *= 2)
#pragma unroll
            for (int l = 0; l < L; l += 2 * h) {
                xpp[l] = __dadd_rn(xpp[l], xpp[l + h]);
                xqq[l] = __dadd_rn(xqq[l], xqq[l + h]);
                xpq[l] = __dadd_rn(xpq[l], xpq[l + h]);
            }
        const double app = xpp[0], aqq = xqq[0], apq = xpq[0];
        if (!finite3(app, aqq, apq) || needs_rotation(app, aqq, apq, tol)) *flag = 1;
    }
    __syncthreads();
    const bool conv = *flag == 0;
    __syncthreads();
    return conv;
}

template <int W>
__global__ __launch_bounds__(kPivotThreads) void k_pivot_solve(PivotSolveArgs a)
{
    constexpr int NW = kPivotThreads / 64;
    constexpr int P = gram_pitch<W>();
    extern __shared__ double lds[];
    double *A = lds;                   // W x W column-major, pitch P: Gram, then R
    double *VP = lds + W * P;          // W x W column-major, pitch P (first: rows of R)
    __shared__ signed char JP[W], JS[W];
    __shared__ int s_piv[W], s_perm[W];
    __shared__ int s_need, s_bad, s_npos, s_conv;
    __shared__ unsigned long long s_rot[NW], s_cl[NW];
    const int pv = blockIdx.x;
    const int4 d = a.piv[pv];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b = a.b;

    if (tid < W) {
        const int c = pivot_col(tid, d, b);
        JP[tid] = (a.J && c >= 0) ? a.J[c] : (signed char)1;
    }
    if (tid == 0) {
        s_need = 0;
        s_bad = 0;
    }
    // A_P, added up over the splits by k_gram_reduce
    {
        const double *src = a.ap + (size_t)pv * W * W;
        constexpr int PER = W * W / kPivotThreads;
        double v[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) v[q] = src[tid + q * kPivotThreads];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * kPivotThreads;
            A[(e / W) * P + (e % W)] = v[q];
        }
    }
    __syncthreads();
    // skip test on the targeted off-diagonal entries; finiteness of all
    for (int e = tid; e < W * W; e += kPivotThreads) {
        const int r = e % W, c = e / W;
        const double x = A[c * P + r];
        if (!isfinite(x)) s_bad = 1;
        if (r < c && (a.all_pairs || (r < b && c >= b))) {
            const double arr = A[r * P + r], acc2 = A[c * P + c];
            if (arr != 0.0 && acc2 != 0.0 && fabs(x) > a.tol * sqrt(arr) * sqrt(acc2)) s_need = 1;
        }
    }
    __syncthreads();
    if (s_bad) {
        if (tid == 0) {
            a.ctr->nonfinite = 1u;
            a.flag[pv] = 0;
        }
        return;
    }
    if (!s_need) {
        if (tid == 0) a.flag[pv] = 0;
        return;
    }
    // Cholesky A_P = R^T R, right-looking: step j writes row j of R
    // (r_jl = a_jl / r_jj) into the VP buffer, then, after a barrier,
    // subtracts r_ji r_jl from the trailing entries (i, l), j < i <= l.
    // A breakdown is seen by every thread at once: the pivot d is read from
    // LDS after a barrier, so each thread records it in its own register and
    // all leave the loop at the same step.
    bool broke = false;
    if (!a.sign_pivot) {
        for (int j = 0; j < W; ++j) {
            const double d = A[j * P + j];
            if (!(d > 0.0)) {
                broke = true;
                break;  // d is the same for every thread: a uniform exit
            }
            const double rjj = sqrt(d);
            for (int l = j + tid; l < W; l += kPivotThreads)
                VP[l * P + j] = (l == j) ? rjj : A[l * P + j] / rjj;
            __syncthreads();
            // trailing update over a 16 x 16 thread grid (no integer
            // division on the per-element path)
            for (int l = j + 1 + (tid >> 4); l < W; l += kPivotThreads / 16) {
                const double rl = VP[l * P + j];
                for (int i = j + 1 + (tid & 15); i <= l; i += 16) A[l * P + i] -= VP[i * P + j] * rl;
            }
            __syncthreads();
        }
    } else {
        // Sign-pivoted Cholesky (Alg. 3.3) as one right-looking elimination
        // over the positions of A_P reordered positive-first: eliminating
        // positions 0..npos-1 with the pivot taken among them factors A_11
        // with diagonal pivoting, forms R_12 = R_11^{-T} P_1^T A_12 in the
        // same rows of R and leaves the Schur complement S = A_22 - R_12^T
        // R_12 in the trailing block, which the remaining steps factor with
        // pivots among positions npos..W-1 ((3.6), (3.7)).  piv maps a
        // position to its column of A_P (rows and columns are not moved);
        // both triangles of A are kept.  At step j the pivot is the largest
        // remaining diagonal entry in the position's sign block (the first
        // on ties); swapping positions j and t also swaps columns j and t of
        // the rows of R formed so far.
        if (wave == 0) {
            const bool in = lane < W;
            const bool isp = in && JP[lane] > 0;
            const unsigned long long bp = __ballot(isp), bn = __ballot(in && !isp);
            const int np = __popcll(bp);
            const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
            if (in) s_piv[isp ? __popcll(bp & below) : np + __popcll(bn & below)] = lane;
            if (lane == 0) s_npos = np;
        }
        __syncthreads();
        const int npos = s_npos;
        for (int j = 0; j < W; ++j) {
            const int hi = (j < npos) ? npos : W;
            if (wave == 0) {
                // the largest remaining diagonal entry: DPP max within rows of
                // 16 lanes, then across the four rows; the first lane holding
                // it gives the position (the entries are finite here)
                const int i = j + lane;
                const double v = (i < hi) ? A[s_piv[i] * P + s_piv[i]] : -1.0;
                double mx = v;
                mx = fmax(mx, dpp_move<0xB1>(mx));
                mx = fmax(mx, dpp_move<0x4E>(mx));
                mx = fmax(mx, dpp_move<0x141>(mx));
                mx = fmax(mx, dpp_move<0x140>(mx));
                mx = fmax(fmax(read_lane(mx, 0), read_lane(mx, 16)),
                          fmax(read_lane(mx, 32), read_lane(mx, 48)));
                const unsigned long long hit = __ballot(i < hi && v == mx);
                const int t = hit ? j + __ffsll((long long)hit) - 1 : W;   // the same in every lane
                if (t != j && t < W) {
                    if (lane < j) {
                        const double x = VP[j * P + lane];
                        VP[j * P + lane] = VP[t * P + lane];
                        VP[t * P + lane] = x;
                    }
                    if (lane == 0) {
                        const int x = s_piv[j];
                        s_piv[j] = s_piv[t];
                        s_piv[t] = x;
                    }
                }
            }
            __syncthreads();
            const int pj = s_piv[j];
            const double d = A[pj * P + pj];
            if (!(d > 0.0)) {
                broke = true;
                break;  // uniform exit
            }
            const double rjj = sqrt(d);
            for (int l = j + tid; l < W; l += kPivotThreads)
                VP[l * P + j] = (l == j) ? rjj : A[s_piv[l] * P + pj] / rjj;
            __syncthreads();
            for (int l = j + 1 + (tid >> 4); l < W; l += kPivotThreads / 16) {
                const double rl = VP[l * P + j];
                const int pl = s_piv[l];
                for (int i = j + 1 + (tid & 15); i < W; i += 16)
                    A[pl * P + s_piv[i]] -= VP[i * P + j] * rl;
            }
            __syncthreads();
        }
    }
    if (broke && !a.G) {
        // no FP64 copy of G to transform in place (the FP32 sweeps): the
        // pivot is left to the FP64 sweeps that follow
        if (tid == 0) {
            atomicAdd(&a.ctr->breakdowns, 1ull);
            a.flag[pv] = 0;
        }
        return;
    }
    unsigned long long rot = 0, ncl = 0;
    int bad = 0;
    if (!broke) {
        // R (upper) from the VP buffer into A; with sign pivoting the
        // columns of the negative block are reversed (Alg. 3.3) and
        // position c takes the sign +1 for c < npos, else -1
        const int npos = a.sign_pivot ? s_npos : W;
        for (int e = tid; e < W * W; e += kPivotThreads) {
            const int r = e % W, c = e / W;
            const int src = (c < npos) ? c : npos + (W - 1 - c);
            A[c * P + r] = (r <= src) ? VP[src * P + r] : 0.0;
        }
        if (a.sign_pivot && tid < W) {
            const int src = (tid < npos) ? tid : npos + (W - 1 - tid);
            s_perm[tid] = s_piv[src];
            JS[tid] = (tid < npos) ? (signed char)1 : (signed char)-1;
        }
        __syncthreads();
    }
    // signs of the inner transforms: of the permuted positions after a
    // sign-pivoted factorisation, else of the pivot's own columns
    const signed char *JI = (a.sign_pivot && !broke) ? JS : JP;
    for (int e = tid; e < W * W; e += kPivotThreads) {   // V_P := I
        const int r = e % W, c = e / W;
        VP[c * P + r] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int sweeps = a.full_block ? a.max_inner : 1;
    for (int it = 0; it < sweeps; ++it) {
        unsigned long long rot_it = 0;
        if (!broke) {
            rot_it = a.all_pairs ? ring_sweep<W, true>(A, VP, JI, a.tol, ncl, bad)
                                 : ring_sweep<W, false>(A, VP, JI, a.tol, ncl, bad);
        } else {
            // G_P is transformed in place; V_P collects the transforms for V
            inner_sweep_global<NW>(a.G, a.ldg, a.m, VP, P, W, JP, a.all_pairs, W, a.tol, d, b,
                                   rot_it, ncl, &bad);
        }
        rot += rot_it;
        // rotations of this inner sweep, summed over the workgroup
        const double dr = (double)rot_it;
        const double wr = wave_sum(dr);
        if (lane == 0) s_rot[wave] = (unsigned long long)wr;
        __syncthreads();
        unsigned long long tot = 0;
        for (int w = 0; w < NW; ++w) tot += s_rot[w];
        __syncthreads();
        if (tot == 0) break;
        // after a sweep with few rotations the next one usually rotates
        // nothing: test that at once instead of running it
        if (!broke && it + 1 < sweeps && tot <= W && ring_converged<W>(A, a.tol, &s_conv)) break;
    }
    {
        const double wr = wave_sum((double)rot), wc = wave_sum((double)ncl);
        if (lane == 0) {
            s_rot[wave] = (unsigned long long)wr;
            s_cl[wave] = (unsigned long long)wc;
        }
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
        if (s_bad) a.ctr->nonfinite = 1u;
        a.flag[pv] = (tot > 0 && !s_bad) ? (broke ? 2 : 1) : 0;
    }
    if (tot > 0) {
        // V_P row-major; after a sign-pivoted factorisation V_P = P V' (the
        // permutation applied to the rows of V', Alg. 3.4), and column c of
        // the pivot block takes the sign of position c
        const bool sp = a.sign_pivot && !broke;
        double *out = a.vpt + (size_t)pv * W * W;
        for (int e = tid; e < W * W; e += kPivotThreads) {
            const int r = e / W, c = e % W;
            out[(sp ? s_perm[r] : r) * W + c] = VP[c * P + r];
        }
        if (sp && a.J && !s_bad && tid < W && pivot_real(tid, d, b)) a.J[pivot_col(tid, d, b)] = JS[tid];
    }
}

// ------------------------------------------------ k_pivot_solve_log (W = 128)
// The pivot solve for W = 128 (b = 64).  R (W x W, pitch W + 1) alone fills
// 129 KiB of the LDS, so V_P is not kept beside it: the inner steps log
// their transforms (one 16-byte entry per pair and step, in global memory),
// and when the inner sweeps are done the LDS of R holds V_P (row-major),
// which the log is replayed on, one thread per row: every row of V_P
// receives the column transforms in the order they were applied to R, with
// the same arithmetic (rotate_elems).  The Cholesky factorisation runs in
// place in the upper triangle of A (the diagonal keeps the pivot d_j until
// the end, when it becomes sqrt(d_j)).  In an inner step lane k of every
// wavefront owns pair k (W/2 = 64 pairs) and wavefront w rows
// [w W/4, (w+1) W/4) of it; the partial dot products meet in LDS as in
// k_pivot_solve.  Unpivoted Cholesky only (the sign pivoting of Alg. 3.3
// runs at W <= 64).  After a breakdown V_P is accumulated in LDS directly
// while the inner sweeps run on G_P (R is not needed then).
// One inner step's transform of pair `lane` in the W = 128 pivot solves:
// the dot products of its columns over this wavefront's RPW rows (xr, yr),
// as pairwise subtrees of RB rows and a pairwise tree over the subtrees,
// meet the other NW - 1 wavefronts' in LDS (red; one barrier) and are added
// pairwise in wavefront order ((w0 + w1) + (w2 + w3) for NW = 4) in every
// wavefront, so all get the same totals.  Returns whether the pair rotates;
// c, sn, and same (trigonometric) then hold the transform (else c = 1,
// sn = 0).
// RB = 0: the rows are summed in four interleaved chains (rows r mod 4),
// added pairwise, which holds 12 partial sums where the subtrees hold 36.
template <int RPW, int RB, int NW, int NP>
__device__ __forceinline__ bool pair_transform(const double *xr, const double *yr, double *red,
                                               int wave, int lane, double tol, bool same_sign,
                                               double &c, double &sn, bool &same, int &bad,
                                               bool &clamped)
{
    constexpr int NG = RB > 0 ? RPW / RB : 1;
    double pxx[NG], pyy[NG], pxy[NG];
    if constexpr (RB == 0) {
        double axx[4], ayy[4], axy[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            axx[k] = xr[k] * xr[k];
            ayy[k] = yr[k] * yr[k];
            axy[k] = xr[k] * yr[k];
        }
#pragma unroll
        for (int r = 4; r < RPW; ++r) {
            axx[r % 4] = fma(xr[r], xr[r], axx[r % 4]);
            ayy[r % 4] = fma(yr[r], yr[r], ayy[r % 4]);
            axy[r % 4] = fma(xr[r], yr[r], axy[r % 4]);
        }
        pxx[0] = (axx[0] + axx[1]) + (axx[2] + axx[3]);
        pyy[0] = (ayy[0] + ayy[1]) + (ayy[2] + ayy[3]);
        pxy[0] = (axy[0] + axy[1]) + (axy[2] + axy[3]);
    }
#pragma unroll
    for (int g = 0; g < (RB > 0 ? RPW / RB : 0); ++g) {
        constexpr int RS = RB > 0 ? RB : 1;
        double sxx[RS], syy[RS], sxy[RS];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const double x = xr[g * RB + r], y = yr[g * RB + r];
            sxx[r] = x * x;
            syy[r] = y * y;
            sxy[r] = x * y;
        }
#pragma unroll
        for (int h = RB / 2; h > 0; h /= 2)
#pragma unroll
            for (int r = 0; r < h; ++r) {
                sxx[r] += sxx[r + h];
                syy[r] += syy[r + h];
                sxy[r] += sxy[r + h];
            }
        pxx[g] = sxx[0];
        pyy[g] = syy[0];
        pxy[g] = sxy[0];
    }
#pragma unroll
    for (int h = NG / 2; h > 0; h /= 2)
#pragma unroll
        for (int g = 0; g < h; ++g) {
            pxx[g] += pxx[g + h];
            pyy[g] += pyy[g + h];
            pxy[g] += pxy[g + h];
        }
    red[(wave * 3 + 0) * NP + lane] = pxx[0];
    red[(wave * 3 + 1) * NP + lane] = pyy[0];
    red[(wave * 3 + 2) * NP + lane] = pxy[0];
    __syncthreads();
    double t[3][NW];
#pragma unroll
    for (int w = 0; w < NW; ++w)
#pragma unroll
        for (int k = 0; k < 3; ++k) t[k][w] = red[(w * 3 + k) * NP + lane];
#pragma unroll
    for (int h = 1; h < NW; h *= 2)
#pragma unroll
        for (int w = 0; w < NW; w += 2 * h)
#pragma unroll
            for (int k = 0; k < 3; ++k) t[k][w] += t[k][w + h];
    const double app = t[0][0], aqq = t[1][0], apq = t[2][0];
    bool act = true;
    if (!finite3(app, aqq, apq)) {
        bad = 1;
        act = false;
    }
    act = act && needs_rotation(app, aqq, apq, tol);
    same = act ? same_sign : true;
    c = 1.0;
    sn = 0.0;
    clamped = act && transform_params(app, aqq, apq, same, c, sn);
    return act;
}

// A_P (column-major W x W, from k_gram_reduce) into LDS with pitch W + 1:
// thread tid takes the entries tid + q NT, up to 32 loads in flight.
template <int W, int NT>
__device__ __forceinline__ void pivot_load_gram(const double *__restrict__ src, double *A, int tid)
{
    constexpr int P = W + 1;
    constexpr int PER = W * W / NT;
    constexpr int BATCH = PER < 32 ? PER : 32;
    static_assert(PER % BATCH == 0, "whole batches");
#pragma unroll
    for (int h = 0; h < PER / BATCH; ++h) {
        double v[BATCH];
#pragma unroll
        for (int q = 0; q < BATCH; ++q) v[q] = src[tid + (h * BATCH + q) * NT];
#pragma unroll
        for (int q = 0; q < BATCH; ++q) {
            const int e = tid + (h * BATCH + q) * NT;
            A[(e / W) * P + (e % W)] = v[q];
        }
    }
}

// The skip test of a pivot, before the factorisation: need = some pair
// (r, c), r < c, of the inner ordering (all pairs, or block I x block J)
// has both columns nonzero and |a_rc| > tol sqrt(a_rr) sqrt(a_cc) (dsh holds
// the square roots of the diagonal); bad = some entry is not finite.  Thread
// tid checks row tid mod W at the columns tid / W + q NT / W, without
// branches.
template <int W, int NT>
__device__ __forceinline__ void pivot_skip_test(const double *A, const double *dsh, int b,
                                                bool all_pairs, double tol, int tid, bool &need,
                                                bool &bad)
{
    constexpr int P = W + 1;
    static_assert(NT % W == 0, "one row per thread");
    const int r = tid % W;
    const double dr = dsh[r];
    int nd = 0, bd = 0;
#pragma unroll 8
    for (int q = 0; q < W * W / NT; ++q) {
        const int c = tid / W + q * (NT / W);
        const double x = A[c * P + r];
        const double dc = dsh[c];
        bd |= !isfinite(x);
        const int pair = (r < c) & (all_pairs | ((r < b) & (c >= b)));
        nd |= pair & (dr != 0.0) & (dc != 0.0) & (fabs(x) > tol * dr * dc);
    }
    need = nd != 0;
    bad = bd != 0;
}

// Unpivoted Cholesky A_P = R^T R in place (R in the upper triangle of A,
// pitch W + 1), blocked right-looking with panels of NB rows.  Wavefront 0
// factors a panel: rows j0 .. j0 + NB - 1 of R at columns l0 = j0 + lane and
// l1 = j0 + 64 + lane (clamped to W - 1: a clamped lane repeats the work of
// the lane that owns column W - 1) stay in registers; the entry (j, j) and
// the row-j entries r_ju of the columns of later panel rows come from the
// lanes that hold them (readlane), so the column loop makes no LDS access.
// Every update is applied to all columns: below the diagonal (l < row) the
// values are junk that the factorisation never reads (the caller zeroes the
// strict lower triangle).  Then all threads subtract the panel's r_ji r_jl
// (j in the panel, in order) from the trailing entries (i, l),
// j0 + NB <= i <= l, in 4 x 4 blocks (each panel value loaded serves four
// products; the blocks on the diagonal also write junk below it).  The
// pivots d_j go to dsh (R's diagonal is sqrt(d_j)).  Wavefront 0 reports a
// breakdown (d_j <= 0 or not a number) in *s_brk (zero on entry), which
// every thread reads after the barrier: the result is the same everywhere.
template <int W, int NT>
__device__ bool pivot_cholesky(double *A, double *dsh, int *s_brk, int tid)
{
    constexpr int P = W + 1;
    constexpr int NB = 16;
    static_assert(W % NB == 0 && W <= 128, "two columns per lane");
    const int lane = tid & 63, wave = tid >> 6;
    for (int j0 = 0; j0 < W; j0 += NB) {
        if (wave == 0) {
            const int l0 = min(j0 + lane, W - 1), l1 = min(j0 + 64 + lane, W - 1);
            double p0[NB], p1[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                p0[u] = A[l0 * P + j0 + u];
                p1[u] = A[l1 * P + j0 + u];
            }
            bool brk = false;
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) {
                const int j = j0 + jj;
                const double dj = read_lane(p0[jj], jj);   // lane jj holds column j
                // a breakdown (the same in every lane) voids the whole pivot:
                // the panel runs on (on junk) so that the loop stays unrolled
                brk = brk || !(dj > 0.0);
                const double rinv = 1.0 / sqrt(dj);
                if (lane == 0) dsh[j] = dj;
                // row j of R at this lane's columns l > j (l = j keeps d_j)
                const double s0 = p0[jj] * rinv, s1 = p1[jj] * rinv;
                p0[jj] = (l0 > j) ? s0 : p0[jj];
                p1[jj] = (l1 > j) ? s1 : p1[jj];
                // the later rows of the panel: a_ul -= r_ju r_jl
#pragma unroll
                for (int u = jj + 1; u < NB; ++u) {
                    const double rju = read_lane(p0[jj], u);   // lane u holds column j0 + u
                    p0[u] -= rju * p0[jj];
                    p1[u] -= rju * p1[jj];
                }
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                A[l0 * P + j0 + u] = p0[u];
                A[l1 * P + j0 + u] = p1[u];
            }
            if (brk && lane == 0) *s_brk = 1;
        }
        __syncthreads();
        if (*s_brk) return true;
        const int t0 = j0 + NB;
        const int nb4 = (W - t0) / 4;
        for (int t = tid; t < nb4 * nb4; t += NT) {
            const int bi = t % nb4, bl = t / nb4;
            if (bi > bl) continue;
            const int i0 = t0 + 4 * bi, c0 = t0 + 4 * bl;
            double acc[4][4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[q][e] = A[(c0 + e) * P + i0 + q];
#pragma unroll
            for (int u0 = 0; u0 < NB; u0 += 4) {
                double pi[4][4], pl[4][4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        pi[q][k] = A[(i0 + q) * P + j0 + u0 + k];
                        pl[q][k] = A[(c0 + q) * P + j0 + u0 + k];
                    }
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[q][e] -= pi[q][k] * pl[e][k];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) A[(c0 + e) * P + i0 + q] = acc[q][e];
        }
        __syncthreads();
    }
    return false;
}

constexpr int kLogThreads = 256;

template <int W>
__global__ __launch_bounds__(kLogThreads) void k_pivot_solve_log(PivotSolveArgs a)
{
    constexpr int NW = kLogThreads / 64;
    constexpr int P = W + 1;
    constexpr int NP = W / 2;          // pairs per inner step: lane k owns pair k
    constexpr int RPW = W / NW;        // rows of R per wavefront
    constexpr int RB = 8;              // rows summed as one pairwise subtree
    static_assert(NP == 64 && RPW % RB == 0, "one lane per pair");
    __shared__ double A[W * P];        // Gram, then R (upper), then V_P
    __shared__ double red[NW * 3 * NP];  // partial dots; in the replay, staged log entries
    __shared__ double dsh[W];          // Cholesky pivots d_j
    __shared__ signed char JP[W];
    __shared__ int s_need, s_bad, s_brk;
    __shared__ unsigned long long s_rot[NW], s_cl[NW];
    const int pv = blockIdx.x;
    const int4 d = a.piv[pv];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b = a.b;

    if (tid < W) {
        const int c = pivot_col(tid, d, b);
        JP[tid] = (a.J && c >= 0) ? a.J[c] : (signed char)1;
    }
    if (tid == 0) {
        s_need = 0;
        s_bad = 0;
        s_brk = 0;
    }
    // A_P, added up over the splits by k_gram_reduce
    pivot_load_gram<W, kLogThreads>(a.ap + (size_t)pv * W * W, A, tid);
    __syncthreads();
    // skip test; the square roots of the diagonal are taken once
    if (tid < W) dsh[tid] = sqrt(A[tid * P + tid]);
    __syncthreads();
    {
        bool need, bad_entry;
        pivot_skip_test<W, kLogThreads>(A, dsh, b, a.all_pairs != 0, a.tol, tid, need, bad_entry);
        if (need) s_need = 1;
        if (bad_entry) s_bad = 1;
    }
    __syncthreads();
    if (s_bad) {
        if (tid == 0) {
            a.ctr->nonfinite = 1u;
            a.flag[pv] = 0;
        }
        return;
    }
    if (!s_need) {
        if (tid == 0) a.flag[pv] = 0;
        return;
    }
    const bool broke = pivot_cholesky<W, kLogThreads>(A, dsh, &s_brk, tid);
    if (broke && !a.G) {
        // no FP64 copy of G to transform in place (the FP32 sweeps): the
        // pivot is left to the FP64 sweeps that follow
        if (tid == 0) {
            atomicAdd(&a.ctr->breakdowns, 1ull);
            a.flag[pv] = 0;
        }
        return;
    }
    unsigned long long rot = 0, ncl = 0;
    int bad = 0;
    const int sweeps = a.full_block ? a.max_inner : 1;
    double2 *log = a.vlog + (size_t)pv * a.log_stride;
    int logged = 0;       // inner sweeps in the log
    int vp_layout = 1;    // V_P in A: 0 row-major, 1 column-major, 2 column-major with
                          // the two halves of the columns swapped
    if (!broke) {
        // R: the diagonal becomes sqrt(d_j), the strict lower triangle zero
        for (int e = tid; e < W * W; e += kLogThreads) {
            const int r = e % W, c = e / W;
            if (r == c) A[c * P + r] = sqrt(dsh[c]);
            else if (r > c) A[c * P + r] = 0.0;
        }
        __syncthreads();
        // The inner sweeps, with the inner ordering fixed at compile time.
        //   I x J pairs (block-oriented after the first step of a sweep):
        //     lane k pairs column k of block I with column (k + s) mod b of
        //     block J at step s, so R's and V_P's block-I columns stay in
        //     registers for the whole sweep; V_P's block-J columns take the
        //     LDS of R's block-I columns, and both are rotated in the step.
        //   all pairs (the first step of a sweep, and full block): both
        //     columns of a pair change every step; the steps log their
        //     transforms, and V_P is formed from the log afterwards in the
        //     LDS of R (it does not fit beside it).
        auto sweeps_and_replay = [&](auto all_c) {
            constexpr bool ALL = decltype(all_c)::value;
            const int nsteps = inner_steps(ALL, W);
            const int r0 = wave * RPW;
            if constexpr (!ALL) {
                constexpr int HB = W / 2;
                double xr[RPW], vx[RPW];
#pragma unroll
                for (int r = 0; r < RPW; ++r) xr[r] = A[lane * P + r0 + r];
                __syncthreads();   // R's block-I columns are read before the LDS takes V_J
                // V_J (block-J columns of V_P := I) at the slots of R's
                // block-I columns: slot c holds column b + c
                for (int e = tid; e < HB * W; e += kLogThreads) {
                    const int r = e % W, c = e / W;
                    A[c * P + r] = (r == HB + c) ? 1.0 : 0.0;
                }
#pragma unroll
                for (int r = 0; r < RPW; ++r) vx[r] = (r0 + r == lane) ? 1.0 : 0.0;
                __syncthreads();
                unsigned long long rot_it = 0;
                for (int s = 0; s < nsteps; ++s) {
                    const int cj = (lane + s) % HB;   // the block-J column of the pair
                    double *yq = A + (HB + cj) * P + r0, *vq = A + cj * P + r0;
                    double yr[RPW], vy[RPW];
#pragma unroll
                    for (int r = 0; r < RPW; ++r) {
                        yr[r] = yq[r];
                        vy[r] = vq[r];
                    }
                    double c, sn;
                    bool same, cl;
                    const bool act = pair_transform<RPW, RB, NW, NP>(
                        xr, yr, red, wave, lane, a.tol, JP[lane] == JP[HB + cj], c, sn, same, bad, cl);
                    if (cl && wave == 0) ++ncl;
                    if (act) {
#pragma unroll
                        for (int r = 0; r < RPW; ++r) {
                            rotate_elems(xr[r], yr[r], c, sn, same);
                            rotate_elems(vx[r], vy[r], c, sn, same);
                        }
#pragma unroll
                        for (int r = 0; r < RPW; ++r) {
                            yq[r] = yr[r];
                            vq[r] = vy[r];
                        }
                        if (wave == 0) ++rot_it;
                    }
                    __syncthreads();
                }
                rot += rot_it;
                // V_P's block-I columns to the (now free) slots of R's
                // block-J columns: slot b + k holds column k
#pragma unroll
                for (int r = 0; r < RPW; ++r) A[(HB + lane) * P + r0 + r] = vx[r];
                vp_layout = 2;
                __syncthreads();
            } else {
                for (int it = 0; it < sweeps; ++it) {
                    unsigned long long rot_it = 0;
                    for (int s = 0; s < nsteps; ++s) {
                        const int2 pq = inner_pair_t<ALL>(W, s, lane);
                        double *yp = A + pq.x * P + r0, *yq = A + pq.y * P + r0;
                        double xr[RPW], yr[RPW];
#pragma unroll
                        for (int r = 0; r < RPW; ++r) {
                            xr[r] = yp[r];
                            yr[r] = yq[r];
                        }
                        double c, sn;
                        bool same, cl;
                        const bool act = pair_transform<RPW, RB, NW, NP>(
                            xr, yr, red, wave, lane, a.tol, JP[pq.x] == JP[pq.y], c, sn, same, bad, cl);
                        if (cl && wave == 0) ++ncl;
                        if (wave == 0)
                            log[((size_t)it * nsteps + s) * NP + lane] =
                                act ? make_double2(same ? c : -c, sn) : make_double2(1.0, 0.0);
                        if (act) {
#pragma unroll
                            for (int r = 0; r < RPW; ++r) rotate_elems(xr[r], yr[r], c, sn, same);
#pragma unroll
                            for (int r = 0; r < RPW; ++r) {
                                yp[r] = xr[r];
                                yq[r] = yr[r];
                            }
                            if (wave == 0) ++rot_it;
                        }
                        __syncthreads();
                    }
                    ++logged;
                    rot += rot_it;
                    const double wr = wave_sum((double)rot_it);
                    if (lane == 0) s_rot[wave] = (unsigned long long)wr;
                    __syncthreads();
                    // only wavefront 0 counted, so its total is the step's
                    const unsigned long long tot = s_rot[0];
                    __syncthreads();
                    if (tot == 0) break;
                }
                // V_P := I (row-major, pitch P), then the logged transforms are
                // replayed on its rows.  Lanes l and l + 32 of wavefront w own row
                // 32 w + l mod 32 and take the first and the second half of each
                // step's pairs: the pairs of a step are disjoint, and the LDS accesses
                // of one wavefront complete in order, so the halves need no barrier
                // between steps.  The log passes through LDS (the red area) RC steps
                // at a time, the next chunk loaded while the current one is replayed;
                // its global writes were made visible first.
                __threadfence();
                for (int e = tid; e < W * W; e += kLogThreads) {
                    const int r = e / W, c = e % W;
                    A[r * P + c] = (r == c) ? 1.0 : 0.0;
                }
                constexpr int RC = kLogThreads / NP;   // steps per chunk: one entry per thread
                static_assert(RC * NP == kLogThreads && RC * NP * 2 <= NW * 3 * NP, "log chunk in red");
                double2 *stage = (double2 *)red;
                const long total = (long)logged * nsteps;   // logged steps
                const int row = wave * 32 + (lane & 31), half = lane >> 5;
                double *vr = A + row * P;
                double2 nxt = (total * NP > tid) ? log[tid] : make_double2(1.0, 0.0);
                for (long c0 = 0; c0 < total; c0 += RC) {
                    __syncthreads();   // the previous chunk is no longer read
                    stage[tid] = nxt;
                    __syncthreads();
                    const long e_next = (c0 + RC) * NP + tid;
                    if (e_next < total * NP) nxt = log[e_next];
                    for (int sc = 0; sc < RC && c0 + sc < total; ++sc) {
                        const int s = (int)((c0 + sc) % nsteps);   // step within its inner sweep
                        const double2 *le = stage + sc * NP + half * (NP / 2);
                        // groups of RG pairs: all loads, then the arithmetic, then the
                        // stores (the pairs of a step are disjoint); a pair that was
                        // not rotated has the entry (1, 0), whose transform leaves
                        // both elements as they are, so there is no branch
                        constexpr int RG = 16;
        #pragma unroll 1
                        for (int i0 = 0; i0 < NP / 2; i0 += RG) {
                            double2 e[RG];
                            int2 pq[RG];
                            double x[RG], y[RG];
        #pragma unroll
                            for (int u = 0; u < RG; ++u) {
                                e[u] = le[i0 + u];
                                pq[u] = inner_pair_t<ALL>(W, s, half * (NP / 2) + i0 + u);
                                x[u] = vr[pq[u].x];
                                y[u] = vr[pq[u].y];
                            }
        #pragma unroll
                            for (int u = 0; u < RG; ++u)
                                rotate_elems(x[u], y[u], fabs(e[u].x), e[u].y, e[u].x > 0.0);
        #pragma unroll
                            for (int u = 0; u < RG; ++u) {
                                vr[pq[u].x] = x[u];
                                vr[pq[u].y] = y[u];
                            }
                        }
                    }
                }
                __syncthreads();
                vp_layout = 0;
            }
        };
        if (a.all_pairs)
            sweeps_and_replay(std::true_type{});
        else
            sweeps_and_replay(std::false_type{});
    } else {
        // G_P is transformed in place; V_P (column-major, pitch P) collects
        // the transforms for V
        for (int e = tid; e < W * W; e += kLogThreads) {
            const int r = e % W, c = e / W;
            A[c * P + r] = (r == c) ? 1.0 : 0.0;
        }
        __syncthreads();
        for (int it = 0; it < sweeps; ++it) {
            unsigned long long rot_it = 0;
            inner_sweep_global<NW>(a.G, a.ldg, a.m, A, P, W, JP, a.all_pairs, W, a.tol, d, b,
                                   rot_it, ncl, &bad);
            rot += rot_it;
            const double wr = wave_sum((double)rot_it);
            if (lane == 0) s_rot[wave] = (unsigned long long)wr;
            __syncthreads();
            unsigned long long tot = 0;
            for (int w = 0; w < NW; ++w) tot += s_rot[w];
            __syncthreads();
            if (tot == 0) break;
        }
    }
    {
        const double wr = wave_sum((double)rot), wc = wave_sum((double)ncl);
        if (lane == 0) {
            s_rot[wave] = (unsigned long long)wr;
            s_cl[wave] = (unsigned long long)wc;
        }
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
        if (s_bad) a.ctr->nonfinite = 1u;
        a.flag[pv] = (tot > 0 && !s_bad) ? (broke ? 2 : 1) : 0;
    }
    if (tot > 0) {
        double *out = a.vpt + (size_t)pv * W * W;
        for (int e = tid; e < W * W; e += kLogThreads) {
            const int r = e / W, c = e % W;
            out[e] = vp_layout == 0   ? A[r * P + c]
                     : vp_layout == 1 ? A[c * P + r]
                                      : A[((c + W / 2) % W) * P + r];
        }
    }
}

// ------------------------------------------------- k_pivot_solve_ij (W = 128)
// The pivot solve of the block-oriented steps at W = 128 (b = 64): the one
// inner sweep over the pairs (block I column, block J column) of Alg. 3.4,
// in the bipartite shift order (step s pairs column k with column
// b + (k + s) mod b).  Eight wavefronts in two roles.  Wavefronts 0-3 keep
// rows [32 w, 32 w + 32) of R in registers: lane k the block-I column k and,
// at step s, the block-J column (k + s) mod b, which is the column its pair
// rotates; they form the dot products (partials meet in LDS, double-buffered
// by step parity: one barrier per step), the transforms, and rotate R.
// Wavefronts 4-7 keep the same rows of V_P and apply each step's transforms
// one step later, from the (c, s) that wavefront 0 leaves in LDS, while the
// R wavefronts wait on their reductions.  After each step every block-J
// column moves to the lane below (a DPP rotate of the wavefront), the lane
// that pairs it next; after b steps each column is back in its lane.  The
// rotation is applied without a branch (a pair that does not rotate has
// c = 1, s = 0).  The load, skip test and Cholesky factorisation are those
// of k_pivot_solve_log; after a breakdown V_P is accumulated in LDS while
// the inner sweep runs on G_P.
constexpr int kIJThreads = 512;
// DPP control: wavefront rotate by one lane, lane k taking lane k + 1's value
constexpr int kDppWaveRol1 = 0x134;

template <int W>
__global__ __launch_bounds__(kIJThreads) void k_pivot_solve_ij(PivotSolveArgs a)
{
    constexpr int NT = kIJThreads;
    constexpr int NW = NT / 64;
    constexpr int P = W + 1;
    constexpr int HB = W / 2;          // b: pairs per step, one per lane
    constexpr int NP = HB;
    constexpr int NR = NW / 2;         // wavefronts per role
    constexpr int RPW = W / NR;        // rows of R (or of V_P) per wavefront
    constexpr int RB = 0;              // dot products in four interleaved chains
    static_assert(NP == 64 && RPW % 4 == 0, "one lane per pair");
    __shared__ double A[W * P];        // Gram, then R (upper); V_P after a breakdown
    __shared__ double red[2][NR * 3 * NP];   // partial dots, by step parity
    __shared__ double cs[2][3 * NP];         // c, s and the signed s of each pair, by step parity
    __shared__ double dsh[W];          // square roots of the diagonal, then the pivots d_j
    __shared__ signed char JP[W];
    __shared__ int s_need, s_bad, s_brk;
    __shared__ unsigned long long s_rot[NW], s_cl[NW];
    const int pv = blockIdx.x;
    const int4 d = a.piv[pv];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int b = a.b;

    if (tid < W) {
        const int c = pivot_col(tid, d, b);
        JP[tid] = (a.J && c >= 0) ? a.J[c] : (signed char)1;
    }
    if (tid == 0) {
        s_need = 0;
        s_bad = 0;
        s_brk = 0;
    }
    pivot_load_gram<W, NT>(a.ap + (size_t)pv * W * W, A, tid);
    __syncthreads();
    if (tid < W) dsh[tid] = sqrt(A[tid * P + tid]);
    __syncthreads();
    {
        bool need, bad_entry;
        pivot_skip_test<W, NT>(A, dsh, b, false, a.tol, tid, need, bad_entry);
        if (need) s_need = 1;
        if (bad_entry) s_bad = 1;
    }
    __syncthreads();
    if (s_bad) {
        if (tid == 0) {
            a.ctr->nonfinite = 1u;
            a.flag[pv] = 0;
        }
        return;
    }
    if (!s_need) {
        if (tid == 0) a.flag[pv] = 0;
        return;
    }
    const bool broke = pivot_cholesky<W, NT>(A, dsh, &s_brk, tid);
    if (broke && !a.G) {
        // no FP64 copy of G to transform in place (the FP32 sweeps): the
        // pivot is left to the FP64 sweeps that follow
        if (tid == 0) {
            atomicAdd(&a.ctr->breakdowns, 1ull);
            a.flag[pv] = 0;
        }
        return;
    }
    unsigned long long rot = 0, ncl = 0;
    int bad = 0;
    const bool rwave = wave < NR;
    const int r0 = (wave % NR) * RPW;
    double *out = a.vpt + (size_t)pv * W * W;
    if (!broke) {
        const int ci = lane, cj = HB + lane;
        const signed char jpi = JP[ci];
        if (rwave) {
            // R's block-I column `lane` and the block-J column in the lane
            // (the diagonal sqrt(d_j), zero below it)
            double xr[RPW], yr[RPW];
            const double di = sqrt(dsh[ci]), dj = sqrt(dsh[cj]);
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int row = r0 + r;
                const double ai = A[ci * P + row], aj = A[cj * P + row];
                xr[r] = row < ci ? ai : (row == ci ? di : 0.0);
                yr[r] = row < cj ? aj : (row == cj ? dj : 0.0);
            }
            for (int s = 0; s < HB; ++s) {
                const bool same_sign = jpi == JP[HB + ((lane + s) & (HB - 1))];
                double c, sn;
                bool same, cl;
                const bool act = pair_transform<RPW, RB, NR, NP>(xr, yr, red[s & 1], wave, lane, a.tol,
                                                                 same_sign, c, sn, same, bad, cl);
                // x' = c x - s y (trigonometric) or c x + s y (hyperbolic), y' = s x + c y
                const double sx = same ? -sn : sn;
                if (wave == 0) {
                    cs[s & 1][lane] = c;
                    cs[s & 1][NP + lane] = sn;
                    cs[s & 1][2 * NP + lane] = sx;
                    rot += act ? 1ull : 0ull;
                    ncl += cl ? 1ull : 0ull;
                }
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    const double x0 = xr[r], y0 = yr[r];
                    xr[r] = c * x0 + sx * y0;
                    yr[r] = sn * x0 + c * y0;
                }
#pragma unroll
                for (int r = 0; r < RPW; ++r) yr[r] = dpp_move<kDppWaveRol1>(yr[r]);
            }
            __syncthreads();   // pairs with the V wavefronts' last pass
        } else {
            // V_P's columns `lane` and b + lane of I; pass s applies step
            // s - 1 (one barrier per pass, as the R wavefronts' steps)
            double vx[RPW], vy[RPW];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                vx[r] = r0 + r == ci ? 1.0 : 0.0;
                vy[r] = r0 + r == cj ? 1.0 : 0.0;
            }
            for (int s = 0; s <= HB; ++s) {
                __syncthreads();
                if (s == 0) continue;
                const double *e = cs[(s - 1) & 1];
                const double c = e[lane], sn = e[NP + lane], sx = e[2 * NP + lane];
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    const double x0 = vx[r], y0 = vy[r];
                    vx[r] = c * x0 + sx * y0;
                    vy[r] = sn * x0 + c * y0;
                }
#pragma unroll
                for (int r = 0; r < RPW; ++r) vy[r] = dpp_move<kDppWaveRol1>(vy[r]);
            }
            // V_P row-major (the update reads it only if a pair rotated)
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                out[(size_t)(r0 + r) * W + lane] = vx[r];
                out[(size_t)(r0 + r) * W + HB + lane] = vy[r];
            }
        }
    } else {
        // G_P is transformed in place; V_P (column-major, pitch P) collects
        // the transforms for V
        for (int e = tid; e < W * W; e += NT) {
            const int r = e % W, c = e / W;
            A[c * P + r] = (r == c) ? 1.0 : 0.0;
        }
        __syncthreads();
        inner_sweep_global<NW>(a.G, a.ldg, a.m, A, P, W, JP, 0, W, a.tol, d, b, rot, ncl, &bad);
    }
    {
        const double wr = wave_sum((double)rot), wc = wave_sum((double)ncl);
        if (lane == 0) {
            s_rot[wave] = (unsigned long long)wr;
            s_cl[wave] = (unsigned long long)wc;
        }
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
        if (s_bad) a.ctr->nonfinite = 1u;
        a.flag[pv] = (tot > 0 && !s_bad) ? (broke ? 2 : 1) : 0;
    }
    if (tot > 0 && broke) {
        // V_P row-major from the LDS copy
        for (int e = tid; e < W * W; e += NT) {
            const int r = e / W, c = e % W;
            out[e] = A[c * P + r];
        }
    }
}

// ---------------------------------------------------------------- k_update
// One workgroup (four wavefronts) handles consecutive 64-row tiles of one
// pivot (of G, or of V): V_P is staged in LDS once, and the loads of tile
// t+1 are in flight while the MFMAs of tile t run.  At W = 128 V_P takes
// 144 KiB of LDS, so one workgroup fills a CU: its wavefronts then have the
// whole register file (one per SIMD), which the 32 k-steps of operands of
// two tiles need, and eight tiles per workgroup amortise the staging.
template <int W> struct UpdateShape {
    static constexpr int threads = 256;
    static constexpr int tile_rows = 64;   // 16 rows per wavefront
    static constexpr int tiles = W <= 64 ? 4 : 8;
    static constexpr int group_rows = tile_rows * tiles;
};

// The row tiles of one k_update workgroup: V_P (W x W, FP64 row-major) is
// staged in S (row pitch W + 16), then the wavefront transforms rows
// wrow + lane % 16 + TR t.  FULL: all rows of the workgroup exist, so no
// load or store is predicated and the compiler waits for the prefetched
// operands alone (a predicated memory operation leaves the count of those in
// flight unknown, and it then waits for all of them, the stores included).
// Otherwise the loads are clamped to the last row (the lanes past it only
// feed result rows that are not stored) and the stores are guarded.
// UNEVEN: the pivot may have empty positions; their loads read column 0 of
// the block (the row of V_P for an empty position is e_k, so the value only
// meets zeros in real output columns) and their results are not stored.
template <int W, class T, bool FULL, bool UNEVEN>
__device__ __forceinline__ void update_tiles(T *__restrict__ X, long ld, int rows, int wrow,
                                             int lane, int4 d, const double *__restrict__ src, T *S)
{
    constexpr int NTH = UpdateShape<W>::threads;
    constexpr int TR = UpdateShape<W>::tile_rows;
    constexpr int kUpdateTiles = UpdateShape<W>::tiles;
    constexpr int KS = W / 4;   // k-steps of the MFMA
    constexpr int NT = W / 16;  // output column tiles
    constexpr int SP = W + 16;
    constexpr int SE = W * W / NTH;
    constexpr int HB = W / 2;
    auto clamp_row = [&](int r) { return FULL ? r : min(r, rows - 1); };
    // Pivot positions 4g .. 4g+3 lie in one block (b is a multiple of 4), so
    // the element of lane l in k-step ks is at a wave-uniform base (the block,
    // then column 4 ks - bp of it) plus a per-lane byte offset that is the
    // same for every k-step of a tile: (l / 16) columns and the row.  With
    // empty positions (UNEVEN) the lane part is formed per k-step instead
    // (column 0 of the block for an empty position).
    const int lq = lane / 16;
    const int row0 = wrow + lane % 16;
    const char *xI = (const char *)(X + (size_t)d.x * ld), *xJ = (const char *)(X + (size_t)d.z * ld);
    const size_t colb = (size_t)ld * sizeof(T);   // bytes per column
    auto kbase = [&](int ks) -> const char * {
        return (4 * ks < HB) ? xI + (size_t)(4 * ks) * colb : xJ + (size_t)(4 * ks - HB) * colb;
    };
    // the element of (column 4 ks - bp + l / 16, row): kbase(ks) plus a
    // 32-bit byte offset, or with empty positions a signed 64-bit one (an
    // empty position reads column 0 of the block, behind kbase(ks))
    auto kload = [&](int ks, int row) -> T {
        if constexpr (!UNEVEN) {
            const unsigned off = ((unsigned)lq * (unsigned)ld + (unsigned)row) * (unsigned)sizeof(T);
            return *(const T *)(kbase(ks) + off);
        } else {
            const bool in_i = 4 * ks < HB;
            const int o = (in_i ? 4 * ks : 4 * ks - HB) + lq;
            const bool real = o < (in_i ? d.y : d.w);
            const long back = real ? (long)lq : -(long)(in_i ? 4 * ks : 4 * ks - HB);
            return *(const T *)(kbase(ks) + (back * ld + row) * (long)sizeof(T));
        }
    };

    // all loads of V_P and of the first tile in flight before the LDS stores
    double sv[SE];
#pragma unroll
    for (int i = 0; i < SE; ++i) sv[i] = src[threadIdx.x + NTH * i];
    T bf[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) bf[ks] = kload(ks, clamp_row(row0));
#pragma unroll
    for (int i = 0; i < SE; ++i) {
        const int e = threadIdx.x + NTH * i;
        S[(e / W) * SP + (e % W)] = (T)sv[i];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kUpdateTiles; ++t) {
        const int row = row0 + t * TR;
        if (!FULL && wrow + t * TR >= rows) break;   // wave-uniform
        const bool more = t + 1 < kUpdateTiles;
        const int nrow = clamp_row(row + TR);
        typename Mfma<T>::acc acc[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[q] = typename Mfma<T>::acc{0, 0, 0, 0};
        // fully unrolled (a rolled k-loop indexes bf[] at run time).  The
        // V_P operands go through two register sets: those of k-step ks + 1
        // are read while the MFMAs of k-step ks run, and the empty asm
        // statement (no instruction) keeps the reads of later k-steps from
        // being hoisted further, where they would take many more registers.
        // Once the MFMAs of k-step ks are issued, bf[ks] is reloaded with the
        // next tile's operand (a whole tile ahead of its use), so one set of
        // G operands is live, not two.
        const T *sbase = S + lq * SP + (lane % 16);
        T a_cur[NT], a_nxt[NT];
#pragma unroll
        for (int q = 0; q < NT; ++q) a_cur[q] = sbase[q * 16];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            if (ks + 1 < KS) {
#pragma unroll
                for (int q = 0; q < NT; ++q) a_nxt[q] = sbase[4 * (ks + 1) * SP + q * 16];
            }
            asm volatile("" ::: "memory");
#pragma unroll
            for (int q = 0; q < NT; ++q) acc[q] = mfma16x16x4(a_cur[q], bf[ks], acc[q]);
            if (more) bf[ks] = kload(ks, nrow);
            if (ks + 1 < KS) {
#pragma unroll
                for (int q = 0; q < NT; ++q) a_cur[q] = a_nxt[q];
            }
        }
        if (FULL || row < rows) {
            // element r of tile q is pivot position q 16 + Mfma<T>::row(lane, r)
            // (a 16-position tile lies inside one block: 16 | b)
            // a uniform base (the block, the tile's first column of this
            // element) plus a 32-bit per-lane byte offset
            const unsigned lane_st =
                ((unsigned)Mfma<T>::row(lane, 0) * (unsigned)ld + (unsigned)row) * (unsigned)sizeof(T);
#pragma unroll
            for (int q = 0; q < NT; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const bool in_i = q * 16 < HB;
                    const int c0 = (in_i ? q * 16 : q * 16 - HB) + Mfma<T>::row(0, r);   // uniform
                    if (UNEVEN && c0 + Mfma<T>::row(lane, 0) >= (in_i ? d.y : d.w)) continue;
                    char *cb = (char *)(X + (size_t)(in_i ? d.x : d.z) * ld) + (size_t)c0 * colb;
                    *(T *)(cb + lane_st) = acc[q][r];
                }
        }
    }
}

template <int W, class T, bool UNEVEN>
__device__ __forceinline__ void update_body(T *__restrict__ G, int m, long ldg, T *__restrict__ V,
                                            int nv, long ldv, const int4 *__restrict__ piv,
                                            const double *__restrict__ vpt,
                                            const int *__restrict__ flag, int groups_g, T *S)
{
    constexpr int GR = UpdateShape<W>::group_rows;
    const int pv = blockIdx.y;
    const bool is_v = (int)blockIdx.x >= groups_g;
    const int f = flag[pv];
    if (!(f == 1 || (is_v && f == 2))) return;   // flag 2: G_P already transformed
    T *X = is_v ? V : G;
    const long ld = is_v ? ldv : ldg;
    const int rows = is_v ? nv : m;
    const int4 d = piv[pv];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int group = is_v ? (int)blockIdx.x - groups_g : (int)blockIdx.x;
    const int wrow = group * GR + wave * 16;   // first row of the wavefront
    const double *src = vpt + (size_t)pv * W * W;
    if ((group + 1) * GR <= rows)   // the same for the whole workgroup
        update_tiles<W, T, true, UNEVEN>(X, ld, rows, wrow, lane, d, src, S);
    else
        update_tiles<W, T, false, UNEVEN>(X, ld, rows, wrow, lane, d, src, S);
}

// V_P row-major with a row pitch of W + 16 elements: the four 16-lane row
// groups of a fragment read then cover all 64 LDS banks in two cycles.
template <int W, class T, bool UNEVEN>
__global__ __launch_bounds__(256) void k_update(T *__restrict__ G, int m, long ldg,
                                                T *__restrict__ V, int nv, long ldv,
                                                const int4 *__restrict__ piv,
                                                const double *__restrict__ vpt,
                                                const int *__restrict__ flag, int groups_g)
{
    static_assert(W <= 64, "256 threads");
    __shared__ T S[W * (W + 16)];
    update_body<W, T, UNEVEN>(G, m, ldg, V, nv, ldv, piv, vpt, flag, groups_g, S);
}

template <class T, bool UNEVEN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_update128(T *__restrict__ G, int m, long ldg,
                                                   T *__restrict__ V, int nv, long ldv,
                                                   const int4 *__restrict__ piv,
                                                   const double *__restrict__ vpt,
                                                   const int *__restrict__ flag, int groups_g)
{
    __shared__ T S[128 * (128 + 16)];
    update_body<128, T, UNEVEN>(G, m, ldg, V, nv, ldv, piv, vpt, flag, groups_g, S);
}

// ------------------------------------------------------------ host driver
bool block_width_supported(int b) { return b == 16 || b == 32 || b == 64; }

// Blocks of the uniform partition (Sec. 3): N = 2 ceil(n / 2b) blocks,
// widths n / N or n / N + 1 (the first n mod N blocks are the wider ones),
// all at most b; every block needs a column.
static int block_count(int n, int b) { return 2 * ((n + 2 * b - 1) / (2 * b)); }

bool block_shape_supported(int m, int n, int b)
{
    return block_width_supported(b) && n >= 2 && m >= n && block_count(n, b) <= n;
}

bool block_partition_even(int n, int b) { return n % (2 * b) == 0; }

int choose_block_width(int m, int n)
{
    // the autotuner's choice when it has measured this shape, else the
    // widest block whose pivot still leaves every step a few hundred
    // workgroups of Gram and update work
    int b = tuned_block_width(m, n);
    if (b > 0) return b;
    if (n >= 4096) return 64;
    if (n >= 512) return 32;
    return 16;
}

int auto_variant(int m, int n)
{
    const int v = tuned_variant(m, n);
    if (v >= 0) return v;
    // the block path wins once the matrix no longer fits the caches that
    // make the pointwise steps cheap (measured on the MI355X: n = 1024 runs
    // faster pointwise, n = 2048 and above block-oriented)
    return n >= 2048 ? JEVD_VAR_BLOCK_ORIENTED : JEVD_VAR_POINTWISE;
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
    int b = -1, n = -1;
    std::vector<int> outer_start;   // host copy of the block ordering's step offsets
    int4 *d_outer = nullptr;        // pivots of every step (ring order): column ranges
    size_t cap_outer = 0;
};

static BlockTables *tables_of(BlockWorkspace *ws)
{
    if (!ws->tables) ws->tables = new BlockTables();
    return (BlockTables *)ws->tables;
}

static int prepare_tables(BlockWorkspace *ws, int n, int b, hipStream_t st)
{
    BlockTables *t = tables_of(ws);
    if (t->n == n && t->b == b) return JEVD_OK;
    const int N = block_count(n, b);
    std::vector<int> os, op, bstart(N + 1, 0);
    for (int k = 0; k < N; ++k) bstart[k + 1] = bstart[k] + n / N + (k < n % N ? 1 : 0);
    build_ordering(N, kOrdModModulus, os, op);
    std::vector<int4> desc(op.size() / 2);
    for (size_t e = 0; e < desc.size(); ++e) {
        const int I = op[2 * e], J = op[2 * e + 1];
        desc[e] = make_int4(bstart[I], bstart[I + 1] - bstart[I], bstart[J], bstart[J + 1] - bstart[J]);
    }
    int rc = grow(&t->d_outer, &t->cap_outer, desc.size() + 1);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(t->d_outer, desc.data(), desc.size() * sizeof(int4),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    t->outer_start = os;
    t->n = n;
    t->b = b;
    return JEVD_OK;
}

static size_t pivot_lds_bytes(int W)
{
    return 2 * (size_t)W * (W + 1) * sizeof(double);
}

// Entries of the inner-transform log of one pivot (W = 128): one per pair
// of every inner step of every inner sweep it may run.
static long log_entries(int W, bool full_block, int max_inner)
{
    return (long)(full_block ? max_inner : 1) * W * (W / 2);
}

// One outer step: Gram, pivot solve, update of G and V (one launch each) on
// the iterate G (and V) of element type T.  The pivot solve always runs in
// FP64 on the Gram partials; tol is the step's rotation threshold.  For
// T = float there is no FP64 copy of G for the in-place breakdown path, so a
// pivot whose Cholesky breaks down is left for the FP64 sweeps.
// Launches the update of one step: rows of G (is_v false) or of V.
template <int W, class T>
static hipError_t launch_update(const BlockRunArgs &a, bool is_v, bool uneven, T *G, long ldg, T *V,
                                long ldv, const int4 *piv, const double *vp, const int *flags,
                                hipStream_t st)
{
    constexpr int GR = UpdateShape<W>::group_rows;
    const int npiv = block_count(a.n, a.b) / 2;
    // groups_g = 0 sends every workgroup of the launch to V
    const int groups = is_v ? (a.n + GR - 1) / GR : (a.m + GR - 1) / GR;
    const int groups_g = is_v ? 0 : groups;
    const dim3 grid(groups, npiv);
    if constexpr (W == 128) {
        if (uneven)
            k_update128<T, true><<<grid, 256, 0, st>>>(G, a.m, ldg, V, a.n, ldv, piv, vp, flags,
                                                       groups_g);
        else
            k_update128<T, false><<<grid, 256, 0, st>>>(G, a.m, ldg, V, a.n, ldv, piv, vp, flags,
                                                        groups_g);
    } else {
        if (uneven)
            k_update<W, T, true><<<grid, 256, 0, st>>>(G, a.m, ldg, V, a.n, ldv, piv, vp, flags,
                                                       groups_g);
        else
            k_update<W, T, false><<<grid, 256, 0, st>>>(G, a.m, ldg, V, a.n, ldv, piv, vp, flags,
                                                        groups_g);
    }
    return hipGetLastError();
}

// V(:,P) <- V(:,P) V_P for the step whose pivots start at outer step k and
// whose transforms sit in parity `par`, on the second stream, after the
// solve's stream has recorded evReady; records evVdone[par].
template <int W, class T>
static hipError_t launch_v_update(BlockWorkspace *ws, const BlockRunArgs &a, BlockTables *t, int k,
                                  int par, T *G, long ldg, T *V, long ldv)
{
    const int npiv = block_count(a.n, a.b) / 2;
    const int4 *piv = t->d_outer + t->outer_start[k];
    const double *vp = ws->vp + (size_t)par * npiv * W * W;
    const int *flags = ws->flags + (size_t)par * npiv;
    hipStream_t vs = ws->vstream;
    hipError_t e;
    if ((e = hipStreamWaitEvent(vs, ws->evReady, 0)) != hipSuccess) return e;
    if ((e = a.timer->begin(vs, JEVD_K_UPDATE)) != hipSuccess) return e;
    if ((e = launch_update<W, T>(a, true, !block_partition_even(a.n, a.b), G, ldg, V, ldv, piv, vp,
                                 flags, vs)) != hipSuccess)
        return e;
    if ((e = a.timer->end(vs)) != hipSuccess) return e;
    return hipEventRecord(ws->evVdone[par], vs);
}

// One parallel step of Alg. 3.4 (outer step k; its transforms V_P and flags
// go to the buffer of parity `par`).  G is updated on the solve's stream.
// V is read by no later step, so V's update is deferred: the update of the
// previous step (outer step pend_k >= 0, parity par ^ 1) is released once
// this step's Gram is formed and runs on the second stream beside this
// step's pivot solve, which occupies one CU per pivot.  Before the pivot
// solve overwrites a parity's buffer, the solve's stream waits for the V
// update that last read it (wait_v).  On the last step of a sweep (last),
// evReady is recorded after the pivot solve for the caller's flush of that
// step's V update.
template <int W, class T>
static hipError_t launch_step(BlockWorkspace *ws, const BlockRunArgs &a, BlockTables *t, int k,
                              int par, bool wait_v, int pend_k, bool last, int nsplit,
                              int rows_per_split, bool gram_rows, SweepCounters *ctr, T *G,
                              long ldg, T *V, long ldv, double tol)
{
    const int npiv = block_count(a.n, a.b) / 2;
    const int4 *piv = t->d_outer + t->outer_start[k];
    const bool uneven = !block_partition_even(a.n, a.b);
    double *vp = ws->vp + (size_t)par * npiv * W * W;
    int *flags = ws->flags + (size_t)par * npiv;
    hipStream_t st = a.stream;
    hipError_t e;
    if ((e = a.timer->begin(st, JEVD_K_GRAM)) != hipSuccess) return e;
    if constexpr (W == 128) {
        if constexpr (sizeof(T) == sizeof(double)) {
            if (gram_rows)
                k_gram128_rows<<<dim3(npiv, nsplit), 256, 0, st>>>((const double *)G, a.m, ldg, piv,
                                                                   rows_per_split, ws->partial);
            else
                k_gram128<T><<<dim3(npiv, nsplit), 256, 0, st>>>(G, a.m, ldg, piv, rows_per_split,
                                                                 ws->partial);
        } else {
            k_gram128<T><<<dim3(npiv, nsplit), 256, 0, st>>>(G, a.m, ldg, piv, rows_per_split,
                                                             ws->partial);
        }
    } else
        k_gram<W, T><<<dim3(npiv, nsplit), 256, 0, st>>>(G, a.m, ldg, piv, rows_per_split, ws->partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_gram_reduce<W><<<dim3((W * W + 255) / 256, npiv), 256, 0, st>>>(ws->partial, nsplit, piv, a.b,
                                                                     ws->ap);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = a.timer->end(st)) != hipSuccess) return e;
    if (pend_k >= 0) {
        if ((e = hipEventRecord(ws->evReady, st)) != hipSuccess) return e;
        if ((e = launch_v_update<W, T>(ws, a, t, pend_k, par ^ 1, G, ldg, V, ldv)) != hipSuccess)
            return e;
    }

    PivotSolveArgs p;
    p.ap = ws->ap;
    p.J = a.dJ;
    p.piv = piv;
    p.b = a.b;
    p.tol = tol;
    p.all_pairs = (a.full_block || k == 0) ? 1 : 0;
    p.full_block = a.full_block ? 1 : 0;
    p.max_inner = a.max_inner;
    p.vpt = vp;
    p.flag = flags;
    p.ctr = ctr;
    p.G = (sizeof(T) == sizeof(double)) ? (double *)G : nullptr;
    p.m = a.m;
    p.ldg = ldg;
    p.sign_pivot = a.sign_pivot ? 1 : 0;
    p.vlog = ws->vlog;
    p.log_stride = log_entries(W, a.full_block, a.max_inner);
    if (wait_v && (e = hipStreamWaitEvent(st, ws->evVdone[par], 0)) != hipSuccess) return e;
    if ((e = a.timer->begin(st, JEVD_K_PIVOT_SOLVE)) != hipSuccess) return e;
    if constexpr (W == 128) {
        if (p.all_pairs)
            k_pivot_solve_log<128><<<npiv, kLogThreads, 0, st>>>(p);
        else
            k_pivot_solve_ij<128><<<npiv, kIJThreads, 0, st>>>(p);
    } else
        k_pivot_solve<W><<<npiv, kPivotThreads, pivot_lds_bytes(W), st>>>(p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = a.timer->end(st)) != hipSuccess) return e;
    if (V && last && (e = hipEventRecord(ws->evReady, st)) != hipSuccess) return e;

    if ((e = a.timer->begin(st, JEVD_K_UPDATE)) != hipSuccess) return e;
    if ((e = launch_update<W, T>(a, false, uneven, G, ldg, V, ldv, piv, vp, flags, st))) return e;
    return a.timer->end(st);
}

// Row split of the pivot Grams (about 1024 workgroups per step for W <= 64,
// 512 for W = 128, whose workgroups are twice as long) and the step
// workspaces; sets the pivot solve's LDS limit.
// Whether the Gram of the FP64 sweeps at W = 128 takes k_gram128_rows: an
// even partition, row pairs 16-byte aligned (even ldg), whole chunks of 8
// rows, and the lane offsets within 32 bits.
static bool gram_rows_applies(const BlockRunArgs &a, long ldg, bool fp64)
{
    return fp64 && a.b == 64 && block_partition_even(a.n, a.b) && ldg % 2 == 0 && a.m % 8 == 0 &&
           (ldg + a.m) * 16 * (long)sizeof(double) < (1L << 31);
}

static int prepare_steps(BlockWorkspace *ws, const BlockRunArgs &a, long ldg, bool fp64,
                         int *nsplit_out, int *rows_per_split_out, bool *gram_rows_out)
{
    const int b = a.b, W = 2 * b, npiv = block_count(a.n, b) / 2;
    int rc = prepare_tables(ws, a.n, b, a.stream);
    if (rc) return rc;
    const bool gram_rows = gram_rows_applies(a, ldg, fp64);
    int nsplit, rows_per_split;
    if (gram_rows) {
        // one workgroup per CU (it holds the whole register file), at least
        // 64 rows per split
        nsplit = std::max(1, std::min(256 / npiv, a.m / 64));
        rows_per_split = (a.m + nsplit - 1) / nsplit;
        rows_per_split = (rows_per_split + 7) / 8 * 8;
    } else {
        const int target = (W == 128) ? 512 : 1024;
        nsplit = target / npiv;
        if (nsplit < 1) nsplit = 1;
        int maxsplit = (a.m + 255) / 256;
        if (nsplit > maxsplit) nsplit = maxsplit;
        rows_per_split = (a.m + nsplit - 1) / nsplit;
        rows_per_split = (rows_per_split + 31) / 32 * 32;
    }
    nsplit = (a.m + rows_per_split - 1) / rows_per_split;
    *gram_rows_out = gram_rows;
    rc = grow(&ws->partial, &ws->capPartial, (size_t)npiv * nsplit * W * W);
    if (rc) return rc;
    rc = grow(&ws->vp, &ws->capVp, (size_t)2 * npiv * W * W);   // two parities
    if (rc) return rc;
    rc = grow(&ws->ap, &ws->capAp, (size_t)npiv * W * W);
    if (rc) return rc;
    rc = grow(&ws->flags, &ws->capFlags, (size_t)2 * npiv);
    if (rc) return rc;
    if (W == 128) {
        rc = grow(&ws->vlog, &ws->capVlog, (size_t)npiv * log_entries(W, a.full_block, a.max_inner));
        if (rc) return rc;
    }
    if (a.V && !ws->vstream) {
        // default priority, like the solve's stream
        HIP_TRY(hipStreamCreateWithFlags(&ws->vstream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&ws->evReady, hipEventDisableTiming));
        for (int i = 0; i < 2; ++i)
            HIP_TRY(hipEventCreateWithFlags(&ws->evVdone[i], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&ws->evJoin, hipEventDisableTiming));
    }
    if (W == 64) HIP_TRY(set_lds_limit((const void *)k_pivot_solve<64>, (int)pivot_lds_bytes(64)));
    *nsplit_out = nsplit;
    *rows_per_split_out = rows_per_split;
    return JEVD_OK;
}

// Block sweeps over the iterate (G, V) of type T until a sweep rotates
// nothing (at tol) or max_sweeps; counters in ctr[0 .. max_sweeps).  With
// stop_on_stall the sweeps also end (JEVD_OK) once a sweep after the third
// rotates at least as often as the one before: the rounding of the low-
// precision iterate, not the ordering, then decides the rotations.
template <class T>
static int block_sweeps(BlockWorkspace *ws, const BlockRunArgs &a, T *G, long ldg, T *V, long ldv,
                        double tol, int max_sweeps, SweepCounters *dctr, SweepCounters *hctr,
                        int *sweeps_done, bool stop_on_stall = false)
{
    *sweeps_done = 0;
    int nsplit = 0, rows_per_split = 0;
    bool gram_rows = false;
    int rc = prepare_steps(ws, a, ldg, sizeof(T) == sizeof(double), &nsplit, &rows_per_split,
                           &gram_rows);
    if (rc) return rc;
    BlockTables *t = tables_of(ws);
    const int N = block_count(a.n, a.b);
    HIP_TRY(hipMemsetAsync(dctr, 0, sizeof(SweepCounters) * max_sweeps, a.stream));
    // the second stream starts after what the solve's stream holds (V's
    // initial value) and is joined back into it at the end of every sweep
    const bool split = V != nullptr;
    if (split) {
        HIP_TRY(hipEventRecord(ws->evJoin, a.stream));
        HIP_TRY(hipStreamWaitEvent(ws->vstream, ws->evJoin, 0));
    }
    int step = 0;
    for (int s = 0; s < max_sweeps; ++s) {
        hipError_t e = hipSuccess;
        int pend_k = -1;   // outer step whose V update is not yet enqueued
        for (int k = 0; k < N && e == hipSuccess; ++k, ++step) {
            const int par = step & 1;
            const bool wait_v = split && step >= 2;
            if (a.b == 16)
                e = launch_step<32, T>(ws, a, t, k, par, wait_v, pend_k, k == N - 1, nsplit,
                                        rows_per_split, gram_rows, dctr + s, G, ldg, V, ldv, tol);
            else if (a.b == 32)
                e = launch_step<64, T>(ws, a, t, k, par, wait_v, pend_k, k == N - 1, nsplit,
                                        rows_per_split, gram_rows, dctr + s, G, ldg, V, ldv, tol);
            else
                e = launch_step<128, T>(ws, a, t, k, par, wait_v, pend_k, k == N - 1, nsplit,
                                        rows_per_split, gram_rows, dctr + s, G, ldg, V, ldv, tol);
            pend_k = split ? k : -1;
        }
        if (split) {
            if (e == hipSuccess && pend_k >= 0) {
                const int par = (step - 1) & 1;
                if (a.b == 16)
                    e = launch_v_update<32, T>(ws, a, t, pend_k, par, G, ldg, V, ldv);
                else if (a.b == 32)
                    e = launch_v_update<64, T>(ws, a, t, pend_k, par, G, ldg, V, ldv);
                else
                    e = launch_v_update<128, T>(ws, a, t, pend_k, par, G, ldg, V, ldv);
            }
            // also after a failed launch: nothing may still run on V at return
            hipError_t j = hipEventRecord(ws->evJoin, ws->vstream);
            if (j == hipSuccess) j = hipStreamWaitEvent(a.stream, ws->evJoin, 0);
            if (j != hipSuccess) {
                (void)hipStreamSynchronize(ws->vstream);
                if (e == hipSuccess) e = j;
            }
        }
        HIP_TRY(e);
        HIP_TRY(hipMemcpyAsync(hctr + s, dctr + s, sizeof(SweepCounters), hipMemcpyDeviceToHost,
                               a.stream));
        HIP_TRY(hipStreamSynchronize(a.stream));
        HIP_TRY(a.timer->collect());
        *sweeps_done = s + 1;
        if (hctr[s].nonfinite) return JEVD_ENONFINITE;
        if (hctr[s].rotations == 0) return JEVD_OK;
        if (stop_on_stall && s >= 3 && hctr[s].rotations >= hctr[s - 1].rotations) return JEVD_OK;
    }
    return JEVD_ENOCONV;
}

// Sign pivoting moves columns between pivot positions, so empty positions
// (uneven partitions) and the W = 128 pivot solve (unpivoted only) are
// excluded.
bool block_options_supported(int m, int n, int b, bool sign_pivot)
{
    if (!block_shape_supported(m, n, b)) return false;
    if (sign_pivot && (b == 64 || !block_partition_even(n, b))) return false;
    return true;
}

int run_block(BlockWorkspace *ws, const BlockRunArgs &a, int *sweeps_done)
{
    *sweeps_done = 0;
    if (!block_options_supported(a.m, a.n, a.b, a.sign_pivot)) return JEVD_EINVAL;
    return block_sweeps<double>(ws, a, a.G, a.ldg, a.V, a.ldv, a.tol, a.max_sweeps, a.dctr, a.hctr,
                                sweeps_done);
}

// ------------------------------------------------------- mixed precision
__global__ void k_to_f32(const double *__restrict__ X, long ldx, float *__restrict__ Y, long ldy,
                         int rows, int cols)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)rows * cols) return;
    const int r = (int)(e % rows), c = (int)(e / rows);
    Y[(size_t)c * ldy + r] = (float)X[(size_t)c * ldx + r];
}

__global__ void k_to_f64(const float *__restrict__ X, long ldx, double *__restrict__ Y, long ldy,
                         int rows, int cols)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)rows * cols) return;
    const int r = (int)(e % rows), c = (int)(e / rows);
    Y[(size_t)c * ldy + r] = (double)X[(size_t)c * ldx + r];
}

__global__ void k_identity_f32(float *__restrict__ X, long ldx, int n)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * n) return;
    const int r = (int)(e % n), c = (int)(e / n);
    X[(size_t)c * ldx + r] = (r == c) ? 1.0f : 0.0f;
}

// T <- (3 I - T) / 2 (n x n, ld n)
__global__ void k_newton_schulz(double *__restrict__ T, int n)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * n) return;
    const int r = (int)(e % n), c = (int)(e / n);
    T[e] = ((r == c) ? 1.5 : 0.0) - 0.5 * T[e];
}

static unsigned blocks_for(long count) { return (unsigned)((count + 255) / 256); }

static void gemm1(bool ta, bool tb, int M, int N, int K, const double *A, int lda, const double *B,
                  int ldb, double *D, int ldd, hipStream_t st)
{
    GemmArgs g{};
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.D = D;
    g.ldd = ldd;
    launch_gemm(ta, tb, g, 1, st);
}

int run_block_mixed(BlockWorkspace *ws, const BlockRunArgs &a, int max_sweeps_low, int *sweeps_low,
                    int *sweeps_done)
{
    *sweeps_low = 0;
    *sweeps_done = 0;
    if (!block_options_supported(a.m, a.n, a.b, a.sign_pivot) || !a.V) return JEVD_EINVAL;
    const int m = a.m, n = a.n;
    hipStream_t st = a.stream;
    int rc;
    if ((rc = grow(&ws->g32, &ws->capG32, (size_t)m * n))) return rc;
    if ((rc = grow(&ws->v32, &ws->capV32, (size_t)n * n))) return rc;
    if ((rc = grow(&ws->t64, &ws->capT64, (size_t)n * n))) return rc;
    // w64: two n x n iterates of the orthogonalisation, later G V0 (m x n)
    if ((rc = grow(&ws->w64, &ws->capW64, std::max((size_t)m * n, 2 * (size_t)n * n)))) return rc;
    // 1. FP32 copy of G, V32 = I; FP32 sweeps at the threshold the FP32
    //    Grams can resolve
    k_to_f32<<<blocks_for((long)m * n), 256, 0, st>>>(a.G, a.ldg, ws->g32, m, m, n);
    k_identity_f32<<<blocks_for((long)n * n), 256, 0, st>>>(ws->v32, n, n);
    HIP_TRY(hipGetLastError());
    const double tol_low = std::max(a.tol, 8.0 * std::sqrt((double)m) * 0x1p-24);
    int s32 = 0;
    rc = block_sweeps<float>(ws, a, ws->g32, m, ws->v32, n, tol_low, max_sweeps_low, a.dctr, a.hctr,
                             &s32, true);
    *sweeps_low = s32;
    if (rc != JEVD_OK && rc != JEVD_ENOCONV) return rc;
    // 2. V0 in FP64, made orthogonal to working precision by two Newton-
    //    Schulz steps V <- V (3 I - V^T V) / 2 (quadratic convergence to the
    //    orthogonal polar factor; |V^T V - I| ~ 1e-6 -> 1e-12 -> eps)
    double *V0 = ws->w64, *V1 = ws->w64 + (size_t)n * n;   // n x n, ld n
    k_to_f64<<<blocks_for((long)n * n), 256, 0, st>>>(ws->v32, n, V0, n, n, n);
    HIP_TRY(hipGetLastError());
    gemm1(true, false, n, n, n, V0, n, V0, n, ws->t64, n, st);
    k_newton_schulz<<<blocks_for((long)n * n), 256, 0, st>>>(ws->t64, n);
    gemm1(false, false, n, n, n, V0, n, ws->t64, n, V1, n, st);
    gemm1(true, false, n, n, n, V1, n, V1, n, ws->t64, n, st);
    k_newton_schulz<<<blocks_for((long)n * n), 256, 0, st>>>(ws->t64, n);
    gemm1(false, false, n, n, n, V1, n, ws->t64, n, a.V, a.ldv, st);
    HIP_TRY(hipGetLastError());
    // 3. G <- G V0 in FP64 (the FP32 iterate is discarded)
    gemm1(false, false, m, n, n, a.G, a.ldg, a.V, a.ldv, ws->w64, m, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpy2DAsync(a.G, sizeof(double) * a.ldg, ws->w64, sizeof(double) * m,
                             sizeof(double) * m, n, hipMemcpyDeviceToDevice, st));
    // 4. FP64 sweeps from G V0, accumulating onto V0
    return block_sweeps<double>(ws, a, a.G, a.ldg, a.V, a.ldv, a.tol, a.max_sweeps, a.dctr, a.hctr,
                                sweeps_done);
}

void block_workspace_free(BlockWorkspace *ws)
{
    if (ws->partial) (void)hipFree(ws->partial);
    if (ws->vp) (void)hipFree(ws->vp);
    if (ws->flags) (void)hipFree(ws->flags);
    if (ws->vlog) (void)hipFree(ws->vlog);
    if (ws->ap) (void)hipFree(ws->ap);
    if (ws->g32) (void)hipFree(ws->g32);
    if (ws->v32) (void)hipFree(ws->v32);
    if (ws->t64) (void)hipFree(ws->t64);
    if (ws->w64) (void)hipFree(ws->w64);
    if (ws->vstream) {
        (void)hipStreamSynchronize(ws->vstream);
        (void)hipStreamDestroy(ws->vstream);
        (void)hipEventDestroy(ws->evReady);
        for (int i = 0; i < 2; ++i) (void)hipEventDestroy(ws->evVdone[i]);
        (void)hipEventDestroy(ws->evJoin);
    }
    if (ws->tables) {
        BlockTables *t = (BlockTables *)ws->tables;
        if (t->d_outer) (void)hipFree(t->d_outer);
        delete t;
    }
    *ws = BlockWorkspace();
}

}  // namespace jevd
