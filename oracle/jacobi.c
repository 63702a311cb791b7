/*
 * One-sided Jacobi oracle (pointwise and block).  TEST INFRASTRUCTURE ONLY:
 * it is the plain, slow, obviously correct CPU reference that the GPU
 * library is checked against.  Only tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 *
 * This one source file is compiled three times, with `real` set to
 * double (suffix _d), long double (_l) and __float128 (_q).  Inputs and
 * outputs are always FP64 arrays; the _l and _q builds convert once on
 * entry and round once on exit, so they serve as high-precision truth for
 * the accuracy pins.  Build with -ffp-contract=off and without
 * -ffast-math: every product and sum below is one IEEE operation.
 *
 * Problem (Sec. 1, (1.3) and the hyperbolic SVD that follows it): given a
 * factor G (m x n, column-major, full column rank) and J = diag(j_i),
 * j_i in {+1,-1}, find V with V^T J V = J such that G V = U Sigma has
 * orthogonal columns.  Then H = G J G^T has eigenvalues
 * lambda_i = j_i ||(G V)_i||^2 and eigenvectors (G V)_i / ||(G V)_i||
 * (Sec. 1: squared column norms of the final factor are the eigenvalues;
 * Sec. 3.2: the eigenvector matrix comes from normalising the columns of
 * G V).  J = I is the positive definite (trigonometric) case.
 *
 * The method (Sec. 2.1, hyperbolic one-sided Jacobi): repeatedly pick a
 * pair of columns (g_p, g_q), form the 2x2 Gram A_P = [g_p g_q]^T [g_p g_q],
 * and transform the pair from the right by the 2x2 matrix that
 * diagonalises A_P: a trigonometric rotation (2.1) when j_p == j_q, a
 * hyperbolic one otherwise.  The same 2x2 matrix is applied to the columns
 * p, q of V.  A sweep visits every pair once in the chosen ordering.
 */
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#if defined(ORC_QUAD)
#include <quadmath.h>
typedef __float128 real;
#define R_SQRT(x) sqrtq(x)
#define R_FABS(x) fabsq(x)
#define SFX(name) name##_q
#elif defined(ORC_LONG)
typedef long double real;
#define R_SQRT(x) sqrtl(x)
#define R_FABS(x) fabsl(x)
#define SFX(name) name##_l
#else
typedef double real;
#define R_SQRT(x) sqrt(x)
#define R_FABS(x) fabs(x)
#define SFX(name) name##_d
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENONFINITE = -2, ORC_ENOCONV = -3,
       ORC_ENOMEM = -5 };

int orc_ordering(int n, int kind, int *step_start, int *pairs, int *npairs_out);

static int is_finite_r(real x) { return (x - x) == (x - x); }

/* Gram entries of the column pair (x, y) of length len: x.x, y.y, x.y,
 * summed left to right (Sec. 2.1, step 1 of the hyperbolic algorithm;
 * (3.4) for one column per block). */
static void pair_gram(const real *x, const real *y, int len,
                      real *axx, real *ayy, real *axy)
{
    real sxx = 0, syy = 0, sxy = 0;
    for (int k = 0; k < len; ++k) {
        sxx = sxx + x[k] * x[k];
        syy = syy + y[k] * y[k];
        sxy = sxy + x[k] * y[k];
    }
    *axx = sxx; *ayy = syy; *axy = sxy;
}

/*
 * 2x2 transform that diagonalises A_P = [[app, apq], [apq, aqq]]
 * (Sec. 2.1 step 2).  The paper does not print the formulas; these are the
 * standard ones, derived as follows.
 *
 * Trigonometric, Q = [[c, s], [-s, c]] (the real case of (2.1), sign
 * convention of (A.1)): the new pair is (c g_p - s g_q, s g_p + c g_q); its
 * off-diagonal Gram entry is cs(app - aqq) + (c^2 - s^2) apq.  With
 * t = s/c and zeta = (aqq - app) / (2 apq) it vanishes iff
 * t^2 + 2 zeta t - 1 = 0; the root of smaller modulus is
 * t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2)), and c = 1/sqrt(1+t^2), s = c t.
 *
 * Hyperbolic, Q = [[ch, sh], [sh, ch]] (Sec. 2.1, hyperbolic algorithm):
 * the new pair is (ch g_p + sh g_q, sh g_p + ch g_q); its off-diagonal
 * Gram entry is ch sh (app + aqq) + (ch^2 + sh^2) apq.  With t = sh/ch
 * (= tanh) and zeta = (app + aqq) / (2 apq) it vanishes iff
 * t^2 + 2 zeta t + 1 = 0; the root of smaller modulus is
 * t = -sgn(zeta) / (|zeta| + sqrt((|zeta|-1)(|zeta|+1))), and
 * ch = 1/sqrt((1-t)(1+t)), sh = ch t.  Q^T diag(1,-1) Q = diag(1,-1).
 * Since A_P is positive semidefinite, app + aqq >= 2|apq|, so |zeta| >= 1 in
 * exact arithmetic; when rounding gives |zeta| <= 1 (|t| would be 1) the
 * transform would be singular, and a smaller angle with |tanh| = 0.9 is
 * used instead (Sec. 3.2).
 *
 * sgn(zeta) is +1 for zeta >= 0, including -0.  For |zeta| > 1e150
 * (zeta^2 would overflow) t is replaced by its limit 1/(2 zeta) (trig) or
 * -1/(2 zeta) (hyperbolic).  Returns 1 if the hyperbolic clamp was used.
 */
static int rotation_params(real app, real aqq, real apq, int same_sign,
                           real *c_out, real *s_out)
{
    real zeta, t, c;
    int clamped = 0;
    if (same_sign) {
        zeta = (aqq - app) / (2 * apq);
        if (R_FABS(zeta) > (real)1e150) {
            t = 1 / (2 * zeta);
        } else {
            real sg = (zeta >= 0) ? 1 : -1;
            t = sg / (R_FABS(zeta) + R_SQRT(1 + zeta * zeta));
        }
        c = 1 / R_SQRT(1 + t * t);
    } else {
        zeta = (app + aqq) / (2 * apq);
        real sg = (zeta >= 0) ? 1 : -1;
        real az = R_FABS(zeta);
        if (az <= 1) {
            t = -sg * (real)0.9;
            clamped = 1;
        } else if (az > (real)1e150) {
            t = -1 / (2 * zeta);
        } else {
            t = -sg / (az + R_SQRT((az - 1) * (az + 1)));
        }
        c = 1 / R_SQRT((1 - t) * (1 + t));
    }
    *c_out = c;
    *s_out = c * t;
    return clamped;
}

/* Apply the 2x2 transform to the columns x, y (length len):
 * trig (x, y) <- (c x - s y, s x + c y); hyperbolic (x, y) <- (c x + s y, s x + c y)
 * (Sec. 2.1 step 3; (A.1)). */
static void apply_pair(real *x, real *y, int len, real c, real s, int same_sign)
{
    for (int k = 0; k < len; ++k) {
        real xk = x[k], yk = y[k];
        if (same_sign) {
            x[k] = c * xk - s * yk;
            y[k] = s * xk + c * yk;
        } else {
            x[k] = c * xk + s * yk;
            y[k] = s * xk + c * yk;
        }
    }
}

/*
 * One pivot pair: Gram, threshold, transform.  The pair is rotated only if
 * |apq| > tol sqrt(app) sqrt(aqq) (a zero column is never rotated).
 * Returns 1 if rotated, 0 if skipped, ORC_ENONFINITE on a non-finite Gram.
 */
static int process_pair(real *X, int ldx, int len, real *W, int ldw, int wlen,
                        int p, int q, int same_sign, real tol, long long *nclamp)
{
    real app, aqq, apq, c, s;
    real *xp = X + (size_t)p * ldx, *xq = X + (size_t)q * ldx;
    pair_gram(xp, xq, len, &app, &aqq, &apq);
    if (!is_finite_r(app) || !is_finite_r(aqq) || !is_finite_r(apq))
        return ORC_ENONFINITE;
    if (app == 0 || aqq == 0) return 0;
    if (!(R_FABS(apq) > tol * R_SQRT(app) * R_SQRT(aqq))) return 0;
    if (rotation_params(app, aqq, apq, same_sign, &c, &s) && nclamp) ++*nclamp;
    apply_pair(xp, xq, len, c, s, same_sign);
    if (W) apply_pair(W + (size_t)p * ldw, W + (size_t)q * ldw, wlen, c, s, same_sign);
    return 1;
}

/* Exported for the rotation-parameter pins ((A.3)). */
int SFX(orc_rotation)(double app, double aqq, double apq, int same_sign,
                      double *c, double *s)
{
    real cr, sr;
    int cl = rotation_params((real)app, (real)aqq, (real)apq, same_sign, &cr, &sr);
    *c = (double)cr; *s = (double)sr;
    return cl;
}

static void finalize(int m, int n, const real *Gr, const signed char *J,
                     double *G, int ldg, double *lambda)
{
    for (int i = 0; i < n; ++i) {
        real nrm2 = 0;
        for (int k = 0; k < m; ++k) nrm2 = nrm2 + Gr[(size_t)i * m + k] * Gr[(size_t)i * m + k];
        if (lambda) lambda[i] = (double)((J && J[i] < 0) ? -nrm2 : nrm2);
        for (int k = 0; k < m; ++k) G[(size_t)i * ldg + k] = (double)Gr[(size_t)i * m + k];
    }
}

static int check_args(int m, int n, int ldg, const signed char *J, int ldv, const double *V)
{
    if (n < 1 || m < n || ldg < m) return ORC_EINVAL;
    if (V && ldv < n) return ORC_EINVAL;
    if (J) for (int i = 0; i < n; ++i) if (J[i] != 1 && J[i] != -1) return ORC_EINVAL;
    return ORC_OK;
}

/*
 * Pointwise one-sided Jacobi.  G (m x n, ld ldg) is overwritten by the final
 * iterate G V.  J: n entries in {+1,-1}, NULL means J = I.  ordering: 0
 * row-cyclic, 1 modulus, 2 modified modulus.  V (n x n, ld ldv) may be NULL;
 * if accumulate_v, V holds a prior transform on entry, else V := I.
 * A sweep is one pass over the ordering; the iteration stops after the first
 * sweep that rotates no pair (so *sweeps_out counts that sweep too), or
 * returns ORC_ENOCONV after max_sweeps sweeps, leaving the current iterate.
 * lambda[i] = j_i ||g_i||^2 of the final iterate.  rot_per_sweep (optional,
 * max_sweeps entries) receives the rotations of each sweep.
 */
int SFX(orc_jevd)(int m, int n, double *G, int ldg, const signed char *J, double tol,
                  int ordering, int max_sweeps, int accumulate_v,
                  double *lambda, double *V, int ldv, int *sweeps_out,
                  long long *rot_per_sweep, long long *nclamp_out)
{
    int st = check_args(m, n, ldg, J, ldv, V);
    if (st) return st;
    if (max_sweeps < 1) return ORC_EINVAL;
    int npairs = 0;
    int nsteps = orc_ordering(n, ordering, NULL, NULL, &npairs);
    if (nsteps < 0) return ORC_EINVAL;
    int *step_start = (int *)malloc(sizeof(int) * (size_t)(nsteps + 1));
    int *pairs = (int *)malloc(sizeof(int) * 2 * (size_t)(npairs > 0 ? npairs : 1));
    real *Gr = (real *)malloc(sizeof(real) * (size_t)m * n);
    real *Vr = V ? (real *)malloc(sizeof(real) * (size_t)n * n) : NULL;
    if (!step_start || !pairs || !Gr || (V && !Vr)) {
        free(step_start); free(pairs); free(Gr); free(Vr);
        return ORC_ENOMEM;
    }
    orc_ordering(n, ordering, step_start, pairs, NULL);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < m; ++k) Gr[(size_t)i * m + k] = (real)G[(size_t)i * ldg + k];
    if (Vr)
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k)
                Vr[(size_t)i * n + k] = accumulate_v ? (real)V[(size_t)i * ldv + k]
                                                     : (real)(i == k ? 1 : 0);
    long long nclamp = 0;
    int sweeps = 0;
    st = ORC_ENOCONV;
    while (sweeps < max_sweeps) {
        long long rot = 0;
        ++sweeps;
        for (int sidx = 0; sidx < nsteps && st != ORC_ENONFINITE; ++sidx)
            for (int e = step_start[sidx]; e < step_start[sidx + 1]; ++e) {
                int p = pairs[2 * e], q = pairs[2 * e + 1];
                int same = !J || J[p] == J[q];
                int r = process_pair(Gr, m, m, Vr, n, n, p, q, same, (real)tol, &nclamp);
                if (r < 0) { st = r; break; }
                rot += r;
            }
        if (rot_per_sweep) rot_per_sweep[sweeps - 1] = rot;
        if (st == ORC_ENONFINITE) break;
        if (rot == 0) { st = ORC_OK; break; }
    }
    finalize(m, n, Gr, J, G, ldg, lambda);
    if (Vr)
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) V[(size_t)i * ldv + k] = (double)Vr[(size_t)i * n + k];
    if (sweeps_out) *sweeps_out = sweeps;
    if (nclamp_out) *nclamp_out = nclamp;
    free(step_start); free(pairs); free(Gr); free(Vr);
    return st;
}

/* ------------------------------------------------------------------------
 * Block one-sided Jacobi (Sec. 2.2-2.3, Alg. 3.4 with the unpivoted Cholesky,
 * or with the sign-pivoted Cholesky of Alg. 3.3: HBSC / HFSC).
 *
 * Columns are split into N = 2 ceil(n / (2b)) block columns whose widths
 * differ by at most one (Sec. 3: uniform partition).  Block pairs (I, J)
 * follow the modified modulus ordering over the N blocks.  For one pivot
 * block G_P = [G_I G_J] (m x w):
 *   1. A_P = G_P^T G_P                                           ((3.4))
 *   2. skip the pivot if every targeted off-diagonal entry satisfies
 *      |a_kl| <= tol sqrt(a_kk) sqrt(a_ll)
 *   3. Cholesky A_P = R^T R, R upper triangular                  (Sec. 2.3)
 *   4. one-sided Jacobi on the columns of the square factor R, accumulating
 *      the transforms in V_P (starting from I):
 *        block-oriented, first step of a sweep: one inner sweep over all
 *          pairs of the w columns;
 *        block-oriented, other steps: one inner sweep over the pairs (k, l)
 *          with k in I and l in J only (annihilate each entry of A_IJ once);
 *        full block: inner sweeps over all pairs until one rotates nothing
 *          (or max_inner sweeps).                                (Sec. 2.2)
 *   5. G_P <- G_P V_P and V(:, P) <- V(:, P) V_P  (one update per pivot,
 *      Sec. 2.3).
 * If the Cholesky factorisation breaks down (a non-positive pivot), step 4
 * runs on the columns of G_P itself instead of R.
 * With sign pivoting, step 3 is P^T A_P P = R_S^T R_S (Alg. 3.3), step 4
 * runs on R_S with the signs of the permuted positions (positive first),
 * V_P = P V' (the permutation applied to the rows of the accumulated V'),
 * and after the update column c of the block carries the sign of position
 * c.  Block-oriented steps other than the first of a sweep pair the first
 * w_I positions of R_S with the others.
 * Inner orderings: over all w columns the modified modulus ordering (odd
 * modulus for odd w); over the I x J pairs the bipartite shift: step
 * s = 0..L-1 (L = max(w_I, w_J)) holds the pairs (k, w_I + (k+s) mod L)
 * with k < w_I and (k+s) mod L < w_J.
 * Outer stopping rule: stop after the first block sweep that applies no
 * inner rotation anywhere.
 * ---------------------------------------------------------------------- */

/* Inner sweep over a pair list on the columns of X (len rows, ld ldx). */
static long long inner_sweep(real *X, int ldx, int len, real *VP, int w,
                             const int *step_start, const int *pairs, int nsteps,
                             const signed char *JP, real tol, long long *nclamp, int *bad)
{
    long long rot = 0;
    for (int sidx = 0; sidx < nsteps; ++sidx)
        for (int e = step_start[sidx]; e < step_start[sidx + 1]; ++e) {
            int p = pairs[2 * e], q = pairs[2 * e + 1];
            int same = JP[p] == JP[q];
            int r = process_pair(X, ldx, len, VP, w, w, p, q, same, tol, nclamp);
            if (r < 0) { *bad = 1; return rot; }
            rot += r;
        }
    return rot;
}

/* Bipartite shift ordering of the wi x wj cross pairs (see above). */
static int cross_ordering(int wi, int wj, int *step_start, int *pairs)
{
    int L = wi > wj ? wi : wj, np = 0;
    for (int s = 0; s < L; ++s) {
        step_start[s] = np;
        for (int k = 0; k < wi; ++k) {
            int l = (k + s) % L;
            if (l < wj) { pairs[2 * np] = k; pairs[2 * np + 1] = wi + l; ++np; }
        }
    }
    step_start[L] = np;
    return L;
}

/* ------------------------------------------------------------------------
 * Sign-pivoted Cholesky factorisation of a pivot Gram (Sec. 3.2, (3.5)-(3.7),
 * Alg. 3.3), used by the HBSC / HFSC variants.
 *
 * Cholesky with diagonal pivoting of a k x k symmetric matrix S (column-major,
 * ld lds, read only): P^T S P = R^T R with R upper triangular; at step j the
 * pivot is the largest remaining diagonal entry of the updated matrix (the
 * first one on ties).  perm[c] is the row/column of S moved to position c.
 * Returns 1 on a non-positive pivot (no factor), else 0.
 */
static int pivoted_cholesky(int k, const real *S, int lds, real *R, int ldr, int *perm, real *W)
{
    for (int c = 0; c < k; ++c) {
        perm[c] = c;
        for (int r = 0; r < k; ++r) W[(size_t)c * k + r] = S[(size_t)c * lds + r];
    }
    for (int c = 0; c < k; ++c)
        for (int r = 0; r < k; ++r) R[(size_t)c * ldr + r] = 0;
    for (int j = 0; j < k; ++j) {
        int t = j;
        for (int i = j + 1; i < k; ++i)
            if (W[(size_t)i * k + i] > W[(size_t)t * k + t]) t = i;
        if (t != j) {   /* symmetric swap of rows and columns j, t of W */
            for (int r = 0; r < k; ++r) {
                real x = W[(size_t)j * k + r];
                W[(size_t)j * k + r] = W[(size_t)t * k + r];
                W[(size_t)t * k + r] = x;
            }
            for (int c = 0; c < k; ++c) {
                real x = W[(size_t)c * k + j];
                W[(size_t)c * k + j] = W[(size_t)c * k + t];
                W[(size_t)c * k + t] = x;
            }
            for (int r = 0; r < j; ++r) {   /* rows of R already formed */
                real x = R[(size_t)j * ldr + r];
                R[(size_t)j * ldr + r] = R[(size_t)t * ldr + r];
                R[(size_t)t * ldr + r] = x;
            }
            int x = perm[j];
            perm[j] = perm[t];
            perm[t] = x;
        }
        real d = W[(size_t)j * k + j];
        if (!(d > 0)) return 1;
        real rjj = R_SQRT(d);
        R[(size_t)j * ldr + j] = rjj;
        for (int l = j + 1; l < k; ++l) R[(size_t)l * ldr + j] = W[(size_t)l * k + j] / rjj;
        for (int l = j + 1; l < k; ++l)
            for (int i = j + 1; i < k; ++i)
                W[(size_t)l * k + i] = W[(size_t)l * k + i] - R[(size_t)i * ldr + j] * R[(size_t)l * ldr + j];
    }
    return 0;
}

/*
 * Alg. 3.3 on the w x w pivot Gram A (column-major, ld w) with signs JP.
 * The columns with j = +1 (in their order) form block 1, those with j = -1
 * block 2 ((3.5)):
 *   P1^T A11 P1 = R11^T R11           (diagonal pivoting)
 *   R11^T R12 = P1^T A12              (forward substitution)
 *   S = A22 - R12^T R12,  P2^T S P2 = R22^T R22   ((3.7))
 *   R_S = [R11, R12 P2; 0, R22], then the columns of its second block
 *   column (and P2) are reversed.
 * Outputs RS (w x w, ld w), perm (position c of R_S holds pivot column
 * perm[c]) and npos; the sign of position c is +1 for c < npos, else -1.
 * Returns 1 if a factorisation broke down, else 0.  W needs 3 w^2 reals,
 * iw 3 w ints.
 */
static int sign_pivoted_cholesky(int w, const real *A, const signed char *JP, real *RS, int *perm,
                                 int *npos_out, real *W, int *iw)
{
    int *pos = iw, *neg = iw + w, *pp = iw + 2 * w;
    int np = 0, nn = 0;
    for (int k = 0; k < w; ++k) {
        if (JP[k] > 0) pos[np++] = k;
        else neg[nn++] = k;
    }
    *npos_out = np;
    real *S = W, *R = W + (size_t)w * w, *work = W + 2 * (size_t)w * w;
    for (int c = 0; c < w; ++c)
        for (int r = 0; r < w; ++r) RS[(size_t)c * w + r] = 0;
    /* R11 */
    for (int c = 0; c < np; ++c)
        for (int r = 0; r < np; ++r) S[(size_t)c * np + r] = A[(size_t)pos[c] * w + pos[r]];
    if (np > 0) {
        if (pivoted_cholesky(np, S, np, R, np, pp, work)) return 1;
        for (int c = 0; c < np; ++c) {
            perm[c] = pos[pp[c]];
            for (int r = 0; r <= c; ++r) RS[(size_t)c * w + r] = R[(size_t)c * np + r];
        }
    }
    /* R12: R11^T X = P1^T A12 (X is np x nn), by forward substitution */
    for (int c = 0; c < nn; ++c)
        for (int r = 0; r < np; ++r) {
            real sum = A[(size_t)neg[c] * w + perm[r]];
            for (int k = 0; k < r; ++k) sum = sum - RS[(size_t)r * w + k] * RS[(size_t)(np + c) * w + k];
            RS[(size_t)(np + c) * w + r] = sum / RS[(size_t)r * w + r];
        }
    /* S = A22 - R12^T R12 */
    for (int c = 0; c < nn; ++c)
        for (int r = 0; r < nn; ++r) {
            real sum = A[(size_t)neg[c] * w + neg[r]];
            for (int k = 0; k < np; ++k)
                sum = sum - RS[(size_t)(np + r) * w + k] * RS[(size_t)(np + c) * w + k];
            S[(size_t)c * nn + r] = sum;
        }
    if (nn > 0) {
        if (pivoted_cholesky(nn, S, nn, R, nn, pp, work)) return 1;
        /* R_S,2 = [R12 P2; R22] with its columns (and P2) reversed */
        real *X = work;   /* R12 before the permutation: np x nn */
        for (int c = 0; c < nn; ++c)
            for (int r = 0; r < np; ++r) X[(size_t)c * np + r] = RS[(size_t)(np + c) * w + r];
        for (int c = 0; c < nn; ++c) {
            const int src = pp[nn - 1 - c];         /* reversed P2 */
            for (int r = 0; r < np; ++r) RS[(size_t)(np + c) * w + r] = X[(size_t)src * np + r];
            for (int r = 0; r < nn; ++r)
                RS[(size_t)(np + c) * w + np + r] = R[(size_t)(nn - 1 - c) * nn + r];
            perm[np + c] = neg[src];
        }
    }
    return 0;
}

/* Test hook: Alg. 3.3 on one w x w Gram. */
int SFX(orc_sp_cholesky)(int w, const double *A, const signed char *JP, double *RS, int *perm,
                         int *npos_out)
{
    if (w < 1 || !A || !JP || !RS || !perm || !npos_out) return ORC_EINVAL;
    real *Ar = (real *)malloc(sizeof(real) * (size_t)w * w);
    real *Rr = (real *)malloc(sizeof(real) * (size_t)w * w);
    real *W = (real *)malloc(sizeof(real) * 3 * (size_t)w * w);
    int *iw = (int *)malloc(sizeof(int) * 3 * (size_t)w);
    int st = ORC_ENOMEM;
    if (Ar && Rr && W && iw) {
        for (size_t e = 0; e < (size_t)w * w; ++e) Ar[e] = (real)A[e];
        st = sign_pivoted_cholesky(w, Ar, JP, Rr, perm, npos_out, W, iw) ? 1 : ORC_OK;
        for (size_t e = 0; e < (size_t)w * w; ++e) RS[e] = (double)Rr[e];
    }
    free(Ar); free(Rr); free(W); free(iw);
    return st;
}

static int block_jevd_impl(int m, int n, double *G, int ldg, const signed char *J, double tol,
                           int b, int full_block, int sign_pivot, int max_sweeps, int max_inner,
                           int accumulate_v, double *lambda, double *V, int ldv,
                           int *sweeps_out, long long *rot_per_sweep,
                           long long *nbreakdown_out, int max_steps, signed char *J_out,
                           int nthreads);

int SFX(orc_block_jevd)(int m, int n, double *G, int ldg, const signed char *J, double tol,
                        int b, int full_block, int max_sweeps, int max_inner,
                        int accumulate_v, double *lambda, double *V, int ldv,
                        int *sweeps_out, long long *rot_per_sweep,
                        long long *nbreakdown_out)
{
    return block_jevd_impl(m, n, G, ldg, J, tol, b, full_block, 0, max_sweeps, max_inner,
                           accumulate_v, lambda, V, ldv, sweeps_out, rot_per_sweep,
                           nbreakdown_out, -1, NULL, 1);
}

/* The same with the sign-pivoted Cholesky of Alg. 3.3 (HBSC / HFSC; for
 * J = I the diagonally pivoted Cholesky).  The pivoting permutes the
 * columns of each transformed pivot block and their signs; J_out (n, may be
 * NULL) receives the final signs, and lambda_i carries them. */
int SFX(orc_block_jevd_sp)(int m, int n, double *G, int ldg, const signed char *J, double tol,
                           int b, int full_block, int max_sweeps, int max_inner,
                           int accumulate_v, double *lambda, double *V, int ldv,
                           int *sweeps_out, long long *rot_per_sweep,
                           long long *nbreakdown_out, signed char *J_out)
{
    return block_jevd_impl(m, n, G, ldg, J, tol, b, full_block, 1, max_sweeps, max_inner,
                           accumulate_v, lambda, V, ldv, sweeps_out, rot_per_sweep,
                           nbreakdown_out, -1, J_out, 1);
}

/* The first max_steps outer steps of the first sweep only: a bounded sample
 * of the block algorithm's work, used to time the oracle on inputs too large
 * to solve on the CPU.  G receives the iterate after those steps.  Returns
 * the status of the partial run.  nthreads as for orc_block_jevd_mt. */
int SFX(orc_block_steps)(int m, int n, double *G, int ldg, const signed char *J, double tol,
                         int b, int full_block, int max_inner, int max_steps, int sign_pivot,
                         int nthreads)
{
    int sweeps = 0;
    return block_jevd_impl(m, n, G, ldg, J, tol, b, full_block, sign_pivot, 1, max_inner, 0, NULL,
                           NULL, n, &sweeps, NULL, NULL, max_steps, NULL, nthreads);
}

/* orc_block_jevd / orc_block_jevd_sp with the pivots of each outer step
 * spread over nthreads threads (<= 0: all).  The pivots of a step touch
 * disjoint columns of G and V (Sec. 3: the processes of a step work on
 * disjoint block pairs), and each pivot runs the same operations in the same
 * order as in the sequential routine, so on finite data the results are bit
 * for bit those of orc_block_jevd (a non-finite Gram may stop a different
 * set of pivots in that step; the status is the same). */
int SFX(orc_block_jevd_mt)(int m, int n, double *G, int ldg, const signed char *J, double tol,
                           int b, int full_block, int sign_pivot, int max_sweeps, int max_inner,
                           int accumulate_v, double *lambda, double *V, int ldv,
                           int *sweeps_out, long long *rot_per_sweep,
                           long long *nbreakdown_out, signed char *J_out, int nthreads)
{
    return block_jevd_impl(m, n, G, ldg, J, tol, b, full_block, sign_pivot, max_sweeps, max_inner,
                           accumulate_v, lambda, V, ldv, sweeps_out, rot_per_sweep,
                           nbreakdown_out, -1, J_out, nthreads);
}

/* Work arrays of one pivot (one set per thread). */
typedef struct {
    real *GP, *VB, *AP, *R, *VP, *SW, *VQ;
    signed char *JP, *JS;
    int *colp, *perm, *iw, *istart, *ipairs;
} pivot_work;

static void pivot_work_free(pivot_work *w)
{
    free(w->GP); free(w->VB); free(w->AP); free(w->R); free(w->VP); free(w->SW); free(w->VQ);
    free(w->JP); free(w->JS); free(w->colp); free(w->perm); free(w->iw); free(w->istart);
    free(w->ipairs);
    memset(w, 0, sizeof(*w));
}

static int pivot_work_alloc(pivot_work *w, int m, int n, int wmax)
{
    int maxp = wmax * wmax;                   /* bound on inner pair counts */
    memset(w, 0, sizeof(*w));
    w->GP = (real *)malloc(sizeof(real) * (size_t)m * wmax);
    w->VB = (real *)malloc(sizeof(real) * (size_t)n * wmax);
    w->AP = (real *)malloc(sizeof(real) * (size_t)wmax * wmax);
    w->R = (real *)malloc(sizeof(real) * (size_t)wmax * wmax);
    w->VP = (real *)malloc(sizeof(real) * (size_t)wmax * wmax);
    w->SW = (real *)malloc(sizeof(real) * 3 * (size_t)wmax * wmax);
    w->VQ = (real *)malloc(sizeof(real) * (size_t)wmax * wmax);
    w->JP = (signed char *)malloc((size_t)wmax);
    w->JS = (signed char *)malloc((size_t)wmax);
    w->colp = (int *)malloc(sizeof(int) * (size_t)wmax);
    w->perm = (int *)malloc(sizeof(int) * (size_t)wmax);
    w->iw = (int *)malloc(sizeof(int) * 3 * (size_t)wmax);
    w->istart = (int *)malloc(sizeof(int) * (size_t)(wmax + 1));
    w->ipairs = (int *)malloc(sizeof(int) * 2 * (size_t)maxp);
    if (!w->GP || !w->VB || !w->AP || !w->R || !w->VP || !w->SW || !w->VQ || !w->JP || !w->JS ||
        !w->colp || !w->perm || !w->iw || !w->istart || !w->ipairs) {
        pivot_work_free(w);
        return ORC_ENOMEM;
    }
    return ORC_OK;
}

/* Steps 1-5 above on the pivot block (I, J) = (blocks bi, bj) of the iterate
 * Gr (m x n, ld m) and Vr (n x n, ld n, may be NULL); Jc holds the current
 * column signs.  all_pairs: the inner sweep covers all pairs (full block, or
 * the first step of a block-oriented sweep).  Adds the pivot's rotations,
 * clamps and breakdowns to the counters; sets *bad on a non-finite Gram
 * (then G and V are left as they were for this pivot). */
static void block_pivot(int m, int n, real *Gr, real *Vr, signed char *Jc, const int *bstart,
                        int bi, int bj, int all_pairs, int full_block, int sign_pivot,
                        int max_inner, real tol, pivot_work *pw, long long *rot,
                        long long *nclamp, long long *nbreak, int *bad)
{
    real *GP = pw->GP, *VB = pw->VB, *AP = pw->AP, *R = pw->R, *VP = pw->VP, *VQ = pw->VQ;
    signed char *JP = pw->JP, *JS = pw->JS;
    int *colp = pw->colp, *perm = pw->perm;
    int wi = bstart[bi + 1] - bstart[bi], wj = bstart[bj + 1] - bstart[bj];
    int w = wi + wj;
    for (int k = 0; k < wi; ++k) colp[k] = bstart[bi] + k;
    for (int k = 0; k < wj; ++k) colp[wi + k] = bstart[bj] + k;
    for (int k = 0; k < w; ++k) {
        JP[k] = Jc[colp[k]];
        memcpy(GP + (size_t)k * m, Gr + (size_t)colp[k] * m, sizeof(real) * (size_t)m);
    }
    /* 1. pivot Gram, each entry summed over the rows in order; a_kl and a_lk
     * are the same sum of the same products (x y = y x), so each is formed
     * once and mirrored; up to four entries of a row of A_P are summed side
     * by side (independent sums, each in its own order) */
    for (int k = 0; k < w; ++k)
        for (int l0 = k; l0 < w; l0 += 4) {
            const int nl = (w - l0 < 4) ? w - l0 : 4;
            const real *x = GP + (size_t)k * m;
            const real *y0 = GP + (size_t)l0 * m;
            real acc[4] = {0, 0, 0, 0};
            if (nl == 4) {
                for (int r = 0; r < m; ++r) {
                    acc[0] = acc[0] + x[r] * y0[r];
                    acc[1] = acc[1] + x[r] * y0[(size_t)m + r];
                    acc[2] = acc[2] + x[r] * y0[2 * (size_t)m + r];
                    acc[3] = acc[3] + x[r] * y0[3 * (size_t)m + r];
                }
            } else {
                for (int q = 0; q < nl; ++q)
                    for (int r = 0; r < m; ++r) acc[q] = acc[q] + x[r] * y0[(size_t)q * m + r];
            }
            for (int q = 0; q < nl; ++q) {
                AP[(size_t)(l0 + q) * w + k] = acc[q];
                AP[(size_t)k * w + l0 + q] = acc[q];
            }
        }
    /* 2. skip test on the targeted entries */
    int need = 0;
    for (int k = 0; k < w; ++k)
        for (int l = k + 1; l < w; ++l) {
            if (!all_pairs && !(k < wi && l >= wi)) continue;
            real akk = AP[(size_t)k * w + k], all = AP[(size_t)l * w + l];
            real akl = AP[(size_t)l * w + k];
            if (!is_finite_r(akk) || !is_finite_r(all) || !is_finite_r(akl)) {
                *bad = 1;
                return;
            }
            if (akk != 0 && all != 0 && R_FABS(akl) > tol * R_SQRT(akk) * R_SQRT(all))
                need = 1;
        }
    if (!need) return;
    /* 3. Cholesky A_P = R^T R (upper R, column-major w x w); with sign
     * pivoting P^T A_P P = R_S^T R_S (Alg. 3.3) and the inner signs become
     * those of the permuted positions */
    int broke = 0, npos = 0;
    for (int k = 0; k < w; ++k) { perm[k] = k; JS[k] = JP[k]; }
    if (sign_pivot) {
        broke = sign_pivoted_cholesky(w, AP, JP, R, perm, &npos, pw->SW, pw->iw);
        if (broke) {
            for (int k = 0; k < w; ++k) perm[k] = k;
        } else {
            for (int k = 0; k < w; ++k) JS[k] = (k < npos) ? 1 : -1;
        }
    }
    for (int j = 0; j < w && !broke && !sign_pivot; ++j) {
        for (int i = 0; i <= j; ++i) {
            real sum = AP[(size_t)j * w + i];
            for (int k = 0; k < i; ++k)
                sum = sum - R[(size_t)i * w + k] * R[(size_t)j * w + k];
            if (i == j) {
                if (!(sum > 0)) { broke = 1; break; }
                R[(size_t)j * w + j] = R_SQRT(sum);
            } else {
                R[(size_t)j * w + i] = sum / R[(size_t)i * w + i];
            }
        }
        for (int i = j + 1; i < w; ++i) R[(size_t)j * w + i] = 0;
    }
    if (broke) ++*nbreak;
    /* 4. inner one-sided Jacobi on R (or on G_P after a breakdown) */
    real *X = broke ? GP : R;
    int ldx = broke ? m : w, len = broke ? m : w;
    for (int k = 0; k < w; ++k)
        for (int l = 0; l < w; ++l) VP[(size_t)k * w + l] = (real)(k == l ? 1 : 0);
    long long prot = 0;
    int isteps, inp = 0;
    if (all_pairs) {
        isteps = orc_ordering(w, 2, pw->istart, pw->ipairs, &inp);
    } else {
        isteps = cross_ordering(wi, wj, pw->istart, pw->ipairs);
    }
    int inner = full_block ? max_inner : 1;
    for (int it = 0; it < inner; ++it) {
        long long r = inner_sweep(X, ldx, len, VP, w, pw->istart, pw->ipairs, isteps,
                                  broke ? JP : JS, tol, nclamp, bad);
        prot += r;
        if (*bad || r == 0) break;
    }
    if (*bad) return;
    *rot += prot;
    if (prot == 0) return;
    /* 5. update G_P <- G_P V_P, V(:,P) <- V(:,P) V_P.  After a breakdown
     * G_P was transformed in place and is copied back.  With sign pivoting
     * V_P = P V': the permutation is applied to the rows of the accumulated
     * V' (Alg. 3.4), and column c of the block takes the sign of position c.
     * Each entry of a product is the sum over k = 0..w-1 in that order; the
     * loops run over the rows innermost (the sums themselves are unchanged). */
    if (sign_pivot && !broke) {
        memcpy(VQ, VP, sizeof(real) * (size_t)w * w);
        for (int c = 0; c < w; ++c)
            for (int r = 0; r < w; ++r) VP[(size_t)c * w + perm[r]] = VQ[(size_t)c * w + r];
        for (int c = 0; c < w; ++c) Jc[colp[c]] = JS[c];
    }
    if (broke) {
        for (int c = 0; c < w; ++c)
            memcpy(Gr + (size_t)colp[c] * m, GP + (size_t)c * m, sizeof(real) * (size_t)m);
    } else {
        for (int c = 0; c < w; ++c) {
            real *out = Gr + (size_t)colp[c] * m;
            for (int r = 0; r < m; ++r) out[r] = 0;
            for (int k = 0; k < w; ++k) {
                const real v = VP[(size_t)c * w + k], *in = GP + (size_t)k * m;
                for (int r = 0; r < m; ++r) out[r] = out[r] + in[r] * v;
            }
        }
    }
    if (Vr) {
        for (int k = 0; k < w; ++k)
            memcpy(VB + (size_t)k * n, Vr + (size_t)colp[k] * n, sizeof(real) * (size_t)n);
        for (int c = 0; c < w; ++c) {
            real *out = Vr + (size_t)colp[c] * n;
            for (int r = 0; r < n; ++r) out[r] = 0;
            for (int k = 0; k < w; ++k) {
                const real v = VP[(size_t)c * w + k], *in = VB + (size_t)k * n;
                for (int r = 0; r < n; ++r) out[r] = out[r] + in[r] * v;
            }
        }
    }
}

static int block_jevd_impl(int m, int n, double *G, int ldg, const signed char *J, double tol,
                           int b, int full_block, int sign_pivot, int max_sweeps, int max_inner,
                           int accumulate_v, double *lambda, double *V, int ldv,
                           int *sweeps_out, long long *rot_per_sweep,
                           long long *nbreakdown_out, int max_steps, signed char *J_out,
                           int nthreads)
{
    int st = check_args(m, n, ldg, J, ldv, V);
    if (st) return st;
    if (b < 1 || max_sweeps < 1 || max_inner < 1) return ORC_EINVAL;
    int N = 2 * ((n + 2 * b - 1) / (2 * b));
    if (N > n) return ORC_EINVAL;             /* every block needs a column */
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_num_procs();
#else
    nthreads = 1;
#endif
    if (nthreads > N / 2) nthreads = N / 2;   /* pivots per step */
    if (nthreads < 1) nthreads = 1;
    int *bstart = (int *)malloc(sizeof(int) * (size_t)(N + 1));
    int onp = 0;
    int ons = orc_ordering(N, 2, NULL, NULL, &onp);
    int *ostart = (int *)malloc(sizeof(int) * (size_t)(ons + 1));
    int *opairs = (int *)malloc(sizeof(int) * 2 * (size_t)onp);
    int wmax = 2 * (n / N + 1);
    real *Gr = (real *)malloc(sizeof(real) * (size_t)m * n);
    real *Vr = V ? (real *)malloc(sizeof(real) * (size_t)n * n) : NULL;
    signed char *Jc = (signed char *)malloc((size_t)n);
    pivot_work *pw = (pivot_work *)calloc((size_t)nthreads, sizeof(pivot_work));
    int ok = bstart && ostart && opairs && Gr && (!V || Vr) && Jc && pw;
    for (int t = 0; ok && t < nthreads; ++t)
        if (pivot_work_alloc(&pw[t], m, n, wmax)) ok = 0;
    if (!ok) {
        st = ORC_ENOMEM;
        goto out;
    }
    orc_ordering(N, 2, ostart, opairs, NULL);
    for (int i = 0; i < n; ++i) Jc[i] = (J && J[i] < 0) ? -1 : 1;
    bstart[0] = 0;
    for (int k = 0; k < N; ++k) bstart[k + 1] = bstart[k] + n / N + (k < n % N ? 1 : 0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < m; ++k) Gr[(size_t)i * m + k] = (real)G[(size_t)i * ldg + k];
    if (Vr)
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k)
                Vr[(size_t)i * n + k] = accumulate_v ? (real)V[(size_t)i * ldv + k]
                                                     : (real)(i == k ? 1 : 0);
    long long nclamp = 0, nbreak = 0;
    int sweeps = 0;
    st = ORC_ENOCONV;
    while (sweeps < max_sweeps) {
        long long rot = 0;
        int bad = 0;
        ++sweeps;
        for (int sidx = 0; sidx < ons && !bad && (max_steps < 0 || sidx < max_steps); ++sidx) {
            const int e0 = ostart[sidx], e1 = ostart[sidx + 1];
            const int all_pairs = full_block || sidx == 0;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static, 1) \
    reduction(+ : rot, nclamp, nbreak) reduction(| : bad)
#endif
            for (int e = e0; e < e1; ++e) {
                int t = 0;
#ifdef _OPENMP
                t = omp_get_thread_num();
#endif
                /* in a sequential run a non-finite Gram ends the step at once */
                if (nthreads == 1 && bad) continue;
                block_pivot(m, n, Gr, Vr, Jc, bstart, opairs[2 * e], opairs[2 * e + 1],
                            all_pairs, full_block, sign_pivot, max_inner, (real)tol, &pw[t],
                            &rot, &nclamp, &nbreak, &bad);
            }
        }
        if (rot_per_sweep) rot_per_sweep[sweeps - 1] = rot;
        if (bad) { st = ORC_ENONFINITE; break; }
        if (rot == 0) { st = ORC_OK; break; }
    }
    finalize(m, n, Gr, Jc, G, ldg, lambda);
    if (J_out) memcpy(J_out, Jc, (size_t)n);
    if (Vr)
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) V[(size_t)i * ldv + k] = (double)Vr[(size_t)i * n + k];
    if (sweeps_out) *sweeps_out = sweeps;
    if (nbreakdown_out) *nbreakdown_out = nbreak;
out:
    for (int t = 0; pw && t < nthreads; ++t) pivot_work_free(&pw[t]);
    free(pw); free(bstart); free(ostart); free(opairs); free(Gr); free(Vr); free(Jc);
    return st;
}
