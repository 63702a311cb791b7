/*
 * jevd.h -- one-sided Jacobi eigensolver for AMD MI355X (gfx950): C ABI.
 *
 * Problem (Sec. 1, (1.3) and the hyperbolic SVD defined right after it):
 * H = G J G^T is given by a factor G (m x n, m >= n, full column rank) and a
 * signature J = diag(j_1..j_n), j_i in {+1, -1}.  The library finds V with
 * V^T J V = J such that the columns of G V are mutually orthogonal; then the
 * eigenvalues of H are lambda_i = j_i ||(G V)_i||^2 (Sec. 1: squared column
 * norms of the final factor) and its eigenvectors are the normalised
 * columns u_i = (G V)_i / ||(G V)_i|| (Sec. 3.2).  J = I is the positive
 * definite, purely trigonometric case H = G G^T.
 *
 * The method is the one-sided Jacobi sweep (Sec. 2.1): pivot pairs of
 * columns (pointwise) or of block columns (Sec. 2.2-2.3, block-oriented or
 * full block, with the Gram of the pivot block factored by Cholesky and the
 * accumulated transform applied once per pivot) are orthogonalised by
 * trigonometric rotations when their signs in J agree and by hyperbolic
 * ones otherwise, in the row-cyclic, modulus or modified modulus ordering
 * (Sec. 2.4, Alg. 3.1).  A pair is rotated only when
 * |a_pq| > tol * sqrt(a_pp) * sqrt(a_qq) for its Gram entries; the iteration
 * stops after the first sweep that rotates nothing.
 *
 * Conventions for every entry point:
 *   - matrices are column-major FP64; element (r, c) of X is X[r + c * ldx];
 *   - G, lambda, U and V are DEVICE pointers (memory of the device that is
 *     current when the handle is created); J is a HOST pointer;
 *   - the caller owns every buffer; a handle owns only its workspace;
 *   - all work is ordered on the handle's stream; the solver synchronises
 *     that stream once per sweep (to read the rotation count) and before
 *     returning, so outputs are ready when the call returns;
 *   - no C++ exception crosses the ABI; every function returns a status.
 */
#ifndef JEVD_H
#define JEVD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jevd_handle_s *jevd_handle_t;

/* Status codes. */
enum {
    JEVD_OK = 0,
    JEVD_EINVAL = -1,      /* bad argument; detected before any device work */
    JEVD_ENONFINITE = -2,  /* a NaN or Inf appeared in a Gram entry */
    JEVD_ENOCONV = -3,     /* max_sweeps reached; outputs hold the current iterate */
    JEVD_EHIP = -4,        /* a HIP runtime call failed (no device, launch error, ...) */
    JEVD_ENOMEM = -5       /* device or pinned host allocation failed */
};

/* Pivot orderings (Sec. 2.4, Fig. 2-3, Alg. 3.1). */
enum {
    JEVD_ORD_ROWCYCLIC = 0,   /* (1,2),(1,3),...,(n-1,n); the result of one pair at a
                                 time, run as the 2n - 3 steps of equal i + j */
    JEVD_ORD_MODULUS = 1,     /* step k: all pairs with i + j == k (mod n) */
    JEVD_ORD_MODMODULUS = 2   /* modulus plus the pair of the two idle indices on even steps (default) */
};

/* Variants (Sec. 2.1-2.2). */
enum {
    JEVD_VAR_POINTWISE = 0,       /* 2x2 pivots on single columns */
    JEVD_VAR_BLOCK_ORIENTED = 1,  /* block pivots; annihilate each entry of A_IJ once per step */
    JEVD_VAR_FULL_BLOCK = 2,      /* block pivots; diagonalise every pivot block */
    JEVD_VAR_AUTO = 3             /* the variant jevd_autotune recorded for (m, n); when
                                     the shape has not been tuned, pointwise for n < 2048
                                     and block-oriented from n = 2048 on */
};

typedef struct {
    int ordering;      /* JEVD_ORD_*; default JEVD_ORD_MODMODULUS.  Block variants
                          always order block pairs by the modified modulus ordering. */
    int variant;       /* JEVD_VAR_*; default JEVD_VAR_AUTO */
    int block;         /* block width b of the block variants: 16, 32 or 64 (64 only
                          with JEVD_PIVOT_NONE); 0: the width jevd_autotune recorded
                          for (m, n), else 64 for n >= 4096, 32 for n >= 512, 16
                          below.  The n columns form N = 2 ceil(n / 2b) blocks whose
                          widths differ by at most one (Sec. 3); any n >= 2 with
                          N <= n is accepted, sign pivoting needs n divisible by 2b. */
    int max_sweeps;    /* sweep limit, default 50 (>= 1) */
    int max_inner;     /* full block: inner sweep limit per pivot, default 30 */
    int accumulate_v;  /* 0: V := I before the first sweep; 1: V holds a prior
                          transform on entry (resume from an earlier iterate) */
    int pivot;         /* JEVD_PIVOT_*; default JEVD_PIVOT_NONE */
    int precision;     /* JEVD_PREC_*; default JEVD_PREC_FP64 */
} jevd_opts;

/* Arithmetic of the block sweeps. */
enum {
    JEVD_PREC_FP64 = 0,   /* every sweep in FP64 */
    JEVD_PREC_MIXED = 1   /* block sweeps on an FP32 copy of G (FP32 MFMA Gram and update;
                             Cholesky, rotation angles and the skip test in FP64) at the
                             threshold tol_low = max(tol, 8 sqrt(m) 2^-24), until a sweep
                             rotates nothing there or max_sweeps; then the FP32 transform is
                             made orthogonal in FP64 (Newton-Schulz), G <- G V0 in FP64, and
                             FP64 block sweeps finish at tol.  Requires a block variant,
                             J = I and accumulate_v = 0; V may be NULL (a work array is used).
                             jevd_info.sweeps_low counts the FP32 sweeps; sweeps the FP64 ones. */
};

/* Cholesky factorisation of the pivot Grams of the block variants. */
enum {
    JEVD_PIVOT_NONE = 0,  /* unpivoted (HB / HF, and the trigonometric block variants) */
    JEVD_PIVOT_SIGN = 1   /* sign-pivoted, Alg. 3.3 (HBSC / HFSC; diagonal pivoting for J = I).
                             Requires JEVD_VAR_BLOCK_ORIENTED or JEVD_VAR_FULL_BLOCK.  The
                             pivoting permutes the columns of each transformed pivot block,
                             positive signs first: on return column i of G, U, V carries the
                             sign of lambda_i, which may differ from J[i], and V satisfies
                             V^T J V = diag(sign(lambda)). */
};

/* Per-call diagnostics of the last jacobi_evd on a handle. */
#define JEVD_INFO_MAX_SWEEPS 64
/* Kernel classes of the per-kernel timings. */
enum {
    JEVD_K_PAIR_STEP = 0,    /* pointwise: one parallel step (or the one-workgroup solve) */
    JEVD_K_GRAM = 1,         /* block: pivot Grams G_P^T G_P */
    JEVD_K_PIVOT_SOLVE = 2,  /* block: Cholesky + inner sweeps per pivot */
    JEVD_K_UPDATE = 3,       /* block: G_P <- G_P V_P and V(:,P) <- V(:,P) V_P;
                                pointwise: V updated from the rotation log */
    JEVD_K_CLASSES = 4
};
typedef struct {
    int sweeps;                                    /* same as the *sweeps output */
    int variant;                                   /* variant actually run */
    int block;                                     /* block width used (0: pointwise) */
    int ordering;                                  /* ordering actually run */
    long long rotations[JEVD_INFO_MAX_SWEEPS];     /* rotations applied per sweep */
    long long clamps;                              /* hyperbolic transforms clamped to |tanh| = 0.9 */
    long long breakdowns;                          /* block pivots whose Cholesky broke down */
    /* Filled only when timing is on (jevd_set_timing): summed HIP-event
     * durations of each kernel class and the number of its launches. */
    double kernel_ms[JEVD_K_CLASSES];
    long long kernel_launches[JEVD_K_CLASSES];
    int sweeps_low;    /* JEVD_PREC_MIXED: FP32 sweeps before the FP64 ones */
    int v_deferred;    /* pointwise with V: 1 when the steps logged their rotations
                          and V was updated from the log (timed as JEVD_K_UPDATE),
                          0 when each step rotated its two columns of V */
    int steps_per_launch;  /* pointwise, one launch per step (not the single-
                              workgroup solve): steps of the ordering per launch,
                              1, or 2 for the ring of Alg. 3.1 (modified
                              modulus, n a multiple of 4, 512 < m <= 1024),
                              whose launches give the same bits as one step
                              each */
} jevd_info;

/* Fills *o with the defaults listed above.  Never fails for a non-NULL o. */
int jevd_default_opts(jevd_opts *o);

/* Creates a handle bound to the current device and to `stream` (a
 * hipStream_t; NULL means the default stream).  *h receives the handle.
 * Returns JEVD_EINVAL for h == NULL, JEVD_EHIP if no device is usable. */
int jevd_create(jevd_handle_t *h, void *stream);

/* Frees the handle's workspace.  NULL is accepted. */
int jevd_destroy(jevd_handle_t h);

/*
 * jacobi_evd: one-sided Jacobi eigensolver, H = G J G^T.
 *   m, n     G is m x n with m >= n >= 1; ldg >= m.
 *   G        device, in/out.  On return it holds the final iterate G V
 *            (orthogonal columns, U Sigma).  Overwritten in place (Sec. 3.2).
 *   J        host, n entries each +1 or -1; NULL means J = I.
 *   tol      rotation threshold; <= 0 means n * DBL_EPSILON.
 *   opts     NULL means jevd_default_opts.
 *   lambda   device, n outputs lambda_i = j_i ||g_i||^2 of the final
 *            iterate, in column order (not sorted); may be NULL.
 *   U, ldu   device, m x n outputs u_i = g_i / ||g_i|| (zero column -> 0);
 *            U may equal G (then G is normalised in place); may be NULL.
 *   V, ldv   device, n x n, the accumulated J-orthogonal transform
 *            (G_out = G_in V); in/out when opts->accumulate_v; may be NULL
 *            (then V is not formed, which saves its traffic).
 *   sweeps   host, receives the sweeps executed, including the final sweep
 *            that rotates nothing; may be NULL.
 * Returns JEVD_OK, JEVD_EINVAL (before any device work: m < n, n < 1,
 * leading dimension too small, J entry not +-1, bad option), JEVD_ENONFINITE,
 * JEVD_ENOCONV (after max_sweeps sweeps; G, lambda, U and V hold the current
 * iterate, so a later call with accumulate_v = 1 resumes), JEVD_EHIP or
 * JEVD_ENOMEM.  Buffers must not overlap except U == G.
 */
int jacobi_evd(jevd_handle_t h, int m, int n, double *G, int ldg, const signed char *J,
               double tol, const jevd_opts *opts, double *lambda, double *U, int ldu,
               double *V, int ldv, int *sweeps);

/*
 * Batched solves: many independent instances H_i = G_i J_i G_i^T, each
 * treated exactly as jacobi_evd treats one (pointwise sweeps, the ordering,
 * tolerance and sweep limit of opts), in one persistent launch (Sec. 2.4:
 * instances, like disjoint pivots, are independent).  Meant for many small
 * and medium problems (n up to a few hundred; n_i <= 4096).
 *
 * jevd_batch_create validates every instance (the rules of jacobi_evd;
 * JEVD_EINVAL before any device work), copies the J_i to the device and
 * uploads one descriptor per instance, queued largest first.  All pointer
 * arrays are HOST arrays of length batch: G, lambda, U, V hold DEVICE
 * pointers (lambda, U, V arrays or entries may be NULL), J holds HOST
 * pointers to n_i signs (J or an entry NULL: J = I), tol holds per-instance
 * tolerances (NULL or an entry <= 0: n_i * DBL_EPSILON).  opts->variant must
 * be JEVD_VAR_POINTWISE or JEVD_VAR_AUTO.  The plan refers to the caller's
 * buffers; they must stay valid while it is run.
 * The instances are grouped by size into JEVD_BATCH_CLASSES classes
 * (n <= 48, <= 96, <= 141, larger), each run with workgroups of 4, 8 or 16
 * wavefronts (4, 2 or 1 instances at a time per CU, with that share of its
 * LDS): the size jevd_batch_autotune measured fastest for the class on this
 * machine when the class's per-step arrays fit that share and the class has
 * more instances than the device has CUs, else 16.
 * Consecutive classes of one size share a persistent launch (largest
 * instances first); the largest class's launch runs on `stream`, the others
 * at the same time on a second stream of the plan.
 * jevd_batch_run enqueues the solve of all instances on `stream` (a
 * hipStream_t; NULL: the handle's stream) and returns at once: it launches
 * two kernels per launch group and, with more than one group, records two
 * events (the second stream waits for `stream`'s prior work, and `stream`
 * for the second stream's launches), so it may be captured in a HIP graph
 * and replayed.  Each run restarts from the current contents of the G_i.
 * jevd_batch_results waits for the stream of the last run and copies out
 * the per-instance sweep counts and statuses (JEVD_OK, JEVD_ENOCONV,
 * JEVD_ENONFINITE); either array may be NULL.  It returns JEVD_OK if every
 * instance converged, else the first failing instance's status.
 * Plans of one handle may not run concurrently, and are destroyed before
 * the handle.  A destroyed plan's device arrays are kept by the handle for
 * the next plan (no allocation when they are large enough).
 */
typedef struct jevd_batch_s *jevd_batch_t;

int jevd_batch_create(jevd_handle_t h, int batch, const int *m, const int *n,
                      double *const *G, const int *ldg, const signed char *const *J,
                      const double *tol, const jevd_opts *opts, double *const *lambda,
                      double *const *U, const int *ldu, double *const *V, const int *ldv,
                      jevd_batch_t *plan);
int jevd_batch_run(jevd_batch_t plan, void *stream);
int jevd_batch_results(jevd_batch_t plan, int *sweeps, int *status);
int jevd_batch_destroy(jevd_batch_t plan);

/* create + run on the handle's stream + results + destroy. */
int jacobi_evd_batched(jevd_handle_t h, int batch, const int *m, const int *n,
                       double *const *G, const int *ldg, const signed char *const *J,
                       const double *tol, const jevd_opts *opts, double *const *lambda,
                       double *const *U, const int *ldu, double *const *V, const int *ldv,
                       int *sweeps, int *status);

#define JEVD_BATCH_CLASSES 4

/* The workgroup size (wavefronts) each class of a plan runs with, 0 for an
 * empty class: waves[JEVD_BATCH_CLASSES].  Host-only.  JEVD_EINVAL for NULL
 * arguments. */
int jevd_batch_waves(jevd_batch_t plan, int *waves);

/* Measures, for each size class, a batch of seeded instances of a
 * representative size (n = 40, 80, 128, 192; m = n; columns graded over two
 * decades; J = I; V formed if want_v) with each workgroup size whose LDS
 * share holds the class's step arrays (4, 8, 16 wavefronts), and records the
 * fastest in the autotuner's table on the machine (the file of
 * jevd_tune_file), where jevd_batch_create finds it.  waves_out (NULL or
 * JEVD_BATCH_CLASSES entries) receives the choices.  Allocates and frees
 * device memory (about 0.8 GB at most) and synchronises the handle's stream.
 * JEVD_EINVAL for a NULL h or want_v not 0 or 1; JEVD_ENOMEM / JEVD_EHIP on
 * device failures.  An unwritable table file is not an error. */
int jevd_batch_autotune(jevd_handle_t h, int want_v, int *waves_out);

/* The table's record for a size class (host-only): JEVD_EINVAL if none. */
int jevd_batch_tune_lookup(int size_class, int *waves, double *ms);

/* Records a size class's workgroup size (4, 8 or 16) and time in the table
 * and rewrites its file; JEVD_EINVAL for a class outside
 * [0, JEVD_BATCH_CLASSES), another size, or a negative time. */
int jevd_batch_tune_record(int size_class, int waves, double ms);

/*
 * Canonical outputs and the adjoint, for `batch` instances of one shape
 * m x n (1 <= n <= m), stored column-major at fixed strides: instance b of
 * an array X with leading dimension ldx and batch stride sx starts at
 * X + b * sx (sx >= ldx * n; for lam, w: >= n).  All pointers are DEVICE
 * pointers; both calls only enqueue work on the handle's stream (no
 * synchronisation, no host transfers) and return JEVD_EINVAL on bad sizes,
 * JEVD_ENOMEM / JEVD_EHIP on device errors.
 *
 * jevd_canonicalize: writes a canonical form of solver outputs (lam, U and
 * optionally V, as left by jacobi_evd or a batch plan): eigenpairs sorted by
 * decreasing lambda (equal values by position; NaN ordered as -inf), each
 * u_i signed so that its entry of largest magnitude (the first such) is
 * positive, v_i signed and moved with it.  The outputs use the same leading
 * dimensions and strides and must not overlap the inputs.  The order and
 * signs the iteration leaves depend on its rotation sequence; the canonical
 * form makes (lam, U) a locally smooth function of G for a simple spectrum.
 *
 * jevd_adjoint: dG = dL/dG for L = sum_i w_i lambda_i + <C, U>, given the
 * input G and J of H = G J G^T and the canonical lam, U of its solve (Sec. 1
 * and Sec. 2.1; first-order perturbation theory of a symmetric matrix with
 * a simple spectrum, pulled back through dH = dG J G^T + G J dG^T):
 *   dG = [U M' + (m > n ? C Lambda^{-1} : 0)] W J,  W = U^T G,  K = U^T C,
 *   M'_ki = (K_ki - K_ik) / (lambda_i - lambda_k)  (k != i),  M'_ii = 2 w_i,
 *   and, if m > n, minus K_ki / lambda_i in every entry.
 * J here is a DEVICE array of n int8 signs per instance (batch stride sj >=
 * n), or NULL for J = I.  w or C may be NULL (zero).  The spectrum must be
 * simple and, for m > n, nonzero; otherwise the result holds infinities.
 * dG (ldd >= m) must not overlap the inputs.  Work arrays (3 n^2 + m n
 * doubles per instance) are kept by the handle; the first call at a larger
 * size allocates them (so it cannot be captured in a graph).
 */
int jevd_canonicalize(jevd_handle_t h, int batch, int m, int n, const double *lam, long long slam,
                      const double *U, int ldu, long long su, const double *V, int ldv,
                      long long sv, double *lam_out, double *U_out, double *V_out);
int jevd_adjoint(jevd_handle_t h, int batch, int m, int n, const double *G, int ldg, long long sg,
                 const signed char *J, long long sj, const double *lam, long long slam,
                 const double *U, int ldu, long long su, const double *w, long long sw,
                 const double *C, int ldc, long long sc, double *dG, int ldd, long long sd);

/*
 * Autotuning of the block width and variant (Conclusion: the switching point
 * between algorithms and block sizes is found by profiling on the machine,
 * as self-tuning packages do).  jevd_autotune solves a working copy of the
 * caller's G (device, m x n, ld ldg; not modified) with J, tol and opts
 * (pivot and precision are kept; variant, block and accumulate_v are
 * varied/ignored) once for each candidate -- pointwise (FP64 without
 * pivoting, n <= 2048 only), and block-oriented and full block at every
 * admissible b in {16, 32, 64} (b = 16 for n <= 2048 only: above that it and
 * the pointwise solve take several times as long as the wider blocks) --
 * forming V when want_v, and records the fastest
 * (wall time to convergence) for (m, n) in the process's tune table, which
 * is also written to the tune file.  *block, *variant, *ms (each may be
 * NULL) receive the winner (block 0 for pointwise).  Returns JEVD_OK,
 * JEVD_EINVAL, JEVD_ENOCONV (no candidate converged), JEVD_EHIP or
 * JEVD_ENOMEM.  Synchronises the handle's stream.
 *
 * The tune table maps (m, n) to (block, variant, ms); jacobi_evd and
 * jevd_validate consult it for opts->block == 0 and JEVD_VAR_AUTO.  The tune
 * file holds one line "m n block variant ms" per shape; it is
 * $JEVD_TUNE_FILE, else $HOME/.cache/jevd_tune.txt.  Host-only, no device
 * work: jevd_tune_file(path) empties the table and loads it from path (NULL:
 * the default file; a missing file gives an empty table); jevd_tune_lookup
 * returns JEVD_OK and the record of (m, n), or JEVD_EINVAL if there is none;
 * jevd_tune_record adds or replaces a record (JEVD_EINVAL for a block width
 * the shape does not admit, a variant other than pointwise with block 0 or
 * a block variant, or ms < 0) and rewrites the file.
 */
int jevd_autotune(jevd_handle_t h, int m, int n, const double *G, int ldg, const signed char *J,
                  double tol, const jevd_opts *opts, int want_v, int *block, int *variant,
                  double *ms);
int jevd_tune_file(const char *path);
int jevd_tune_lookup(int m, int n, int *block, int *variant, double *ms);
int jevd_tune_record(int m, int n, int block, int variant, double ms);

/*
 * jevd_adjoint_noalloc: jevd_adjoint for callers that cannot allocate (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results as jevd_adjoint, but the work arrays
 * (3 n^2 + m n doubles per instance) live in a fixed 32 MiB device array of
 * the library (4194304 doubles; one copy per GPU, set up by jevd_create and
 * held until the process ends) instead of the handle's workspace, so the
 * call never allocates.  Returns JEVD_EINVAL, before any device work, when
 * batch * (3 n^2 + m n) exceeds 4194304 doubles, and for the argument errors
 * of jevd_adjoint.  All calls on one GPU share the array: calls that overlap
 * in time on one GPU (other streams, other threads) race and give wrong
 * results; calls ordered on one stream are safe.  Only enqueues work on the
 * handle's stream.
 */
int jevd_adjoint_noalloc(jevd_handle_t h, int batch, int m, int n, const double *G, int ldg,
                         long long sg, const signed char *J, long long sj, const double *lam,
                         long long slam, const double *U, int ldu, long long su, const double *w,
                         long long sw, const double *C, int ldc, long long sc, double *dG, int ldd,
                         long long sd);

/* Host-only argument check that jacobi_evd runs before any device work
 * (same rules; G, lambda and the handle are not examined).  Returns JEVD_OK
 * or JEVD_EINVAL.  No device work. */
int jevd_validate(int m, int n, int ldg, const signed char *J, double tol, const jevd_opts *opts,
                  const double *U, int ldu, const double *V, int ldv);

/* Turns kernel timing on (1) or off (0) for later calls on h: two HIP
 * events on the handle's stream bracket each timed group of launches (all
 * parallel-step launches of a sweep, or a single block-path launch) and the
 * durations are summed into jevd_info.kernel_ms / kernel_launches.  A
 * group's time includes the dispatch gaps between its launches.  Default off. */
int jevd_set_timing(jevd_handle_t h, int on);

/* Diagnostics of the last jacobi_evd call on h. */
int jevd_get_info(jevd_handle_t h, jevd_info *info);

/* Measurement aid for the roofline of the block path (Sec. 2.2: the block
 * update is a matrix product): the FP64 MFMA rate the GPU of h sustains on
 * independent v_mfma_f64_16x16x4f64 instructions whose operands sit in
 * registers (no memory access inside the loop), with waves_per_simd
 * (1, 2 or 4) wavefronts per SIMD on every CU, each running iters x 8
 * MFMAs.  *tflops receives 2048 x MFMAs / seconds / 1e12 from HIP events on
 * the handle's stream.  Allocates and frees a small result buffer; blocks
 * until done.  JEVD_EINVAL for a NULL h or tflops, waves_per_simd not in
 * {1, 2, 4}, or iters < 1. */
int jevd_mfma_f64_rate(jevd_handle_t h, int waves_per_simd, int iters, double *tflops);

/* Static text for a status code. */
const char *jevd_strerror(int status);

/*
 * Host-only helper: the pivot ordering the solver runs (Sec. 2.4, Alg. 3.1),
 * as 0-based pairs (i < j) grouped in steps, each step's pairs in the order
 * they are dealt to workgroups (for the modified modulus ordering on even n:
 * the processes of the ring of Alg. 3.1, arranged so that neighbouring
 * processes share an XCD; for the row-cyclic ordering: the 2n - 3 steps of
 * pairs with equal i + j, i ascending, in which every column meets its
 * pairs in row order, so that the steps give the result of the pairs one at
 * a time).  step_start (nsteps + 1 ints)
 * and pairs (2 ints per pair) may be NULL to query sizes; *nsteps and
 * *npairs receive the counts.  Pairs of a step are disjoint.  No device work.
 */
int jevd_ordering(int n, int ordering, int *step_start, int *pairs, int *nsteps, int *npairs);

#ifdef __cplusplus
}
#endif

#endif /* JEVD_H */
