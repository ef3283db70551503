/*
 * signtri.h -- U = sign(T) for an upper-triangular T on an AMD MI355X (gfx950).
 *
 * The method is the one of Stotland, Schwartz and Toledo, "High-Performance
 * Algorithms for Computing the Sign Function of Triangular Matrices":
 *
 *   - sign(z) is the sign of Re z (Section 1); sign(T) is undefined when some
 *     diagonal entry has a zero real part (Section 1);
 *   - the Parlett-Higham substitution (Algorithm 3): u_ii = sign(t_ii); for
 *     i < j, Eq. (1) (from TU = UT) where sign(t_ii) != sign(t_jj), Eq. (2)
 *     (from U^2 = I) where they agree; computed here in block form (Section 5:
 *     the block equations with accumulators X and Y, Algorithms 4-6), with
 *     diagonal blocks solved element by element and off-diagonal block
 *     accumulations done as matrix products;
 *   - the Parlett-Sylvester form (Algorithm 2 specialised to the sign, whose
 *     diagonal blocks are +I and -I, Section 2): for a T whose diagonal is
 *     already grouped by sign, U = [[s I, X], [0, -s I]] with
 *     T11 X - X T22 = 2 s T12;
 *   - the choice between them by the work estimates of Section 3, driven by
 *     the inertia of the diagonal.
 *
 * Conventions for every entry point:
 *   - Matrices are dense n x n with a leading dimension ld >= max(1, n), in
 *     column-major (element (i, j) at i + j*ld) or row-major (i*ld + j)
 *     order.  SIGNTRI_C128 elements are interleaved (re, im) doubles and ld
 *     counts complex elements.
 *   - T and U are DEVICE pointers.  The caller owns them; the library never
 *     frees them.  T is never written.  U must not overlap T.
 *   - Only the upper triangle of T (diagonal included) is read; its strict
 *     lower triangle may hold anything.  The whole n x n of U is written: its
 *     upper triangle with sign(T) and its strict lower triangle with zeros.
 *     Padding between n and ld is not touched.
 *   - Work is queued on `stream` (a hipStream_t; NULL means the default
 *     stream).  Single-matrix calls synchronise the stream once, after a
 *     device scan of the diagonal, to plan the work; the result in U is ready
 *     when the stream has been synchronised again.  Calls that also wait for
 *     their result before returning: MIXED_REFINED (it reads the refinement's
 *     outcome once at the end; its convergence tests run on the device),
 *     sign_tri(), signtri_batched(), and signtri() with a non-NULL `info`.  Those calls also return SIGNTRI_EHIP if a dependency
 *     wait of a dataflow sweep hit its safety bound (which does not happen in
 *     a correct run; U then holds unusable values).  signtri() with a NULL
 *     `info` and no refinement returns without waiting and cannot report it.
 *   - Testing hooks, read from the environment at each call:
 *     SIGNTRI_DEBUG_SPIN_LIMIT=<int> sets the polls a dependency wait makes
 *     before it gives up (-1: the first wait of each sweep gives up at once);
 *     SIGNTRI_DEBUG_FAIL_ALLOC=1 makes every allocation of the library-owned
 *     workspace fail with SIGNTRI_ENOMEM.
 *   - signtri_dtype, signtri_mode, signtri_algo and signtri_layout are
 *     int32_t with the named constants below, so that any value a caller
 *     passes is a valid argument and is checked (-p when out of range).
 *   - Return codes: 0 on success; -p if argument p (1-based) is invalid;
 *     positive SIGNTRI_E* codes below.  On any nonzero return, U is untouched
 *     except after SIGNTRI_EHIP (a device error mid-computation).
 */
#ifndef SIGNTRI_H
#define SIGNTRI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t signtri_dtype;
enum { SIGNTRI_R64 = 0, SIGNTRI_C128 = 1 };

/* FP64: every operation in FP64 (complex128).
 * MIXED_REFINED: bulk products on FP32 MFMA with FP32 accumulation, divisions by
 *   t_ii - t_jj and diagonal blocks in FP64, then FP64 residuals of U^2 = I and
 *   TU = UT and an FP32 correction solve (iterative refinement); blocks whose
 *   refinement stalls are recomputed in FP64.
 * FP32: the mixed path without refinement (about 1e-6 relative accuracy). */
typedef int32_t signtri_mode;
enum { SIGNTRI_FP64 = 0, SIGNTRI_MIXED_REFINED = 1, SIGNTRI_FP32 = 2 };

/* PH: the Parlett-Higham substitution (Algorithm 3 in block form).
 * PS: the Parlett-Sylvester form (Algorithm 2 with diagonal blocks +-I) on a
 *   diagonal already grouped by sign.
 * PROJ: the Parlett-Sylvester result for a diagonal whose signs are not grouped
 *   (Section 3 reaches it by Schur reordering, the sign-split Sylvester equation
 *   and a transformation back).  Computed here without reordering: the right
 *   and left invariant subspaces of the minority sign class, each from a
 *   triangular substitution, give the spectral projector P of that class, and
 *   U = s (I - 2 P) with s the majority sign.  Real or complex T, in FP64 (every
 *   mode runs it in FP64), at most 512 (real T) or 64 (complex T) entries in
 *   the minority class; real T also needs 2 ceil(m / 8) + 2 compute units for
 *   its persistent launch (else SIGNTRI_ENOTSUP).
 * AUTO picks by work estimates: PS when the diagonal is grouped and the
 *   Section 3 model favours it; in FP64 mode with no sweep or block size pinned
 *   in the options, PROJ when the minority class is within those limits and the
 *   estimate 3 n^2 m (four times that for complex T) is below the PH estimate;
 *   else PH.  signtri_plan_host() reports the FP64-mode choice. */
typedef int32_t signtri_algo;
enum { SIGNTRI_AUTO = 0, SIGNTRI_PH = 1, SIGNTRI_PS = 2, SIGNTRI_PROJ = 3 };

typedef int32_t signtri_layout;
enum { SIGNTRI_COL_MAJOR = 0, SIGNTRI_ROW_MAJOR = 1 };

/* Path actually run. */
enum { SIGNTRI_PATH_TRIVIAL = 0, SIGNTRI_PATH_PH = 1, SIGNTRI_PATH_PS = 2, SIGNTRI_PATH_PROJ = 3 };

enum {
    SIGNTRI_OK = 0,
    SIGNTRI_EDOMAIN = 1,     /* some Re(t_ii) is zero, or t_ii is not finite   */
    SIGNTRI_EHIP = 2,        /* a HIP runtime call failed                      */
    SIGNTRI_EWORKSPACE = 3,  /* ws_bytes smaller than signtri_workspace_size() */
    SIGNTRI_ENOCONV = 4,     /* refinement did not converge, fallback disabled */
    SIGNTRI_ENOTSUP = 5,     /* a combination this build does not implement    */
    SIGNTRI_ENOMEM = 6,      /* the library could not allocate its workspace   */
    SIGNTRI_ETOOBIG = 7      /* signtri_noalloc(): n beyond its fixed scratch   */
};

/* Filled on return when non-NULL (host memory). */
typedef struct {
    int32_t path;             /* SIGNTRI_PATH_* that ran                                 */
    int32_t model_pick;       /* SIGNTRI_PATH_PH or _PS by the Section 3 model, reordering
                                 cost included (the paper's choice)                       */
    int64_t n_pos, n_neg;     /* inertia of the diagonal                                  */
    int64_t swaps;            /* adjacent swaps needed to group the diagonal by sign       */
    double w_ph, w_ps;        /* Section 3 work estimates in real flops                   */
    int32_t refine_steps;     /* refinement steps taken (mixed mode)                      */
    int32_t tile;             /* block size used                                          */
    int64_t fallback_tiles;   /* blocks recomputed in FP64 after a stalled refinement     */
    double correction_rel;    /* max |correction| / max |U| of the last refinement step   */
    int64_t bad_index;        /* 1-based index of the offending diagonal (EDOMAIN), else 0 */
    int32_t sweep;            /* SIGNTRI_SWEEP_* that ran (0 for the trivial path)        */
    int32_t wgs_per_cu;       /* dataflow sweep: persistent workgroups per compute unit   */
} signtri_info;

/* How the off-diagonal blocks are scheduled.
 * DATAFLOW: one persistent kernel per sweep; workgroups take 32 x 32 blocks in
 *   dependency order and wait on per-block completion flags (real or complex T, every
 *   mode, both the substitution and the Sylvester form).
 * SUPERDIAG: one product launch and one solve launch per block superdiagonal,
 *   with a one-superdiagonal lookahead on a second stream, replayed from a
 *   captured graph (FP64 only: real with 32 x 32 or 64 x 64 blocks, complex
 *   with 32 x 32; the substitution only).
 * AUTO: the choice recorded by signtri_autotune() for this dtype, mode, path
 *   and size class, else DATAFLOW for real T and SUPERDIAG for complex T. */
enum { SIGNTRI_SWEEP_AUTO = 0, SIGNTRI_SWEEP_DATAFLOW = 1, SIGNTRI_SWEEP_SUPERDIAG = 2 };

/* Tunables; zero-initialise for defaults. */
typedef struct {
    int32_t tile;                /* block size: 0 = tuned choice or 32; 64 is available on
                                    the superdiagonal sweep of real FP64 only (and selects
                                    that sweep when `sweep` is AUTO)                      */
    int32_t max_refine_steps;    /* mixed mode: refinement steps at most, 0 = default (2),
                                    at most 64 (else -13); negative: none, so every block
                                    counts as not converged (recomputed in FP64, or
                                    SIGNTRI_ENOCONV).  The convergence tests run on the
                                    device: a step found unnecessary runs as empty
                                    kernels, and nothing waits on the host until the end  */
    double stall_ratio;          /* mixed mode: a block stalls when a step leaves its
                                    residual above this fraction of the previous one
                                    (0 = default 0.5)                                    */
    int32_t no_fallback;         /* mixed mode: 1 = return SIGNTRI_ENOCONV instead of
                                    recomputing stalled blocks in FP64                   */
    int32_t max_splits;          /* split-K limit for block products of the superdiagonal
                                    sweeps (0 = default)                                 */
    int64_t force_stall;         /* testing: treat block (I, J) of the 32 x 32 grid as
                                    stalled when this is 1 + I * nb + J (nb = block count
                                    of the row index space), every block when -1, none
                                    when 0                                               */
    int32_t sweep;               /* SIGNTRI_SWEEP_*; 0 = tuned choice or default           */
    int32_t wgs_per_cu;          /* dataflow sweep: persistent workgroups per compute unit,
                                    0 = tuned choice, else as many as fit with the
                                    registers the compiler gives the sweep (a batch: as
                                    many as fit at all); a value above that takes the
                                    sweep's build for one more workgroup per compute unit
                                    (real T), values above what fits are clamped to it  */
    int32_t products;            /* off-diagonal block products of the dataflow sweeps
                                    (Section 5's accumulators X and Y): SIGNTRI_PRODUCTS_*;
                                    other values -13                                     */
} signtri_options;

/* MASKED (0, the default): each 16 x 16 piece of a block's product forms only the
 *   accumulator its entries need: Y (sums of u u) where some row and column share
 *   a sign, X (sums of u t - t u) where some differ, as Section 5.3 proposes.
 * DENSE: every piece forms both, as the recursion of Algorithms 4-6 does; the same
 *   results up to rounding, kept for measuring what the masking saves. */
enum { SIGNTRI_PRODUCTS_MASKED = 0, SIGNTRI_PRODUCTS_DENSE = 1 };

/*
 * Compute U = sign(T).
 *   T, ldt      device input, upper triangle read (see conventions above)
 *   U, ldu      device output, n x n written
 *   n           order, n >= 0 (n == 0 is a no-op)
 *   dtype       SIGNTRI_R64 or SIGNTRI_C128
 *   layout      storage order of both T and U
 *   mode        SIGNTRI_FP64, SIGNTRI_MIXED_REFINED or SIGNTRI_FP32
 *   algo        SIGNTRI_AUTO, SIGNTRI_PH, SIGNTRI_PS or SIGNTRI_PROJ (PS requires a
 *               diagonal already grouped by sign; PROJ 1..512 (real) or 1..64
 *               (complex) entries in the minority sign class; else SIGNTRI_ENOTSUP)
 *   Real and complex T take every mode; the projector form (PROJ) computes in
 *   FP64 whatever the mode.
 *   workspace   device scratch of ws_bytes bytes, or NULL to let the library
 *               use a buffer it allocates and keeps for later calls
 *   stream      hipStream_t to queue work on (NULL = default stream)
 *   opts        tunables, or NULL for defaults
 *   info        optional host output
 * Errors: SIGNTRI_EDOMAIN (detected by the diagonal scan, before U is
 * written; info->bad_index names the entry), SIGNTRI_EWORKSPACE, SIGNTRI_EHIP,
 * SIGNTRI_ENOCONV, SIGNTRI_ENOTSUP, SIGNTRI_ENOMEM, or -p for argument p.
 */
int signtri(const void *T, int64_t ldt, void *U, int64_t ldu, int64_t n,
            signtri_dtype dtype, signtri_layout layout, signtri_mode mode,
            signtri_algo algo, void *workspace, size_t ws_bytes, void *stream,
            const signtri_options *opts, signtri_info *info);

/* Bytes of device workspace signtri() needs for these arguments (an upper
 * bound valid for any diagonal).  Returns 0 for invalid arguments. */
size_t signtri_workspace_size(int64_t n, signtri_dtype dtype, signtri_layout layout,
                              signtri_mode mode, signtri_algo algo);

/*
 * A general function of T (Section 2, Algorithm 1): F = phi(T) by Parlett's
 * substitution, f_ij = [t_ij (f_ii - f_jj) + sum_{i<k<j} (f_ik t_kj - t_ik f_kj)]
 * / (t_ii - t_jj), the element equation of TF = FT, with the caller's values of
 * phi on the diagonal.  Computed in FP64 (complex128) by the dataflow sweep of
 * the substitution, every pair of entries by that equation.
 *   T, ldt      device input, upper triangle read (conventions above), column-major
 *   fdiag       device array of n values phi(t_ii) (SIGNTRI_C128: interleaved pairs)
 *   F, ldf      device output, n x n written (zeros below the diagonal), column-major
 *   n, dtype, stream, info as for signtri() (info: path SIGNTRI_PATH_PH, tile 32)
 * The diagonal entries of T must be distinct: a repeated one divides by zero and
 * leaves non-finite values in F (nothing checks for it); nearby ones amplify
 * rounding errors as 1 / |t_ii - t_jj| (Section 2).  With info, the call waits
 * and reports a dependency wait that gave up (SIGNTRI_EHIP).  Returns 0, -p for
 * argument p (-4 also when F overlaps T or fdiag), SIGNTRI_ENOMEM, SIGNTRI_EHIP.
 * phi = sign on a diagonal without zero real parts gives sign(T) through
 * Eq. (1) alone; signtri() computes it with Eq. (2) where signs agree.
 */
int signtri_fun(const void *T, int64_t ldt, const void *fdiag, void *F, int64_t ldf, int64_t n,
                signtri_dtype dtype, void *stream, signtri_info *info);

/*
 * Batched form: U_b = sign(T_b) for b = 0 .. batch-1, matrices of uneven
 * order, in one graph-captured persistent launch.
 *   T, U        HOST arrays of `batch` DEVICE pointers (host arrays, so that
 *               the call can plan on the host without reading them back; the
 *               captured graph of a batch is keyed by these pointers, so a new
 *               set of buffers captures a new graph, and the same set replays it)
 *   ldt, ldu, n HOST arrays of `batch` leading dimensions and orders
 *   dtype       SIGNTRI_R64 or SIGNTRI_C128
 *   layout      SIGNTRI_COL_MAJOR only in this build (else SIGNTRI_ENOTSUP)
 *   mode        as for signtri(); MIXED_REFINED refines each matrix
 *   workspace   device scratch of ws_bytes, or NULL for a library buffer
 *   infos       optional HOST array of `batch` results
 * The call plans on the host (one stream synchronisation for the diagonal
 * signs), then launches, and waits for the result before returning; a domain
 * error in any matrix returns SIGNTRI_EDOMAIN before anything is written and
 * marks that matrix's info.
 */
int signtri_batched(const void *const *T, const int64_t *ldt, void *const *U,
                    const int64_t *ldu, const int64_t *n, int64_t batch,
                    signtri_dtype dtype, signtri_layout layout, signtri_mode mode,
                    void *workspace, size_t ws_bytes, void *stream,
                    const signtri_options *opts, signtri_info *infos);

/* Device workspace needed by signtri_batched() for these orders. */
size_t signtri_batched_workspace_size(const int64_t *n, int64_t batch,
                                      signtri_dtype dtype, signtri_mode mode);

/*
 * sign(A) for general square matrices of small order (Section 1: a complex
 * Schur decomposition A = Q T Q*, the first step of Algorithm 3, then
 * U = sign(T) by Algorithm 3's substitution, then sign(A) = Q U Q*).  Each
 * matrix is reduced on one wave with its Hessenberg/Schur form and Q in LDS:
 * Householder reduction to Hessenberg form, the shifted QR iteration (implicit
 * single shifts, plane rotations) to the Schur form, Algorithm 3 on T, and the
 * two products.  FP64 / complex128 throughout.
 *   A, lda      host array of `batch` device pointers (column-major inputs, read
 *               only) and their leading dimensions
 *   S, lds      host array of device pointers to the outputs (n x n, column-major,
 *               same dtype as A; a real A gets a real sign(A)); must not overlap A
 *   n           host array of orders, 0 .. 64 (0: nothing done)
 *   dtype       SIGNTRI_R64 or SIGNTRI_C128 for every matrix
 *   stream      HIP stream (NULL: the default stream); the call waits for it
 *   status      optional host array of `batch` codes: SIGNTRI_OK, SIGNTRI_EDOMAIN
 *               (an eigenvalue on the imaginary axis, i.e. with |Re t_ii| at most
 *               n u ||A||_F in the computed Schur form (u = 2^-52), where rounding
 *               decides its sign, or a non-finite entry met on the way: that S is
 *               left untouched), SIGNTRI_ENOCONV (the QR iteration
 *               did not reach the Schur form within 30 max(10, n) sweeps: S left
 *               untouched)
 * Returns SIGNTRI_OK, the first failing matrix's code (in batch order),
 * SIGNTRI_ENOTSUP for an order above 64, SIGNTRI_ENOMEM, SIGNTRI_EHIP, or -p for
 * argument p (-3 also when some S overlaps its A).  sign(A) is ill-conditioned
 * when eigenvalues lie near the imaginary axis (Section 1): the result is then
 * as accurate as that conditioning allows, and nothing checks it.
 */
int signtri_signm_batched(const void *const *A, const int64_t *lda, void *const *S,
                          const int64_t *lds, const int64_t *n, int64_t batch,
                          signtri_dtype dtype, void *stream, int32_t *status);

/*
 * The entry point that allocates nothing: for callers that cannot allocate
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Computes what signtri() computes for FP64 mode,
 * column-major storage, AUTO path and default options (the dataflow sweeps, or
 * the projector form for at most 64 minority entries: with more, the dataflow
 * sweeps), with no device or pinned-host allocation: the scratch
 * memory comes from a fixed device array of 56 MiB that each GPU the library
 * runs on holds until the process ends, and the planner's host staging from a
 * fixed host array.  Orders up to 8192 (real or complex); larger n returns
 * SIGNTRI_ETOOBIG before any device work.  The call plans (one stream
 * synchronisation), runs, and waits for its result before returning, and
 * calls from different host threads of a process are serialised: the fixed
 * arrays are shared by every call, and hold the last call's contents.
 * Arguments, return codes and the info output as for signtri().
 */
int signtri_noalloc(const void *T, int64_t ldt, void *U, int64_t ldu, int64_t n,
                    signtri_dtype dtype, void *stream, signtri_info *info);

/* Human-readable text for a return code (static storage). */
const char *signtri_strerror(int code);

/*
 * The plain form: column-major, ldu = ld, AUTO path, FP64, library workspace,
 * default stream, synchronous (returns after U is complete).
 */
int sign_tri(const void *T, int64_t n, int64_t ld, signtri_dtype dtype, void *U);

/*
 * Section 3 planner on HOST data, without a GPU: from the diagonal signs
 * s[0..n-1] (each +1 or -1) compute the inertia, the swap count and the two
 * work estimates, and the path AUTO would run (into info->path; the other
 * fields as documented for signtri_info).  Returns 0, or -1 for bad input.
 */
int signtri_plan_host(const int8_t *s, int64_t n, signtri_dtype dtype,
                      signtri_info *info);

/*
 * Autotuner.  The sweep variant and the dataflow grid that run fastest depend
 * on the order, the inertia and the mode, so they are measured rather than
 * modelled.  A table, keyed by (dtype, mode, path, size class ceil(log2 n)),
 * holds the best choice measured so far; signtri() consults it for every
 * option left at 0 (sweep, tile, wgs_per_cu).  The table lives in process
 * memory; if the environment variable SIGNTRI_TUNE_FILE names a file, the
 * table is read from it at the first lookup, and signtri_tune_save() writes
 * it back.
 */
typedef struct {
    int32_t dtype, mode, path;  /* key: signtri_dtype, signtri_mode, SIGNTRI_PATH_PH/_PS,
                                   or SIGNTRI_TUNE_BATCHED for signtri_batched()          */
    int32_t log2n;              /* key: ceil(log2 n) (batched: of the largest order)      */
    int32_t sweep, tile, wgs_per_cu;  /* the choice                                       */
    double ms;                  /* its measured time per call, milliseconds               */
} signtri_tune_entry;

/*
 * Time every candidate (sweep variant, block size, dataflow workgroups per
 * compute unit) on this column-major T (device; U is overwritten and holds
 * sign(T) on return), `reps` timed calls each after one untimed call, on
 * `stream`; record the fastest in the table and return it in *best (host).
 * Every candidate computes the same sign(T) to the same accuracy.  Waits for
 * the stream.  Returns 0, -p for argument p, or the first error of a call
 * (SIGNTRI_EDOMAIN, ...).  For the trivial path (one sign) nothing is
 * recorded and best->sweep is 0.
 */
int signtri_autotune(const void *T, int64_t ldt, void *U, int64_t ldu, int64_t n,
                     signtri_dtype dtype, signtri_mode mode, signtri_algo algo,
                     void *stream, int32_t reps, signtri_tune_entry *best);

/*
 * The batched form's key: signtri_batched() runs every matrix of a batch in
 * one persistent dataflow sweep (32 x 32 blocks), so its one choice is the
 * grid, wgs_per_cu; it consults the entry (dtype, mode, SIGNTRI_TUNE_BATCHED,
 * ceil(log2 of the batch's largest order)) when options leave wgs_per_cu at 0.
 */
enum { SIGNTRI_TUNE_BATCHED = 8 };

/*
 * signtri_autotune() for a batch (arguments as signtri_batched(), column-major):
 * times each dataflow grid (workgroups per compute unit) on this batch, `reps`
 * timed calls each after one untimed call, records the fastest under the key
 * above and returns it in *best (host).  U is overwritten with sign(T).
 * Waits for the stream.  Returns 0, -p for argument p (as signtri_batched();
 * -12 for reps out of [1, 1000], -13 for best == NULL), or the first error of a
 * call.
 */
int signtri_autotune_batched(const void *const *T, const int64_t *ldt, void *const *U,
                             const int64_t *ldu, const int64_t *n, int64_t batch,
                             signtri_dtype dtype, signtri_mode mode, void *stream, int32_t reps,
                             signtri_tune_entry *best);

/* The recorded choice for this key, copied to *out: 1 if found, else 0. */
int signtri_tune_lookup(signtri_dtype dtype, signtri_mode mode, int32_t path, int64_t n,
                        signtri_tune_entry *out);

/* Write the table as text (one entry per line) / merge a file written so.
 * Return 0, or -1 if the file cannot be opened or holds a malformed line
 * (nothing is merged then). */
int signtri_tune_save(const char *path);
int signtri_tune_load(const char *path);

/* Forget every recorded choice. */
void signtri_tune_clear(void);

/* Release the library-owned workspace buffers (all devices). */
void signtri_release(void);

/*
 * Kernel timers, for measurement.  signtri_profile_enable(1) clears the
 * counters and, until signtri_profile_enable(0), brackets every kernel the
 * library launches with a pair of HIP events on the launching stream (this
 * adds a little time per launch).  signtri_profile_read() waits for the
 * recorded events and returns, for one kernel family, the summed event time
 * in milliseconds, the number of launches and the algorithmic flops of that
 * work (Section 3 counting: a real multiply-add is 2 flops, a complex one 8).
 * Returns 0, -1 for an unknown family, or SIGNTRI_EHIP.
 */
enum {
    SIGNTRI_K_SCAN = 0,        /* diagonal scan                                       */
    SIGNTRI_K_DIAG = 1,        /* diagonal blocks, element by element                 */
    SIGNTRI_K_GEMM = 2,        /* block products of the superdiagonal sweeps          */
    SIGNTRI_K_SOLVE = 3,       /* block equations of the superdiagonal sweeps         */
    SIGNTRI_K_AUX = 4,         /* zeroing, fills, task lists                          */
    SIGNTRI_K_RESID = 5,       /* FP64 residuals of refinement                        */
    SIGNTRI_K_CORR = 6,        /* correction sweep of refinement (products + solves)  */
    SIGNTRI_K_SYL = 7,         /* Sylvester dataflow sweep (products + solves)        */
    SIGNTRI_K_FLOW = 8,        /* Parlett-Higham dataflow sweep (products + solves)   */
    SIGNTRI_K_BATCHED = 9,     /* batched persistent sweep                            */
    SIGNTRI_K_CONVERT = 10,    /* precision and layout conversions                    */
    SIGNTRI_K_PROJ = 11,       /* projector form: the two invariant-subspace substitutions */
    SIGNTRI_K_PROJ_OUT = 12    /* projector form: W^T Z, its inverse, U = s (I - 2 P)  */
};
void signtri_profile_enable(int on);
int signtri_profile_read(int family, double *ms, int64_t *launches, double *flops);

#ifdef __cplusplus
}
#endif

#endif /* SIGNTRI_H */
