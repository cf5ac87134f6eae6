/*
 * tchol: tiled FP64 Cholesky factorization and solve on one AMD MI355X
 * (gfx950), executed by a persistent kernel that runs the tile task DAG with
 * device-side dependency counters in upward-rank (critical-path) order.
 *
 * The computation is the tile Cholesky factorization DPOTRF of PLASMA in
 * double precision, with tiles of 512 in the paper's runs (arXiv 1402.6601,
 * section 4.1, "Benchmarks" and "Methodology"): a DAG of POTRF, TRSM, SYRK
 * and GEMM tile tasks.  The paper's runtime makes a task ready when its
 * predecessors have completed (section 2.2, "activate") and its HEFT strategy
 * recalls the upward-rank priority rule (section 3.1); on one GPU these
 * become per-task dependency counters and a priority-ordered ticket list.
 *
 * Conventions for every entry point
 *  - Matrix pointers are DEVICE pointers to column-major FP64 storage with
 *    leading dimension n (B: leading dimension n, nrhs columns).  Only the
 *    lower triangle of A / L is read or written; the strict upper triangle
 *    is never touched.  Row-major callers pass A unchanged (a symmetric
 *    matrix is its own transpose) and find L^T in the upper triangle of
 *    their row-major view.
 *  - The caller owns every buffer.  The library never allocates or frees
 *    device memory: all scratch (dependency counters, task descriptors, the
 *    ticket list) lives in a caller-provided device workspace of at least
 *    tchol_workspace_bytes() bytes, 256-byte aligned.  Its contents on entry
 *    do not matter and on return are unspecified.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it and the stream is then synchronised, so the
 *    return code is final when the call returns.  Calls that share a
 *    workspace must not overlap.  The host-side plan cache is thread-safe.
 *  - Return codes: 0 success; k > 0: the leading minor of order k is not
 *    positive definite (its pivot was zero, negative or NaN; LAPACK's
 *    convention) and A is partly overwritten; -i: argument i is invalid
 *    (checked before any HIP call); <= -100: TCHOL_E_* runtime errors.
 */
#ifndef TCHOL_H
#define TCHOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define TCHOL_API __attribute__((visibility("default")))
#else
#define TCHOL_API
#endif

#define TCHOL_OP_FACTOR 0
#define TCHOL_OP_SOLVE 1
#define TCHOL_OP_BATCHED 2 /* factor + solve of many systems (plan introspection only) */
#define TCHOL_OP_BACKWARD 3 /* adjoint of the factorization */
#define TCHOL_OP_MIXED_FACTOR 4 /* the factorization launch of tchol_solve_mixed (plan introspection only) */
#define TCHOL_OP_FACTOR_SOLVE 5 /* the merged launch of tchol_factor_solve (plan introspection only) */

#define TCHOL_POLICY_LIST 0   /* HEFT's list schedule (section 3.1), the default
                                 (NULL options or a zeroed struct): ready items by
                                 decreasing upward rank on 256 identical workers,
                                 with measured task times as costs, in simulated
                                 start order */
#define TCHOL_POLICY_RANK 1   /* decreasing upward rank (task by task)      */
#define TCHOL_POLICY_FIFO 2   /* step-major: (k, kind, i, j) ascending      */
#define TCHOL_POLICY_RANDOM 3 /* a seeded random topological order          */

#define TCHOL_E_HIP (-100)         /* a HIP runtime call failed              */
#define TCHOL_E_TIMEOUT (-101)     /* the kernel's bounded wait expired      */
#define TCHOL_E_UNSUPPORTED (-102) /* size beyond what the planner supports  */
#define TCHOL_E_INTERNAL (-103)    /* inconsistent device state at exit      */
#define TCHOL_E_NOCONV (-104)      /* refinement missed its target in maxit  */
#define TCHOL_E_SCRATCH (-105)     /* the problem needs more scheduler scratch than
                                      tchol_factor_solve_noalloc's fixed array  */

#define TCHOL_LOWP_FP32 1 /* mixed precision: FP32 working copy, FP32 matrix-core updates */
#define TCHOL_LOWP_BF16 2 /* mixed precision: FP32 working copy, BF16 matrix-core updates
                             (each panel value as three BF16 terms, six term products
                             with FP32 accumulation: FP32-level update accuracy)   */

#define TCHOL_NB_MIN 16
#define TCHOL_NB_MAX 512

/* Optional knobs; pass NULL to the _ex entry points for the defaults. */
typedef struct tchol_opts {
  int32_t policy;      /* TCHOL_POLICY_*; 0 (a zeroed struct, like NULL options)
                          is TCHOL_POLICY_LIST                                   */
  uint32_t seed;       /* seed of TCHOL_POLICY_RANDOM                             */
  int64_t wait_limit_us; /* bound on any single dependency wait inside the kernel;
                            0 = default (30 s); it turns a hang into
                            TCHOL_E_TIMEOUT                                      */
  float *kernel_ms;    /* out (host pointer, may be NULL): duration of the
                          persistent kernel measured with HIP events on `stream` */
  uint64_t *trace;     /* device buffer of 4 x uint64 per work item of the launch
                          (tchol_plan_query counts[2] for its op; for
                          tchol_factor_solve, TCHOL_OP_FACTOR_SOLVE (opts.subst
                          = 0); for tchol_solve_mixed, TCHOL_OP_MIXED_FACTOR), or NULL:
                          {claim, start} and {end} wall clock (100 MHz),
                          {task, part | wg<<32}                                  */
  int64_t trace_words; /* length of trace in uint64 words; with trace set, a call
                          whose launch has more than trace_words / 4 work items
                          returns -i for its opts argument i and launches nothing */
  int32_t subst;       /* FP64 solve (tchol_solve_ex, tchol_factor_solve): 0 (the
                          default) applies explicit inverses of the diagonal
                          tiles, L_kk^{-1} and L_kk^{-T}, computed in the same
                          launch, by row strips over many workgroups (short
                          dependency chain); its backward error grows with the
                          condition of the diagonal tiles (at most sqrt(cond(A))
                          for SPD A).  1: substitution against the tiles, one
                          workgroup per diagonal step, backward stable (and
                          exact on integer data whose intermediates are exact).
                          A ragged last tile (order not a multiple of 16) always
                          substitutes.                                          */
  const int32_t *wgs;  /* tchol_factor_solve_batched only (host pointer, may be
                          NULL): per system, the workgroups that share the
                          factorization of a one-tile system whose order exceeds
                          128 (the tile's sub-block DAG, section 2.1's workers
                          taking its units), in [0, 8]; 0 or 1: one workgroup.
                          A value outside [0, 8] returns -i for the opts
                          argument i.  The tuned tables choose it per order
                          bucket.                                               */
  int32_t inv_trsm;    /* tchol_factor_ex: 1 factors as tchol_factor_solve does:
                          TRSM(i, k) applies L_kk^{-1} (from TRTRI(k) in the same
                          launch, between POTRF(k) and the step's TRSMs) by
                          128-row blocks on the matrix cores, so the factor is
                          bitwise that of tchol_factor_solve; its backward error
                          grows with the condition of the diagonal tiles (as for
                          the solve with subst = 0).  0 (the default): TRSM by
                          substitution (exact on integer data whose
                          intermediates are exact).  tchol_factor_solve applies
                          the inverses in its TRSMs whenever its solve does
                          (subst = 0).                                          */
} tchol_opts;

/* Bytes of device workspace needed by `op` (TCHOL_OP_FACTOR, _SOLVE or
   _BACKWARD) for order n and tile size nb (nrhs is read by TCHOL_OP_SOLVE only).  Returns -i for an invalid
   argument i, TCHOL_E_UNSUPPORTED beyond the supported sizes. */
TCHOL_API int64_t tchol_workspace_bytes(int32_t op, int64_t n, int64_t nb, int64_t nrhs);

/* Factor A = L L^T in place: on success the lower triangle of A holds L.
   Paper: the Cholesky tile DAG (section 4.1, "Benchmarks").
   Arguments: 1 A, 2 n >= 0, 3 nb in [16, 512] and a multiple of 16,
   4 ws, 5 ws_bytes, 6 stream.  n need not be a multiple of nb (edge tiles). */
TCHOL_API int32_t tchol_factor(double *A, int64_t n, int64_t nb, void *ws, int64_t ws_bytes, void *stream);
TCHOL_API int32_t tchol_factor_ex(double *A, int64_t n, int64_t nb, void *ws, int64_t ws_bytes, void *stream,
                        const tchol_opts *opts);

/* Solve (L L^T) X = B in place (B := X) given the factor from tchol_factor,
   by a forward then a backward tiled substitution on the same scheduler.
   The diagonal steps apply the tiles' explicit inverses, computed by the same
   launch (see tchol_opts.subst); the workspace holds them (n nb doubles) and
   the intermediate Y (n nrhs doubles).
   Arguments: 1 L, 2 n, 3 nb, 4 B (n x nrhs, column-major, ld n), 5 nrhs >= 0,
   6 ws, 7 ws_bytes, 8 stream. */
TCHOL_API int32_t tchol_solve(const double *L, int64_t n, int64_t nb, double *B, int64_t nrhs, void *ws,
                    int64_t ws_bytes, void *stream);
TCHOL_API int32_t tchol_solve_ex(const double *L, int64_t n, int64_t nb, double *B, int64_t nrhs, void *ws,
                       int64_t ws_bytes, void *stream, const tchol_opts *opts);

/* Adjoint of the factorization (reverse-mode derivative): given the factor L
   of A (from tchol_factor) and Lbar = df/dL for a scalar f, overwrites the
   lower triangle of Lbar with that of Abar = df/dA, the symmetric gradient
   (off-diagonal entries of a symmetric perturbation count once in each
   triangle, so f(A + h (E_ij + E_ji)) changes by 2 h Abar_ij).  For
   f = log det A (Lbar = diag(2 / L_ii)) the result is A^{-1}.
   The derivative of the paper's tile Cholesky DAG (section 4.1) taken in
   reverse: the steps from the last to the first, the GEMM / SYRK updates
   of each step reversed as GEMMs into the adjoints of its panel (chained
   per tile in a fixed order), its TRSMs as triangular solves with L_kk, its
   POTRF as the adjoint of the diagonal tile's factorization, on the same
   persistent scheduler in upward-rank order.  The diagonal tile's adjoint
   is taken in closed form, S / 2 with S = L_kk^{-T} (M + M^T) L_kk^{-1} and
   M = the lower triangle of L_kk^T Lbar_kk with its diagonal halved, by
   products over 64 x 64 blocks (L_kk^{-T} computed in the same launch),
   when the tile's order is a multiple of 16; a ragged last tile reverses its
   factorization panel by panel.  Results do not depend on the claim order.
   L must have a positive diagonal (a factor tchol_factor
   returned with info 0); only lower triangles are read or written.
   Workspace: tchol_workspace_bytes(TCHOL_OP_BACKWARD, n, nb, 0) bytes
   (about 2 n^2 + n^2 / 2 + 3 n nb doubles: the transposed factor, twice
   the adjoint, per-tile partial products, and per diagonal tile its
   inverse and two scratch tiles).
   Arguments: 1 L, 2 n, 3 nb (as for tchol_factor; n / nb at most 160),
   4 Lbar (n x n, ld n), 5 ws, 6 ws_bytes, 7 stream, 8 opts (_ex). */
TCHOL_API int32_t tchol_backward(const double *L, int64_t n, int64_t nb, double *Lbar, void *ws, int64_t ws_bytes,
                                 void *stream);
TCHOL_API int32_t tchol_backward_ex(const double *L, int64_t n, int64_t nb, double *Lbar, void *ws,
                                    int64_t ws_bytes, void *stream, const tchol_opts *opts);

/* Factor A = L L^T and solve (L L^T) X = B in ONE launch: the factorization
   DAG and the solve DAG merged as one DAG (the solve reads each tile of L as
   soon as it is final: POTRF(k) before FTRSV(k), TRSM(i, k) before
   FGEMV(i, k)), so the forward substitution runs while the factorization
   still has work in flight; the claim order is decreasing upward rank over
   both (section 3.1).  With opts.subst = 0 (the default) the diagonal
   tiles' explicit inverses, TRTRI(k) between POTRF(k) and the step's TRSMs,
   serve both the factorization's TRSMs (products with L_kk^{-1} on the
   matrix cores) and the solve's diagonal steps; results are then identical
   to tchol_factor_ex with opts.inv_trsm = 1 followed by tchol_solve.  With
   opts.subst = 1 both substitute, identical to tchol_factor followed by
   tchol_solve with opts.subst = 1.
   Arguments: 1 A (in/out as for tchol_factor), 2 n, 3 nb,
   4 B (n x nrhs, ld n, in/out as for tchol_solve), 5 nrhs >= 0, 6 ws,
   7 ws_bytes >= tchol_factor_solve_workspace_bytes(n, nb, nrhs), 8 stream,
   9 opts (NULL or as for tchol_factor_ex).  Returns 0, k > 0 (leading minor
   of order k not positive definite; B is then partly overwritten), or a
   negative code. */
TCHOL_API int64_t tchol_factor_solve_workspace_bytes(int64_t n, int64_t nb, int64_t nrhs);
TCHOL_API int32_t tchol_factor_solve(double *A, int64_t n, int64_t nb, double *B, int64_t nrhs, void *ws,
                                     int64_t ws_bytes, void *stream, const tchol_opts *opts);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   merged factor + solve launch as tchol_factor_solve with opts.subst = 1 (the
   diagonal tiles' inverses would not fit the fixed array), bitwise the same
   results, but with no workspace argument.  Its scheduler
   scratch (header, dependency counters, task descriptors, successor lists,
   ticket list) lives in a fixed device array of the library,
   TCHOL_NOALLOC_SCRATCH_BYTES per GPU, held by every GPU the library runs on
   until the process ends.  The call itself allocates nothing on the device
   and no pinned host memory (the plan, built on the first call for an
   (n, nb), is kept in ordinary host memory).  Every call on one GPU shares
   that GPU's array and leaves its contents behind; each call clears what
   must start at zero.  Calls that overlap on one GPU (other host threads,
   other streams) race on the array and must be serialised by the caller.
   Arguments: 1 A, 2 n, 3 nb, 4 B, 5 nrhs (as for tchol_factor_solve),
   6 stream.  Returns as tchol_factor_solve, or TCHOL_E_SCRATCH (checked
   before any HIP call) when the launch's scheduler scratch, the same as
   tchol_batched_workspace_bytes for the one system (n, nb) when nb < n, exceeds
   TCHOL_NOALLOC_SCRATCH_BYTES (n = 32768 with nb = 512 needs 8.3 MiB;
   nb = 256 about 31 MiB). */
#define TCHOL_NOALLOC_SCRATCH_BYTES (16 << 20)
TCHOL_API int32_t tchol_factor_solve_noalloc(double *A, int64_t n, int64_t nb, double *B, int64_t nrhs,
                                             void *stream);

/* Batched factor + solve of `batch` independent SPD systems in ONE launch
   of the persistent kernel.  Paper: the same tile DAG (section 4.1) per
   system; the systems' DAGs are merged into one, each system's solve
   joined to its factorization by data flow (POTRF(k) before FTRSV(k),
   TRSM(i, k) before FGEMV(i, k)), and claimed in HEFT's list-schedule
   order over decreasing upward rank (section 3.1), with each task's cost its
   kind's measured time scaled by the cube of its tile size, so that long
   critical paths start first.
   Host arrays, one entry per system s:
     a_off[s]  element offset of A_s from A; A_s is n[s] x n[s], column-major,
               leading dimension lda[s] >= max(1, n[s]); lower triangle used;
     b_off[s]  element offset of B_s from B; B_s is n[s] x nrhs, column-major,
               leading dimension n[s]; overwritten by the solution;
     n[s] >= 0 its order; nb[s] its tile size (as for tchol_factor), chosen
               per system (e.g. by a tuned table: one tile, or several tiles
               that spread one system over many workgroups).
   info (host, batch entries, out): 0, or the LAPACK-style failing column of
   that system; a failing system stops only its own remaining work (its A
   and B are then partly overwritten), the others complete.
   Systems must not overlap in memory.  The faster 16-byte transfer path is
   used when every lda[s] is even, every A_s is 16-byte aligned, and every
   odd n[s] has lda[s] > n[s] (e.g. lda[s] = n[s] rounded up to even).
   When, in addition, every system is one tile (nb[s] >= n[s]) factored by
   one workgroup (opts.wgs absent or at most 1), the launch runs a compact
   kernel instance (two workgroups per compute unit) and, for nrhs <= 4,
   solves forward inside each factorization; the results and their
   contract are the same.
   Arguments: 1 A, 2 a_off, 3 lda, 4 B, 5 b_off, 6 n, 7 nb, 8 nrhs >= 0,
   9 batch >= 0, 10 info, 11 ws, 12 ws_bytes, 13 stream, 14 opts (NULL or as
   for tchol_factor_ex; opts.wgs applies).  Returns 0 when the launch ran
   (per-system failures are reported in info only), or a negative code.
   tchol_batched_workspace_bytes: the workspace of that launch for any
   opts.wgs. */
TCHOL_API int64_t tchol_batched_workspace_bytes(const int32_t *n, const int32_t *nb, int32_t batch);
TCHOL_API int32_t tchol_factor_solve_batched(double *A, const int64_t *a_off, const int32_t *lda, double *B,
                                             const int64_t *b_off, const int32_t *n, const int32_t *nb,
                                             int32_t nrhs, int32_t batch, int32_t *info, void *ws,
                                             int64_t ws_bytes, void *stream, const tchol_opts *opts);

/* Batched factor + solve of `batch` independent SPD systems stored in FP32,
   in ONE launch of the persistent kernel (the DAG and priority as for
   tchol_factor_solve_batched).  Precision: the trailing SYRK / GEMM updates
   run on FP32 matrix cores on the FP32 storage; each system's diagonal tiles
   are kept in FP64 in the workspace (their SYRK updates added in FP64, POTRF
   in FP64); TRSM and the solves compute in FP64 against them (the
   right-hand sides are staged in FP64); results are rounded to FP32 when
   written back.  No refinement.  When every system is one tile, a compact
   kernel instance (two workgroups per compute unit) reads each FP32 matrix
   itself, keeps L in FP64 in the workspace for its products and solves, and
   writes L rounded to FP32 back; only the right-hand sides are staged.
   Arguments as for tchol_factor_solve_batched with FP32 A and B (offsets in
   floats), except: every non-empty system needs lda[s] a multiple of 4 and
   lda[s] >= n[s] + 3 (the FP32 tile loads move four rows per 16-byte lane and
   may read three rows past the order), a_off[s] a multiple of 4 and A 16-byte
   aligned (else -3, -2, -1).  Workspace: tchol_batched_f32_workspace_bytes
   (n, nb, batch, nrhs) bytes (about sum_s T_s nb_s^2 + n_s nrhs doubles). */
TCHOL_API int64_t tchol_batched_f32_workspace_bytes(const int32_t *n, const int32_t *nb, int32_t batch, int32_t nrhs);
TCHOL_API int32_t tchol_factor_solve_batched_f32(float *A, const int64_t *a_off, const int32_t *lda, float *B,
                                                 const int64_t *b_off, const int32_t *n, const int32_t *nb,
                                                 int32_t nrhs, int32_t batch, int32_t *info, void *ws,
                                                 int64_t ws_bytes, void *stream, const tchol_opts *opts);

/* Mixed-precision solve with iterative refinement: X = A^{-1} B to FP64
   accuracy from a factorization whose trailing updates run in low precision.
   A (n x n, column-major, ld n, lower triangle read, not modified) is first
   copied to a low-precision working copy in the workspace; that copy is
   factored on the same tile DAG and scheduler as tchol_factor (the paper's
   Cholesky DAG, section 4.1): SYRK / GEMM / TRSM on the copy with FP32
   matrix-core products, each diagonal tile promoted to FP64 for its POTRF
   and kept in FP64.  With lowp = TCHOL_LOWP_BF16 the GEMM updates run on
   the BF16 matrix cores instead: each TRSM result is also stored as three
   BF16 terms (hi + mid + lo), and the six term products whose orders add up
   to at most two are accumulated in FP32, which keeps the updates at FP32
   accuracy (the SYRK updates of the diagonal tiles stay FP32 products).  Then x_0 = L~^{-T} L~^{-1} b, and while the normwise
   backward error eta_j = ||r_j||_inf / (||A||_inf ||x_j||_inf + ||b_j||_inf)
   of some column exceeds tol: r = b - A x in FP64 against the original A,
   x += L~^{-T} L~^{-1} r (substitutions in FP64 arithmetic on the stored
   factor).  Each iteration reads the stopping test back to the host once.
   Arguments: 1 A, 2 n >= 0, 3 nb (as for tchol_factor), 4 B (n x nrhs, ld n,
   in: right-hand sides, out: solutions), 5 nrhs >= 0, 6 lowp
   (TCHOL_LOWP_FP32 or TCHOL_LOWP_BF16), 7 tol > 0 (target eta, e.g. 1e-12), 8 maxit >= 0
   (corrections at most), 9 berr_out (host, nrhs entries or NULL: final eta
   per column), 10 iters_out (host or NULL: corrections applied), 11 ws,
   12 ws_bytes >= tchol_mixed_workspace_bytes_ex(n, nb, nrhs, lowp), 13 stream,
   14 opts (NULL or as for tchol_factor_ex; kernel_ms and trace describe the
   factorization's launch).
   Returns 0 when every column met tol; k > 0 when the low-precision
   factorization found the leading minor of order k not positive definite
   (B unchanged); TCHOL_E_NOCONV when maxit corrections did not reach tol (B
   holds the last iterate, berr_out its eta; LAPACK's mixed solvers then
   fall back to the FP64 path, tchol_factor + tchol_solve); other negative
   codes as for tchol_factor. */
TCHOL_API int64_t tchol_mixed_workspace_bytes(int64_t n, int64_t nb, int64_t nrhs);
/* The same for a given lowp (TCHOL_LOWP_FP32 as above; TCHOL_LOWP_BF16 adds the
   panels' BF16 terms, 6 bytes per element of the T nb x T nb grid); -4 for
   another lowp. */
TCHOL_API int64_t tchol_mixed_workspace_bytes_ex(int64_t n, int64_t nb, int64_t nrhs, int32_t lowp);
TCHOL_API int32_t tchol_solve_mixed(const double *A, int64_t n, int64_t nb, double *B, int64_t nrhs, int32_t lowp,
                                    double tol, int32_t maxit, double *berr_out, int32_t *iters_out, void *ws,
                                    int64_t ws_bytes, void *stream, const tchol_opts *opts);

/* Human-readable text for a return code (static storage). */
TCHOL_API const char *tchol_strerror(int32_t code);

/* Host-only plan introspection (no HIP call).  Fills, when the pointers are
   non-NULL: counts[0..3] = {ntask, nedge, nitem, critical-path task count};
   per task (ntask entries): kind, i, j, k, parts, initial dependency count,
   upward rank; succ_off (ntask + 1) and succ (nedge); and the claim order as
   work items item_task / item_part (nitem).  Returns 0 or a negative code. */
TCHOL_API int32_t tchol_plan_query(int32_t op, int64_t n, int64_t nb, int32_t policy, uint32_t seed, int64_t *counts,
                         int32_t *kind, int32_t *ti, int32_t *tj, int32_t *tk, int32_t *parts,
                         int32_t *dep0, int64_t *rank, int32_t *succ_off, int32_t *succ,
                         int32_t *item_task, int32_t *item_part);

/* The same introspection for the merged DAG of tchol_factor_solve_batched
   (systems given by n and nb, batch entries, and wgs as tchol_opts.wgs, NULL
   for the default); sys (ntask) receives each task's system.  Returns 0 or
   a negative code (-6 for a wgs entry outside [0, 8]). */
TCHOL_API int32_t tchol_batched_plan_query(const int32_t *n, const int32_t *nb, int32_t batch, int32_t policy,
                                           uint32_t seed, const int32_t *wgs, int64_t *counts, int32_t *kind,
                                           int32_t *ti, int32_t *tj,
                                           int32_t *tk, int32_t *sys, int32_t *parts, int32_t *dep0, int64_t *rank,
                                           int32_t *succ_off, int32_t *succ, int32_t *item_task,
                                           int32_t *item_part);

/* Library version string. */
TCHOL_API const char *tchol_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TCHOL_H */
