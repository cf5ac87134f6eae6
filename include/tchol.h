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

#define TCHOL_POLICY_RANK 0   /* decreasing upward rank (default)          */
#define TCHOL_POLICY_FIFO 1   /* step-major: (k, kind, i, j) ascending      */
#define TCHOL_POLICY_RANDOM 2 /* a seeded random topological order          */

#define TCHOL_E_HIP (-100)         /* a HIP runtime call failed              */
#define TCHOL_E_TIMEOUT (-101)     /* the kernel's bounded wait expired      */
#define TCHOL_E_UNSUPPORTED (-102) /* size beyond what the planner supports  */
#define TCHOL_E_INTERNAL (-103)    /* inconsistent device state at exit      */

#define TCHOL_NB_MIN 16
#define TCHOL_NB_MAX 512

/* Optional knobs; pass NULL to the _ex entry points for the defaults. */
typedef struct tchol_opts {
  int32_t policy;      /* TCHOL_POLICY_*                                         */
  uint32_t seed;       /* seed of TCHOL_POLICY_RANDOM                             */
  int64_t wait_limit_us; /* bound on any single dependency wait inside the kernel;
                            0 = default (30 s); it turns a hang into
                            TCHOL_E_TIMEOUT                                      */
  float *kernel_ms;    /* out (host pointer, may be NULL): duration of the
                          persistent kernel measured with HIP events on `stream` */
  uint64_t *trace;     /* device buffer of 4 x uint64 per work item, or NULL:
                          {start, end} wall clock (100 MHz), {task, part | wg<<32} */
} tchol_opts;

/* Bytes of device workspace needed by `op` (TCHOL_OP_*) for order n and tile
   size nb (nrhs is ignored by TCHOL_OP_FACTOR).  Returns -i for an invalid
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
   Arguments: 1 L, 2 n, 3 nb, 4 B (n x nrhs, column-major, ld n), 5 nrhs >= 0,
   6 ws, 7 ws_bytes, 8 stream. */
TCHOL_API int32_t tchol_solve(const double *L, int64_t n, int64_t nb, double *B, int64_t nrhs, void *ws,
                    int64_t ws_bytes, void *stream);
TCHOL_API int32_t tchol_solve_ex(const double *L, int64_t n, int64_t nb, double *B, int64_t nrhs, void *ws,
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

/* Library version string. */
TCHOL_API const char *tchol_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TCHOL_H */
