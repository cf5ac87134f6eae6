/* Arguments of the persistent kernel, shared by the host launcher and the
   device code.  Plain C types only. */
#ifndef TCHOL_KARGS_H
#define TCHOL_KARGS_H
#include <stdint.h>

/* header words of the device workspace */
#define HDR_TICKET 0   /* next ticket to hand out                          */
#define HDR_ABORT 1    /* non-zero: every worker stops                      */
#define HDR_INFO 2     /* first failing pivot column (1-based), 0 if none   */
#define HDR_ERROR 3    /* DEV_ERR_* code of the first runtime error, 0 if none */
#define HDR_DONE 4     /* work items completed                              */
#define HDR_WORDS 64   /* 256 bytes                                         */

/* runtime error codes in HDR_ERROR */
#define DEV_ERR_TIMEOUT 1 /* a dependency wait exceeded its bound                  */
#define DEV_ERR_LAYOUT 2  /* a work item violated the launch's alignment contract  */

typedef struct KArgs {
  double *A;            /* factor: in/out matrix; solve: the factor L (read only);
                           mixed precision: the FP32 working copy, cast             */
  double *B;            /* solve: right-hand sides, overwritten by the solution   */
  int64_t n, nb, ld, ldb, nrhs;
  int32_t T, nitem;
  int32_t gemm_m, gemm_n, trsm_rows, gemv_rows;
  int32_t *hdr;         /* HDR_WORDS header words                                 */
  int32_t *dep;         /* per task: predecessors not yet completed               */
  int32_t *done;        /* per task: work items completed                         */
  const int32_t *desc;  /* per task: kind, i, j, k, parts, succ_begin, succ_end, 0 */
  const int32_t *succ;  /* successor lists                                        */
  const int32_t *items; /* per ticket: task, part                                 */
  const int64_t *sys;   /* per system, SYS_WORDS words: a_off, b_off, n, nb, ld   */
  int32_t *sinfo;       /* per system: failing column (batched launches)          */
  int32_t batched;      /* 1: a failing system stops only its own work             */
  int32_t nsys;
  double *D;            /* mixed precision: FP64 diagonal tiles, nb x nb each, T of them */
  int32_t mixed;        /* 0: FP64; 1: mixed-precision factor, 2: its solves, 4: both
                           (A is the FP32 working copy); 3: the adjoint of the
                           factorization (A = L, B = Lbar, D = partial-product slots);
                           5: the factorization with BF16 updates; 6: FP64 batched
                           systems of one tile each (the compact instance); 7: the
                           same for FP32 batched systems (their FP64 copies in A) */
  int32_t syrk_b;       /* SYRK output sub-tile (square)                          */
  int32_t inv;          /* FP64 launches: 1 when the launch computes the diagonal
                           tiles' explicit inverses (TRTRI tasks) and applies them:
                           the solve's diagonal steps (y in S) and the TRSMs (by
                           128-row blocks); 0: substitution in place          */
  double *Dinv;         /* mixed precision: L_kk^{-1}, nb x nb each (FP64); adjoint:
                           two scratch tiles per diagonal tile (Mn, Y^T)          */
  double *DinvT;        /* mixed precision, inv and adjoint: L_kk^{-T}, nb x nb each */
  double *S;            /* mixed precision and inv: the solve's intermediate y, like B */
  double *Q;            /* adjoint: Q = twice the symmetric adjoint, ld ldq        */
  double *LT;           /* adjoint: L^T, ld ldq                                   */
  int64_t ldq;
  int64_t wait_limit;   /* bound on one dependency wait, in 100 MHz clock ticks   */
  uint64_t *trace;      /* optional: 4 words per work item                        */
  int32_t *pool;        /* POOL_WORDS counters per diagonal tile of every system
                           (the split POTRF's sub-unit pool), zeroed per launch */
  uint16_t *H;          /* BF16-update factorization: three BF16 terms of every panel
                           tile, K-contiguous: column block k, row r, column c of
                           term t at H[((t T + k) hrows + r) nb + c]             */
  int64_t hrows;        /* rows per column block of H (T nb)                      */
  float *A32;           /* mode 7: the systems' FP32 matrices (system s at A32 +
                           sys word 5, leading dimension sys word 7), read for the
                           factorization and overwritten by L rounded to FP32   */
} KArgs;

#define DESC_WORDS 8   /* kind, i, j, k, parts, succ_begin, succ_end, system */
#define SYS_WORDS 8    /* a_off, b_off, n, nb, ld, d_off (mixed precision: offset of the
                          system's FP64 diagonal tiles and inverses; mode 7: of
                          its FP32 matrix in A32), pool_off (index of the
                          system's first diagonal tile among all systems'
                          diagonal tiles, for the POTRF pools), ld2 (mode 7:
                          the FP32 matrix's leading dimension; else 0)        */
#define POOL_WORDS 64  /* counters of one diagonal tile's POTRF pool          */

#endif
