// Device side of tchol: one persistent kernel that executes a tile DAG.
//
// Worker loop (one workgroup = one worker, section 2.1 of the paper: a worker
// repeatedly takes a task, runs it, then activates its successors):
//   claim   ticket t = atomicAdd(ticket); (task, part) = items[t]
//   wait    until dep[task] == 0 (agent-scope acquire; bounded by a watchdog)
//   run     the work item (a POTRF tile, a TRSM row strip, a GEMM/SYRK
//           sub-tile, a solve block)
//   release agent-scope release, then done[task] += 1; the last work item
//           of a task decrements dep[s] of every successor s ("activate")
// Tickets are handed out in a topological order, so the worker holding the
// oldest unfinished ticket always has its predecessors finished or held by
// running workers: the loop cannot deadlock, whatever the grid size.
//
// All matrices are column-major FP64 with leading dimension `ld`; tile (i, j)
// of the matrix starts at A + (j*nb)*ld + i*nb.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kargs.h"
#include "tchol_kinds.h"

#define NT 256                 // threads per workgroup: 4 wavefronts of 64
#define LDS_DOUBLES 18176      // 145408 bytes of LDS per workgroup

typedef double d4 __attribute__((ext_vector_type(4)));

// FP64 matrix-core product on 16x16x4 blocks:  D = A(16x4) * B(4x16) + C.
// Lane l supplies A[l%16][l/16] and B[l/16][l%16]; it receives D[4i + l/16][l%16]
// in element i of the result.  Every caller below passes the B-panel fragment
// as the A operand and the (negated) A-panel fragment as the B operand, so a
// lane's four results are four consecutive COLUMNS of one row of the output
// tile: rows map to l%16 and columns to 4i + l/16.
__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }

// ---------------------------------------------------------------------------
// Matrix-core tile product used by every update:
//     C[M x N] -= Ap[M x K] * Bp[N x K]^T,   M <= BM, N <= BN.
// The four wavefronts form a WGM x (4/WGM) grid; each owns a (BM/WGM) x
// (BN*WGM/4) piece of C as 16x16 MFMA blocks held in registers from the
// first load of C to the final store.  K is streamed in chunks of KC columns
// through LDS, double buffered: the global loads of the next chunk are in
// flight while the matrix cores consume the current one.  With lower_only,
// entries of C above its diagonal are left untouched (diagonal blocks of
// SYRK and of the POTRF panels).
template <int BM, int BN, int KC, int WGM>
__device__ __forceinline__ void gemm_core(double* __restrict__ C, const double* __restrict__ Ap,
                                          const double* __restrict__ Bp, int64_t ld, int M, int N, int K,
                                          bool lower_only, double* lds) {
  constexpr int WGN = 4 / WGM;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int RB = WTM / 16, CB = WTN / 16;
  constexpr int ALD = BM + 8, BLD = BN + 8;
  constexpr int NA = BM * KC / NT, NB = BN * KC / NT;
  static_assert(NA * NT == BM * KC && NB * NT == BN * KC, "staging must divide evenly");
  double* As = lds;                  // [2][KC][ALD]
  double* Bs = lds + 2 * KC * ALD;   // [2][KC][BLD]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int l16 = lane & 15, lg = lane >> 4;

  d4 acc[RB][CB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * WTM + rb * 16 + l16, col = wn * WTN + cb * 16 + 4 * i + lg;
        // out-of-range lanes read a clamped in-range address and discard it,
        // so that every load is unconditional
        const double v = C[(int64_t)imin(col, N - 1) * ld + imin(row, M - 1)];
        acc[rb][cb][i] = ((row < M) & (col < N)) ? v : 0.0;
      }

  double ra[NA], rbv[NB];
  const int nch = (K + KC - 1) / KC;
  // Byte offsets from the (wave-uniform) panel bases fit in 32 bits: a tile
  // column block spans at most 512 columns of a matrix of order <= 614400.
  const char* Ab = reinterpret_cast<const char*>(Ap);
  const char* Bb = reinterpret_cast<const char*>(Bp);
  const uint32_t ld8 = (uint32_t)ld * 8u;
#define GEMM_GLOAD(k0)                                                                 \
  _Pragma("unroll") for (int s = 0; s < NA; ++s) {                                     \
    const int idx = tid + NT * s, r = idx % BM, k = (k0) + idx / BM;                   \
    const double v = *reinterpret_cast<const double*>(Ab + ((uint32_t)imin(k, K - 1) * ld8 + (uint32_t)imin(r, M - 1) * 8u)); \
    ra[s] = ((r < M) & (k < K)) ? v : 0.0;                                               \
  }                                                                                    \
  _Pragma("unroll") for (int s = 0; s < NB; ++s) {                                     \
    const int idx = tid + NT * s, r = idx % BN, k = (k0) + idx / BN;                   \
    const double v = *reinterpret_cast<const double*>(Bb + ((uint32_t)imin(k, K - 1) * ld8 + (uint32_t)imin(r, N - 1) * 8u)); \
    rbv[s] = ((r < N) & (k < K)) ? v : 0.0;                                               \
  }
#define GEMM_LSTORE(st)                                                  \
  _Pragma("unroll") for (int s = 0; s < NA; ++s) {                       \
    const int idx = tid + NT * s;                                        \
    As[((st) * KC + idx / BM) * ALD + idx % BM] = ra[s];                 \
  }                                                                      \
  _Pragma("unroll") for (int s = 0; s < NB; ++s) {                       \
    const int idx = tid + NT * s;                                        \
    Bs[((st) * KC + idx / BN) * BLD + idx % BN] = rbv[s];                \
  }
  GEMM_GLOAD(0)
  GEMM_LSTORE(0)
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int st = ch & 1;
    if (ch + 1 < nch) { GEMM_GLOAD((ch + 1) * KC) }
    const double* as = As + st * KC * ALD;
    const double* bs = Bs + st * KC * BLD;
#pragma unroll 2
    for (int ks = 0; ks < KC / 4; ++ks) {
      double fa[RB], fb[CB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) fa[rb] = -as[(ks * 4 + lg) * ALD + wm * WTM + rb * 16 + l16];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) fb[cb] = bs[(ks * 4 + lg) * BLD + wn * WTN + cb * 16 + l16];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma_f64(fb[cb], fa[rb], acc[rb][cb]);
    }
    if (ch + 1 < nch) { GEMM_LSTORE(st ^ 1) }
    __syncthreads();
  }
#undef GEMM_GLOAD
#undef GEMM_LSTORE

#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * WTM + rb * 16 + l16, col = wn * WTN + cb * 16 + 4 * i + lg;
        if (row < M && col < N && (!lower_only || row >= col)) C[(int64_t)col * ld + row] = acc[rb][cb][i];
      }
}

// GEMM / SYRK work item: a 128 x 128 sub-tile of C, K = nb.
#define GB 128
__device__ __forceinline__ void gemm_nt(double* C, const double* Ap, const double* Bp, int64_t ld, int M, int N,
                                        int K, bool lower_only, double* lds) {
  gemm_core<GB, GB, 16, 2>(C, Ap, Bp, ld, M, N, K, lower_only, lds);
}

// ---------------------------------------------------------------------------
// POTRF work item: Akk (m x m, m <= 512) := chol(Akk), lower, in place.
// Left-looking by panels of PW columns.  For each panel: the matrix cores
// apply all earlier columns to it (a 512 x 32 product with K = the panel's
// offset), the panel is loaded into LDS, its columns are factored one by one
// (sqrt, division, rank-1 update of the panel's later columns) and it is
// written back.  Returns 0, or the 1-based column (within the tile) whose
// pivot is not positive.
#define PW 32
#define PLD 512

__device__ __forceinline__ int potrf_tile(double* __restrict__ Akk, int64_t ld, int m, double* lds) {
  double* Ps = lds;  // [PW][PLD]
  const int tid = threadIdx.x;
  for (int c0 = 0; c0 < m; c0 += PW) {
    const int w = imin(PW, m - c0);
    const int R = m - c0;
    double* P = Akk + (int64_t)c0 * ld + c0;
    if (c0 > 0) {
      gemm_core<PLD, PW, 8, 4>(P, Akk + c0, Akk + c0, ld, R, w, c0, true, lds);
      __syncthreads();
    }
    for (int c = 0; c < w; ++c)
      for (int r = c + tid; r < R; r += NT) Ps[c * PLD + r] = P[(int64_t)c * ld + r];
    __syncthreads();
    for (int cc = 0; cc < w; ++cc) {
      const double d = Ps[cc * PLD + cc];
      if (!(d > 0.0)) return c0 + cc + 1;
      const double lkk = sqrt(d);
      __syncthreads();
      for (int r = cc + 1 + tid; r < R; r += NT) Ps[cc * PLD + r] = Ps[cc * PLD + r] / lkk;
      if (tid == 0) Ps[cc * PLD + cc] = lkk;
      __syncthreads();
      for (int c2 = cc + 1; c2 < w; ++c2) {
        const double l2 = Ps[cc * PLD + c2];
        for (int r = c2 + tid; r < R; r += NT) Ps[c2 * PLD + r] -= Ps[cc * PLD + r] * l2;
      }
      __syncthreads();
    }
    for (int c = 0; c < w; ++c)
      for (int r = c + tid; r < R; r += NT) P[(int64_t)c * ld + r] = Ps[c * PLD + r];
    __syncthreads();
  }
  return 0;
}

// ---------------------------------------------------------------------------
// TRSM work item: a strip of S <= 32 rows of A_ik, X := X L_kk^{-T}
// (mk = order of L_kk, a multiple of 16).  The strip lives in LDS.  For each
// block of 16 columns: one wavefront solves the 16x16 triangle by forward
// substitution (each lane one row, in registers), then the matrix cores
// subtract the block's contribution from every later column of the strip.
#define TS 32

__device__ __forceinline__ void trsm_strip(double* __restrict__ X, const double* __restrict__ Lkk, int64_t ld, int S, int mk,
                           double* lds) {
  double* Xs = lds;               // [mk][TS]
  double* Ld = lds + 512 * TS;    // [16][17] diagonal block of L_kk
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  {
    const int r = tid & (TS - 1);
    for (int c = tid / TS; c < mk; c += NT / TS) Xs[c * TS + r] = (r < S) ? X[(int64_t)c * ld + r] : 0.0;
  }
  __syncthreads();
  for (int q0 = 0; q0 < mk; q0 += 16) {
    {
      const int a = tid >> 4, b = tid & 15;
      Ld[a * 17 + b] = (a >= b) ? Lkk[(int64_t)(q0 + b) * ld + q0 + a] : 0.0;
    }
    __syncthreads();
    if (tid < TS) {
      double x[16];
#pragma unroll
      for (int b = 0; b < 16; ++b) x[b] = Xs[(q0 + b) * TS + tid];
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        x[b] = x[b] / Ld[b * 17 + b];
#pragma unroll
        for (int a = b + 1; a < 16; ++a) x[a] -= x[b] * Ld[a * 17 + b];
      }
#pragma unroll
      for (int b = 0; b < 16; ++b) Xs[(q0 + b) * TS + tid] = x[b];
    }
    __syncthreads();
    // X[:, c2] -= X[:, q0:q0+16] L[c2, q0:q0+16]^T for the later column blocks
    const int ncb = (mk - q0 - 16) >> 4;
    for (int u = wave; u < 2 * ncb; u += 4) {
      const int rbk = u & 1, cbase = q0 + 16 + (u >> 1) * 16;
      d4 acc;
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = Xs[(cbase + 4 * i + lg) * TS + rbk * 16 + l16];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int q = q0 + kk * 4 + lg;
        const double fa = -Xs[q * TS + rbk * 16 + l16];
        const double fb = Lkk[(int64_t)q * ld + cbase + l16];
        acc = mfma_f64(fb, fa, acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) Xs[(cbase + 4 * i + lg) * TS + rbk * 16 + l16] = acc[i];
    }
    __syncthreads();
  }
  {
    const int r = tid & (TS - 1);
    if (r < S)
      for (int c = tid / TS; c < mk; c += NT / TS) X[(int64_t)c * ld + r] = Xs[c * TS + r];
  }
}

// ---------------------------------------------------------------------------
// Solve work items.  Right-hand sides are processed 16 columns at a time,
// staged in LDS as Ys[j][r] (16 x 512).
#define YLD 512

__device__ __forceinline__ void stage_rhs(double* Ys, const double* Bk, int64_t ldb, int m, int j0, int jn) {
  for (int idx = threadIdx.x; idx < 16 * YLD; idx += NT) {
    const int j = idx / YLD, r = idx % YLD;
    Ys[idx] = (j < jn && r < m) ? Bk[(int64_t)(j0 + j) * ldb + r] : 0.0;
  }
}

__device__ __forceinline__ void unstage_rhs(const double* Ys, double* Bk, int64_t ldb, int m, int j0, int jn) {
  for (int idx = threadIdx.x; idx < 16 * YLD; idx += NT) {
    const int j = idx / YLD, r = idx % YLD;
    if (j < jn && r < m) Bk[(int64_t)(j0 + j) * ldb + r] = Ys[idx];
  }
}

// Y_k := L_kk^{-1} B_k, forward substitution by blocks of 16 rows.
__device__ __forceinline__ void ftrsv(const double* __restrict__ Lkk, int64_t ld, double* Bk, int64_t ldb, int m, int nrhs,
                      double* lds) {
  double* Ys = lds;
  const int tid = threadIdx.x;
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    const int jn = imin(16, nrhs - j0);
    stage_rhs(Ys, Bk, ldb, m, j0, jn);
    __syncthreads();
    for (int r0 = 0; r0 < m; r0 += 16) {
      const int bw = imin(16, m - r0);
      if (tid < 16) {
        double* y = Ys + tid * YLD + r0;
        for (int a = 0; a < bw; ++a) {
          double s = y[a];
          for (int b = 0; b < a; ++b) s -= Lkk[(int64_t)(r0 + b) * ld + r0 + a] * y[b];
          y[a] = s / Lkk[(int64_t)(r0 + a) * ld + r0 + a];
        }
      }
      __syncthreads();
      const int rl = tid & 63, jg = tid >> 6;
      for (int r = r0 + bw + rl; r < m; r += 64) {
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int b = 0; b < bw; ++b) {
          const double l = Lkk[(int64_t)(r0 + b) * ld + r];
          s0 += l * Ys[(jg * 4 + 0) * YLD + r0 + b];
          s1 += l * Ys[(jg * 4 + 1) * YLD + r0 + b];
          s2 += l * Ys[(jg * 4 + 2) * YLD + r0 + b];
          s3 += l * Ys[(jg * 4 + 3) * YLD + r0 + b];
        }
        Ys[(jg * 4 + 0) * YLD + r] -= s0;
        Ys[(jg * 4 + 1) * YLD + r] -= s1;
        Ys[(jg * 4 + 2) * YLD + r] -= s2;
        Ys[(jg * 4 + 3) * YLD + r] -= s3;
      }
      __syncthreads();
    }
    unstage_rhs(Ys, Bk, ldb, m, j0, jn);
    __syncthreads();
  }
}

// X_k := L_kk^{-T} Y_k, backward substitution by blocks of 16 rows.
__device__ __forceinline__ void btrsv(const double* __restrict__ Lkk, int64_t ld, double* Bk, int64_t ldb, int m, int nrhs,
                      double* lds) {
  double* Ys = lds;
  const int tid = threadIdx.x;
  const int nblk = (m + 15) >> 4;
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    const int jn = imin(16, nrhs - j0);
    stage_rhs(Ys, Bk, ldb, m, j0, jn);
    __syncthreads();
    for (int rb = nblk - 1; rb >= 0; --rb) {
      const int r0 = rb * 16, bw = imin(16, m - r0);
      if (tid < 16) {
        double* y = Ys + tid * YLD + r0;
        for (int a = bw - 1; a >= 0; --a) {
          double s = y[a];
          for (int b = a + 1; b < bw; ++b) s -= Lkk[(int64_t)(r0 + a) * ld + r0 + b] * y[b];
          y[a] = s / Lkk[(int64_t)(r0 + a) * ld + r0 + a];
        }
      }
      __syncthreads();
      const int rl = tid & 63, jg = tid >> 6;
      for (int r = rl; r < r0; r += 64) {
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        const double* colr = Lkk + (int64_t)r * ld + r0;  // L[r0 + b][r], contiguous in b
        for (int b = 0; b < bw; ++b) {
          const double l = colr[b];
          s0 += l * Ys[(jg * 4 + 0) * YLD + r0 + b];
          s1 += l * Ys[(jg * 4 + 1) * YLD + r0 + b];
          s2 += l * Ys[(jg * 4 + 2) * YLD + r0 + b];
          s3 += l * Ys[(jg * 4 + 3) * YLD + r0 + b];
        }
        Ys[(jg * 4 + 0) * YLD + r] -= s0;
        Ys[(jg * 4 + 1) * YLD + r] -= s1;
        Ys[(jg * 4 + 2) * YLD + r] -= s2;
        Ys[(jg * 4 + 3) * YLD + r] -= s3;
      }
      __syncthreads();
    }
    unstage_rhs(Ys, Bk, ldb, m, j0, jn);
    __syncthreads();
  }
}

// B_i[rows] -= L_ik[rows, :] Y_k  (forward update), rows = a strip of <= 128.
__device__ __forceinline__ void fgemv(const double* __restrict__ Lik, int64_t ld, double* Bi, const double* Yk, int64_t ldb,
                      int rows, int mk, int nrhs, double* lds) {
  double* Ys = lds;
  const int tid = threadIdx.x, r = tid & 127, jh = tid >> 7;
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    const int jn = imin(16, nrhs - j0);
    stage_rhs(Ys, Yk, ldb, mk, j0, jn);
    __syncthreads();
    if (r < rows) {
      double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int c = 0; c < mk; ++c) {
        const double l = Lik[(int64_t)c * ld + r];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) s[jj] += l * Ys[(jh * 8 + jj) * YLD + c];
      }
#pragma unroll
      for (int jj = 0; jj < 8; ++jj)
        if (jh * 8 + jj < jn) Bi[(int64_t)(j0 + jh * 8 + jj) * ldb + r] -= s[jj];
    }
    __syncthreads();
  }
}

// Y_i[cols] -= L_ki[:, cols]^T X_k  (backward update), cols = a strip of <= 128.
__device__ __forceinline__ void bgemv(const double* __restrict__ Lki, int64_t ld, double* Yi, const double* Xk, int64_t ldb,
                      int cols, int mk, int nrhs, double* lds) {
  double* Xs = lds;
  const int tid = threadIdx.x, c = tid & 127, jh = tid >> 7;
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    const int jn = imin(16, nrhs - j0);
    stage_rhs(Xs, Xk, ldb, mk, j0, jn);
    __syncthreads();
    if (c < cols) {
      double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      const double* colc = Lki + (int64_t)c * ld;
      for (int r = 0; r < mk; ++r) {
        const double l = colc[r];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) s[jj] += l * Xs[(jh * 8 + jj) * YLD + r];
      }
#pragma unroll
      for (int jj = 0; jj < 8; ++jj)
        if (jh * 8 + jj < jn) Yi[(int64_t)(j0 + jh * 8 + jj) * ldb + c] -= s[jj];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// scheduler
__device__ __forceinline__ int ld_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t tile_size(const KArgs& a, int t) {
  const int64_t r = a.n - (int64_t)t * a.nb;
  return r < a.nb ? r : a.nb;
}

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Executed by a whole wavefront with every decision made wave-uniform
// (readfirstlane), so the compiler keeps the control flow scalar: a barrier
// must never end up inside lane-masked loop structure.  Waits until the
// task's counter reaches zero; false when the run is being aborted or the
// wait exceeded its bound.
__device__ __forceinline__ bool wait_ready(const KArgs& a, int task, int lane) {
  if (uniform_i(ld_relaxed(&a.dep[task])) == 0) return uniform_i(ld_relaxed(&a.hdr[HDR_ABORT])) == 0;
  const uint64_t t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(2);
    if (uniform_i(ld_relaxed(&a.dep[task])) == 0) break;
    if (uniform_i(ld_relaxed(&a.hdr[HDR_ABORT])) != 0) return false;
    if ((int64_t)(wall_clock64() - t0) > a.wait_limit) {
      if (lane == 0) {
        __hip_atomic_store(&a.hdr[HDR_ERROR], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.hdr[HDR_ABORT], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      return false;
    }
  }
  return uniform_i(ld_relaxed(&a.hdr[HDR_ABORT])) == 0;
}

__global__ void __launch_bounds__(NT, 1) tchol_persistent(KArgs a) {
  __shared__ double lds[LDS_DOUBLES];
  __shared__ int s_claim[3];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = uniform_i(tid >> 6);
  for (;;) {
    // claim: wavefront 0 takes the next ticket and waits for its task
    if (wave == 0) {
      int t = 0;
      if (lane == 0) t = __hip_atomic_fetch_add(&a.hdr[HDR_TICKET], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      t = uniform_i(t);
      int task = -1, part = 0;
      uint64_t tw = 0;
      if (t < a.nitem) {
        task = uniform_i(a.items[2 * t]);
        part = uniform_i(a.items[2 * t + 1]);
        if (a.trace) tw = wall_clock64();
        if (!wait_ready(a, task, lane)) task = -1;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (lane == 0) {
        s_claim[0] = task;
        s_claim[1] = part;
        s_claim[2] = t;
        if (a.trace && task >= 0) {
          a.trace[4 * (int64_t)t + 0] = tw;
          a.trace[4 * (int64_t)t + 1] = wall_clock64();
        }
      }
    }
    __syncthreads();
    const int task = uniform_i(s_claim[0]), part = uniform_i(s_claim[1]), ticket = uniform_i(s_claim[2]);
    if (task < 0) break;
    const int32_t* d = a.desc + DESC_WORDS * (int64_t)task;
    const int kind = uniform_i(d[0]), ti = uniform_i(d[1]), tj = uniform_i(d[2]), tk = uniform_i(d[3]);
    const int64_t ld = a.ld, nb = a.nb;
    int ok = 1;
    switch (kind) {
      case TK_POTRF: {
        double* Akk = a.A + (tk * nb) * ld + tk * nb;
        const int info = uniform_i(potrf_tile(Akk, ld, (int)tile_size(a, tk), lds));
        if (info != 0) {
          ok = 0;
          if (tid == 0) {
            __hip_atomic_store(&a.hdr[HDR_INFO], (int)(tk * nb) + info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.hdr[HDR_ABORT], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
        break;
      }
      case TK_TRSM: {
        const int r0 = part * a.trsm_rows;
        const int S = imin(a.trsm_rows, (int)tile_size(a, ti) - r0);
        trsm_strip(a.A + (tk * nb) * ld + ti * nb + r0, a.A + (tk * nb) * ld + tk * nb, ld, S, (int)tile_size(a, tk),
                   lds);
        break;
      }
      case TK_SYRK:
      case TK_GEMM: {
        int si, sj;
        if (kind == TK_SYRK) {
          si = 0;
          while ((si + 1) * (si + 2) / 2 <= part) ++si;
          sj = part - si * (si + 1) / 2;
        } else {
          const int ncj = (int)((tile_size(a, tj) + a.gemm_n - 1) / a.gemm_n);
          si = part / ncj;
          sj = part % ncj;
        }
        const int M = imin(a.gemm_m, (int)tile_size(a, ti) - si * a.gemm_m);
        const int N = imin(a.gemm_n, (int)tile_size(a, tj) - sj * a.gemm_n);
        double* C = a.A + (tj * nb + sj * a.gemm_n) * ld + ti * nb + si * a.gemm_m;
        const double* Ap = a.A + (tk * nb) * ld + ti * nb + si * a.gemm_m;
        const double* Bp = a.A + (tk * nb) * ld + tj * nb + sj * a.gemm_n;
        gemm_nt(C, Ap, Bp, ld, M, N, (int)tile_size(a, tk), kind == TK_SYRK && si == sj, lds);
        break;
      }
      case TK_FTRSV:
        ftrsv(a.A + (tk * nb) * ld + tk * nb, ld, a.B + tk * nb, a.ldb, (int)tile_size(a, tk), (int)a.nrhs, lds);
        break;
      case TK_BTRSV:
        btrsv(a.A + (tk * nb) * ld + tk * nb, ld, a.B + tk * nb, a.ldb, (int)tile_size(a, tk), (int)a.nrhs, lds);
        break;
      case TK_FGEMV: {
        const int r0 = part * a.gemv_rows;
        const int rows = imin(a.gemv_rows, (int)tile_size(a, ti) - r0);
        fgemv(a.A + (tk * nb) * ld + ti * nb + r0, ld, a.B + ti * nb + r0, a.B + tk * nb, a.ldb, rows,
              (int)tile_size(a, tk), (int)a.nrhs, lds);
        break;
      }
      case TK_BGEMV: {
        const int c0 = part * a.gemv_rows;
        const int cols = imin(a.gemv_rows, (int)tile_size(a, ti) - c0);
        bgemv(a.A + (ti * nb + c0) * ld + tk * nb, ld, a.B + ti * nb + c0, a.B + tk * nb, a.ldb, cols,
              (int)tile_size(a, tk), (int)a.nrhs, lds);
        break;
      }
      default:
        ok = 0;
        break;
    }
    // make this work item's stores visible device-wide, then activate
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (wave == 0 && ok) {
      int prev = 0;
      if (lane == 0) prev = __hip_atomic_fetch_add(&a.done[task], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      prev = uniform_i(prev);
      if (prev == uniform_i(d[4]) - 1) {
        const int e0 = uniform_i(d[5]), e1 = uniform_i(d[6]);
        for (int e = e0 + lane; e < e1; e += 64)
          __hip_atomic_fetch_sub(&a.dep[a.succ[e]], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (lane == 0) {
        __hip_atomic_fetch_add(&a.hdr[HDR_DONE], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a.trace) {
          a.trace[4 * (int64_t)ticket + 2] = wall_clock64();
          a.trace[4 * (int64_t)ticket + 3] = (uint64_t)(uint32_t)task | ((uint64_t)(uint32_t)blockIdx.x << 32);
        }
      }
    }
  }
}

// Clears the header and the per-task completion counters and copies the
// initial dependency counters; the plan's constant part is copied by the host.
__global__ void tchol_reset(int32_t* hdr, int32_t* dep, int32_t* done, const int32_t* dep0, int32_t ntask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < HDR_WORDS) hdr[i] = 0;
  if (i < ntask) {
    dep[i] = dep0[i];
    done[i] = 0;
  }
}

extern "C" hipError_t tchol_dev_launch(const KArgs* a, int32_t ntask, const int32_t* dep0, int grid,
                                       hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1) {
  const int rb = 256;
  const int64_t cover = ntask > HDR_WORDS ? ntask : HDR_WORDS;
  hipLaunchKernelGGL(tchol_reset, dim3((unsigned)((cover + rb - 1) / rb)), dim3(rb), 0, stream, a->hdr, a->dep,
                     a->done, dep0, ntask);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev0) {
    e = hipEventRecord(ev0, stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(tchol_persistent, dim3(grid), dim3(NT), 0, stream, *a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev1) e = hipEventRecord(ev1, stream);
  return e;
}

extern "C" hipError_t tchol_dev_max_grid(int device, int* grid) {
  int cus = 0, occ = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, tchol_persistent, NT, 0);
  if (e != hipSuccess) return e;
  *grid = cus * (occ > 0 ? occ : 1);
  return hipSuccess;
}
