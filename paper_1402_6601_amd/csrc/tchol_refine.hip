// Kernels of the mixed-precision solve's iterative refinement (the FP64
// side): the FP32 working copy of A, the residual R = B - A X with A
// symmetric and only its lower triangle read, column max-norms, and the
// update X += D.  The factorization and the correction solves themselves run
// on the persistent tile scheduler (tchol_device.hip).
//
// Refinement: x_0 = solve with the low-precision factor; repeat
// r = b - A x (FP64), stop when the normwise backward error
// ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf) meets the target, else
// x += solve(r).  The residual dominates nothing here: it is two passes over
// the lower triangle (HBM-bound); the correction solves dominate.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define RT 256  // threads per workgroup of these kernels

typedef double r4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int rimin(int a, int b) { return a < b ? a : b; }

// W[c * ldw + r] = (float) A[c * lda + r] for r >= c (r < n), 0 elsewhere in
// the first ldw rows of each of the n columns (the padding rows included).
__global__ void refine_convert(const double* __restrict__ A, int64_t lda, float* __restrict__ W, int64_t ldw,
                               int64_t n) {
  for (int64_t c = blockIdx.x; c < n; c += gridDim.x)
    for (int64_t r = threadIdx.x; r < ldw; r += RT) {
      float v = 0.f;
      if (r >= c && r < n) v = (float)A[c * lda + r];
      W[c * ldw + r] = v;
    }
}

// D_k := the lower triangle of A's diagonal tile k in FP64 (D: T tiles of
// nb x nb, ld nb): the diagonal tiles of the mixed-precision factorization.
__global__ void refine_diag(const double* __restrict__ A, int64_t lda, int64_t n, int64_t nb,
                            double* __restrict__ D) {
  const int64_t k = blockIdx.y;
  const int64_t m = n - k * nb < nb ? n - k * nb : nb;
  for (int64_t idx = (int64_t)blockIdx.x * RT + threadIdx.x; idx < m * m; idx += (int64_t)gridDim.x * RT) {
    const int64_t c = idx / m, r = idx - c * m;
    if (r >= c) D[k * nb * nb + c * nb + r] = A[(k * nb + c) * lda + k * nb + r];
  }
}

// The residual R = B - A X reads A by its lower triangle in two passes, each
// split into (128-row or 128-column strip) x (chunk of at most ck
// rows/columns of the other index) blocks so that every workgroup streams a
// similar amount of A; each block writes its partial product to a slot of
// its chunk, and a last kernel combines the slots in a fixed order
// (deterministic).  MFMA layout: A operand = the A fragment (rows on
// lanes % 16), B operand = the X fragment (right-hand sides on lanes % 16).

// Row pass: rows [r0, r0 + 128), columns [c*ck, ...) up to the strip's
// diagonal block: P1[c][j][r] = sum over those columns cc <= r of A[r][cc] X[cc][j].
// absmode: |A| and X = 1 (row sums of |A|, one column).
__global__ void __launch_bounds__(RT, 1) refine_rows(const double* __restrict__ A, int64_t lda, int64_t n,
                                                     const double* __restrict__ X, double* __restrict__ P1,
                                                     int64_t ldb, int nrhs, int absmode, int64_t ck) {
  __shared__ double Xs[16 * 516];  // X chunk: 512 rows x 16 RHS, Xs[j * 516 + k]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 128;
  const int64_t kend = r0 + 128 < n ? r0 + 128 : n;  // columns past the strip's diagonal block hold no lower entries
  const int64_t cbeg = (int64_t)blockIdx.y * ck;
  if (cbeg >= kend) return;
  const int64_t cend = cbeg + ck < kend ? cbeg + ck : kend;
  double* const Pc = P1 + (int64_t)blockIdx.y * n * (absmode ? 1 : nrhs);
  const int nj = absmode ? 1 : nrhs;
  for (int j0 = 0; j0 < nj; j0 += 16) {
    const int jn = rimin(16, nj - j0);
    r4 acc[2] = {r4{0, 0, 0, 0}, r4{0, 0, 0, 0}};
    const int64_t ra = r0 + (wave * 2) * 16 + l16, rb = ra + 16;  // A-fragment rows of the wave's two blocks
    for (int64_t kc = cbeg; kc < cend; kc += 512) {
      const int kw = (int)((cend - kc) < 512 ? (cend - kc) : 512);
      __syncthreads();
      for (int idx = tid; idx < 16 * 512; idx += RT) {
        const int j = idx >> 9, k = idx & 511;
        double v = 0.0;
        if (j < jn && k < kw) v = absmode ? 1.0 : X[(int64_t)(j0 + j) * ldb + kc + k];
        Xs[j * 516 + k] = v;
      }
      __syncthreads();
      for (int kb = 0; kb < kw; kb += 32) {
        double f0[8], f1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t c = kc + rimin(kb + 4 * u + lg, kw - 1);
          f0[u] = A[c * lda + (ra < n ? ra : n - 1)];
          f1[u] = A[c * lda + (rb < n ? rb : n - 1)];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = kb + 4 * u + lg;
          const int64_t c = kc + k;
          double a0 = (k < kw && ra < n && ra >= c) ? f0[u] : 0.0;
          double a1 = (k < kw && rb < n && rb >= c) ? f1[u] : 0.0;
          if (absmode) {
            a0 = fabs(a0);
            a1 = fabs(a1);
          }
          const double fx = Xs[l16 * 516 + rimin(k, 511)];
          acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, fx, acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, fx, acc[1], 0, 0, 0);
        }
      }
    }
    if (l16 < jn) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t r = r0 + (wave * 2 + t) * 16 + 4 * i + lg;
          if (r < n) Pc[(int64_t)(j0 + l16) * n + r] = acc[t][i];
        }
    }
  }
}

// Column pass: columns [c0, c0 + 128) of A, rows [max(c0, c*ck), ...):
// P2[c][j][cc] = sum over those rows r > cc of A[r][cc] X[r][j] (the
// strictly lower part read by columns: the strictly upper part of the
// symmetric A applied to X).  absmode: row sums of |A| as above.
__global__ void __launch_bounds__(RT, 1) refine_cols(const double* __restrict__ A, int64_t lda, int64_t n,
                                                     const double* __restrict__ X, double* __restrict__ P2,
                                                     int64_t ldb, int nrhs, int absmode, int64_t ck) {
  __shared__ double Xs[16 * 516];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * 128;
  const int64_t rb0 = (int64_t)blockIdx.y * ck;
  const int64_t rbeg = rb0 > c0 ? rb0 : c0;
  const int64_t rend = rb0 + ck < n ? rb0 + ck : n;
  if (rbeg >= rend) return;
  double* const Pc = P2 + (int64_t)blockIdx.y * n * (absmode ? 1 : nrhs);
  const int nj = absmode ? 1 : nrhs;
  for (int j0 = 0; j0 < nj; j0 += 16) {
    const int jn = rimin(16, nj - j0);
    r4 acc[2] = {r4{0, 0, 0, 0}, r4{0, 0, 0, 0}};
    const int64_t ca = c0 + (wave * 2) * 16 + l16, cb = ca + 16;  // A^T fragment rows = columns of A
    const int64_t caa = ca < n ? ca : n - 1, cbb = cb < n ? cb : n - 1;
    for (int64_t kc = rbeg; kc < rend; kc += 512) {  // rows of A
      const int kw = (int)((rend - kc) < 512 ? (rend - kc) : 512);
      __syncthreads();
      for (int idx = tid; idx < 16 * 512; idx += RT) {
        const int j = idx >> 9, k = idx & 511;
        double v = 0.0;
        if (j < jn && k < kw) v = absmode ? 1.0 : X[(int64_t)(j0 + j) * ldb + kc + k];
        Xs[j * 516 + k] = v;
      }
      __syncthreads();
      for (int kb = 0; kb < kw; kb += 32) {
        double f0[8], f1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t r = kc + rimin(kb + 4 * u + lg, kw - 1);
          f0[u] = A[caa * lda + r];
          f1[u] = A[cbb * lda + r];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = kb + 4 * u + lg;
          const int64_t r = kc + k;
          double a0 = (k < kw && ca < n && r > ca) ? f0[u] : 0.0;
          double a1 = (k < kw && cb < n && r > cb) ? f1[u] : 0.0;
          if (absmode) {
            a0 = fabs(a0);
            a1 = fabs(a1);
          }
          const double fx = Xs[l16 * 516 + rimin(k, 511)];
          acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, fx, acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, fx, acc[1], 0, 0, 0);
        }
      }
    }
    if (l16 < jn) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t c = c0 + (wave * 2 + t) * 16 + 4 * i + lg;
          if (c < n) Pc[(int64_t)(j0 + l16) * n + c] = acc[t][i];
        }
    }
  }
}

// Out = Bin - (sum of the row pass's slots) - (sum of the column pass's
// slots), chunks ascending; absmode: Out = the sums (row sums of |A|).
// A chunk's slot holds a value for row r only if that chunk has a block
// covering r; the same rules as the passes decide which.
__global__ void refine_combine(const double* __restrict__ Bin, double* __restrict__ Out, const double* __restrict__ P1,
                               const double* __restrict__ P2, int64_t n, int64_t ldb, int nrhs, int absmode,
                               int64_t ck, int nchunk) {
  const int nj = absmode ? 1 : nrhs;
  const int64_t tot = n * nj;
  for (int64_t idx = (int64_t)blockIdx.x * RT + threadIdx.x; idx < tot; idx += (int64_t)gridDim.x * RT) {
    const int64_t j = idx / n, r = idx - j * n;
    const int64_t s0 = r / 128 * 128;
    const int64_t kend = s0 + 128 < n ? s0 + 128 : n;
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) {
      if ((int64_t)c * ck < kend) acc += P1[(int64_t)c * n * nj + j * n + r];
      const int64_t rb0 = (int64_t)c * ck, rbeg = rb0 > s0 ? rb0 : s0, rend = rb0 + ck < n ? rb0 + ck : n;
      if (rbeg < rend) acc += P2[(int64_t)c * n * nj + j * n + r];
    }
    Out[j * ldb + r] = absmode ? acc : Bin[j * ldb + r] - acc;
  }
}

// out[j] = max_r |V[j * ldv + r]| for the ncols columns (one workgroup each).
__global__ void __launch_bounds__(RT) refine_colmax(const double* __restrict__ V, int64_t ldv, int64_t n,
                                                    double* __restrict__ out) {
  __shared__ double red[RT];
  const int j = blockIdx.x;
  double m = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += RT) m = fmax(m, fabs(V[(int64_t)j * ldv + r]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = RT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

// X += D (count elements).
__global__ void refine_axpy(double* __restrict__ X, const double* __restrict__ D, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < count; i += (int64_t)gridDim.x * RT) X[i] += D[i];
}

extern "C" hipError_t tchol_refine_diag(const double* A, int64_t lda, int64_t n, int64_t nb, double* D,
                                        hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t T = (n + nb - 1) / nb;
  const int64_t g = (nb * nb + RT - 1) / RT;
  hipLaunchKernelGGL(refine_diag, dim3((unsigned)(g < 64 ? g : 64), (unsigned)T), dim3(RT), 0, s, A, lda, n, nb, D);
  return hipGetLastError();
}

extern "C" hipError_t tchol_refine_convert(const double* A, int64_t lda, float* W, int64_t ldw, int64_t n,
                                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(refine_convert, dim3((unsigned)(n < 16384 ? n : 16384)), dim3(RT), 0, s, A, lda, W, ldw, n);
  return hipGetLastError();
}

// Chunk length of the residual's passes: at most 8 chunks, each a multiple of 512.
extern "C" int64_t tchol_refine_chunk(int64_t n) {
  const int64_t c = (n + 7) / 8;
  const int64_t ck = (c + 511) / 512 * 512;
  return ck < 4096 ? 4096 : ck;
}

// Out = Bin - A X (absmode: Out = |A| 1, the row sums of |A|); Out may equal
// Bin.  P: scratch of 2 * 8 * n * max(nrhs, 1) doubles for the partial sums.
extern "C" hipError_t tchol_refine_residual(const double* A, int64_t lda, int64_t n, const double* X,
                                            const double* Bin, double* Out, int64_t ldb, int nrhs, int absmode,
                                            double* P, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t ck = tchol_refine_chunk(n);
  const int nchunk = (int)((n + ck - 1) / ck);
  const int64_t slot = 8 * n * (int64_t)(nrhs > 1 ? nrhs : 1);
  double* P1 = P;
  double* P2 = P + slot;
  const unsigned g = (unsigned)((n + 127) / 128);
  hipLaunchKernelGGL(refine_rows, dim3(g, (unsigned)nchunk), dim3(RT), 0, s, A, lda, n, X, P1, ldb, nrhs, absmode, ck);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(refine_cols, dim3(g, (unsigned)nchunk), dim3(RT), 0, s, A, lda, n, X, P2, ldb, nrhs, absmode, ck);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tot = n * (absmode ? 1 : nrhs);
  const int64_t gb = (tot + RT - 1) / RT;
  hipLaunchKernelGGL(refine_combine, dim3((unsigned)(gb < 8192 ? gb : 8192)), dim3(RT), 0, s, Bin, Out, P1, P2, n, ldb,
                     nrhs, absmode, ck, nchunk);
  return hipGetLastError();
}

extern "C" hipError_t tchol_refine_colmax(const double* V, int64_t ldv, int64_t n, int ncols, double* out,
                                          hipStream_t s) {
  if (ncols == 0) return hipSuccess;
  hipLaunchKernelGGL(refine_colmax, dim3((unsigned)ncols), dim3(RT), 0, s, V, ldv, n, out);
  return hipGetLastError();
}

extern "C" hipError_t tchol_refine_axpy(double* X, const double* D, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const int64_t g = (count + RT - 1) / RT;
  hipLaunchKernelGGL(refine_axpy, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(RT), 0, s, X, D, count);
  return hipGetLastError();
}
