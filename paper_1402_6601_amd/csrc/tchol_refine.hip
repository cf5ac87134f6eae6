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

// Row pass: for the 128-row strip [r0, r0 + 128) and 16 right-hand sides
// starting at j0, Out = Bin - sum over columns c <= r of A[r][c] X[c][:]
// (rows below the strip's diagonal block are not read: entries above the
// diagonal are masked).  With absmode, |A| and X = 1 give row sums of the
// lower triangle (Bin, X ignored).  MFMA layout: A operand = A fragment
// (rows on lanes % 16), B operand = X fragment (right-hand sides on lanes % 16).
__global__ void __launch_bounds__(RT, 1) refine_rows(const double* __restrict__ A, int64_t lda, int64_t n,
                                                     const double* __restrict__ X, const double* __restrict__ Bin,
                                                     double* __restrict__ Out, int64_t ldb, int nrhs, int absmode) {
  __shared__ double Xs[16 * 516];  // X chunk: 512 rows x 16 RHS, Xs[j * 516 + k]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 128;
  const int64_t kend = r0 + 128 < n ? r0 + 128 : n;  // columns 0 .. kend-1 may hold lower entries of the strip
  for (int j0 = 0; j0 < (absmode ? 1 : nrhs); j0 += 16) {
    const int jn = absmode ? 1 : rimin(16, nrhs - j0);
    r4 acc[2] = {r4{0, 0, 0, 0}, r4{0, 0, 0, 0}};
    const int64_t ra = r0 + (wave * 2) * 16 + l16, rb = ra + 16;  // A-fragment rows of the wave's two blocks
    for (int64_t kc = 0; kc < kend; kc += 512) {
      const int kw = (int)((kend - kc) < 512 ? (kend - kc) : 512);
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
          if (r < n) {
            const int64_t o = (int64_t)(j0 + l16) * ldb + r;
            Out[o] = absmode ? acc[t][i] : Bin[o] - acc[t][i];
          }
        }
    }
  }
}

// Column pass: for the 128-column strip [c0, c0 + 128), Out[c][:] -=
// sum over rows r > c of A[r][c] X[r][:] (the strictly lower part read by
// columns, i.e. the strictly upper part of the symmetric A applied to X).
// With absmode, Out[c] += sum over r > c of |A[r][c]| (row sums of |A|).
__global__ void __launch_bounds__(RT, 1) refine_cols(const double* __restrict__ A, int64_t lda, int64_t n,
                                                     const double* __restrict__ X, double* __restrict__ Out,
                                                     int64_t ldb, int nrhs, int absmode) {
  __shared__ double Xs[16 * 516];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * 128;
  for (int j0 = 0; j0 < (absmode ? 1 : nrhs); j0 += 16) {
    const int jn = absmode ? 1 : rimin(16, nrhs - j0);
    r4 acc[2] = {r4{0, 0, 0, 0}, r4{0, 0, 0, 0}};
    const int64_t ca = c0 + (wave * 2) * 16 + l16, cb = ca + 16;  // A^T fragment rows = columns of A
    const int64_t caa = ca < n ? ca : n - 1, cbb = cb < n ? cb : n - 1;
    for (int64_t kc = c0; kc < n; kc += 512) {  // rows of A
      const int kw = (int)((n - kc) < 512 ? (n - kc) : 512);
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
          if (c < n) {
            const int64_t o = (int64_t)(j0 + l16) * ldb + c;
            Out[o] = absmode ? Out[o] + acc[t][i] : Out[o] - acc[t][i];
          }
        }
    }
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

extern "C" hipError_t tchol_refine_convert(const double* A, int64_t lda, float* W, int64_t ldw, int64_t n,
                                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(refine_convert, dim3((unsigned)(n < 16384 ? n : 16384)), dim3(RT), 0, s, A, lda, W, ldw, n);
  return hipGetLastError();
}

// Out = Bin - A X (absmode: Out = |A| 1, row sums of |A|); Out may equal Bin.
extern "C" hipError_t tchol_refine_residual(const double* A, int64_t lda, int64_t n, const double* X,
                                            const double* Bin, double* Out, int64_t ldb, int nrhs, int absmode,
                                            hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned g = (unsigned)((n + 127) / 128);
  hipLaunchKernelGGL(refine_rows, dim3(g), dim3(RT), 0, s, A, lda, n, X, Bin, Out, ldb, nrhs, absmode);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(refine_cols, dim3(g), dim3(RT), 0, s, A, lda, n, X, Out, ldb, nrhs, absmode);
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
