// Data movement around the batched FP32 launch.  The systems live in FP32
// (A_s with leading dimension lda_s, B_s with leading dimension n_s); the
// persistent kernel keeps each system's diagonal tiles in FP64 (their
// SYRK updates, POTRF, inverses) and runs the solves in FP64 on a compact
// FP64 copy of the right-hand sides.  Before the launch: diagonal tiles
// A_s,kk -> D (lower triangles) and B -> Bd.  After it: the factored
// diagonal tiles D -> A (lower, rounded) and the solutions Bd -> B.
//
// desc: per system, 8 words: a_off, lda, n, nb, d_off, b_off, bd_off, own
// (a_off and b_off in floats from A and B, d_off and bd_off in doubles
// from D and Bd; D holds T_s tiles of nb_s x nb_s per system; own != 0: the
// launch itself reads A_s and writes L_s back, only B is staged).
#include <hip/hip_runtime.h>
#include <stdint.h>

#define BT 256

// Columns of the diagonal tiles are dealt to the wavefronts of the x blocks
// (one division per column, not per entry); a wavefront moves its column's
// rows four 64-row runs at a time, their loads issued before their stores.
__global__ void b32_prepare(const int64_t* __restrict__ desc, int32_t batch, const float* __restrict__ A,
                            const float* __restrict__ B, double* __restrict__ D, double* __restrict__ Bd, int nrhs) {
  for (int32_t sy = blockIdx.y; sy < batch; sy += gridDim.y) {
    const int64_t* d = desc + 8 * (int64_t)sy;
    const int64_t a_off = d[0], lda = d[1], d_off = d[4], b_off = d[5], bd_off = d[6];
    const int n = (int)d[2], nb = (int)d[3];
    const int T = d[7] != 0 ? 0 : (n + nb - 1) / nb;  // own: no diagonal tiles to move
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int col = blockIdx.x * (BT / 64) + wave; col < T * nb; col += gridDim.x * (BT / 64)) {
      const int k = col / nb, c = col - k * nb;
      const int m = n - k * nb < nb ? n - k * nb : nb;
      if (c >= m) continue;
      const float* src = A + a_off + (int64_t)(k * nb + c) * lda + k * nb;
      double* dst = D + d_off + (int64_t)k * nb * nb + (int64_t)c * nb;
      for (int r0 = c; r0 < m; r0 += 4 * 64) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = r0 + lane + 64 * u;
          v[u] = r < m ? src[r] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = r0 + lane + 64 * u;
          if (r < m) dst[r] = (double)v[u];
        }
      }
    }
    for (int64_t idx = (int64_t)blockIdx.x * BT + threadIdx.x; idx < (int64_t)n * nrhs; idx += (int64_t)gridDim.x * BT)
      Bd[bd_off + idx] = (double)B[b_off + idx];
  }
}

__global__ void b32_finish(const int64_t* __restrict__ desc, int32_t batch, float* __restrict__ A,
                           float* __restrict__ B, const double* __restrict__ D, const double* __restrict__ Bd, int nrhs) {
  for (int32_t sy = blockIdx.y; sy < batch; sy += gridDim.y) {
    const int64_t* d = desc + 8 * (int64_t)sy;
    const int64_t a_off = d[0], lda = d[1], d_off = d[4], b_off = d[5], bd_off = d[6];
    const int n = (int)d[2], nb = (int)d[3];
    const int T = d[7] != 0 ? 0 : (n + nb - 1) / nb;  // own: no diagonal tiles to move
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int col = blockIdx.x * (BT / 64) + wave; col < T * nb; col += gridDim.x * (BT / 64)) {
      const int k = col / nb, c = col - k * nb;
      const int m = n - k * nb < nb ? n - k * nb : nb;
      if (c >= m) continue;
      float* dst = A + a_off + (int64_t)(k * nb + c) * lda + k * nb;
      const double* src = D + d_off + (int64_t)k * nb * nb + (int64_t)c * nb;
      for (int r0 = c; r0 < m; r0 += 4 * 64) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = r0 + lane + 64 * u;
          v[u] = r < m ? src[r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = r0 + lane + 64 * u;
          if (r < m) dst[r] = (float)v[u];
        }
      }
    }
    for (int64_t idx = (int64_t)blockIdx.x * BT + threadIdx.x; idx < (int64_t)n * nrhs; idx += (int64_t)gridDim.x * BT)
      B[b_off + idx] = (float)Bd[bd_off + idx];
  }
}

extern "C" hipError_t tchol_b32_prepare(const int64_t* desc, int32_t batch, const float* A, const float* B, double* D,
                                        double* Bd, int nrhs, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  const unsigned gy = (unsigned)(batch < 32768 ? batch : 32768);
  hipLaunchKernelGGL(b32_prepare, dim3(16, gy), dim3(BT), 0, s, desc, batch, A, B, D, Bd, nrhs);
  return hipGetLastError();
}

extern "C" hipError_t tchol_b32_finish(const int64_t* desc, int32_t batch, float* A, float* B, const double* D,
                                       const double* Bd, int nrhs, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  const unsigned gy = (unsigned)(batch < 32768 ? batch : 32768);
  hipLaunchKernelGGL(b32_finish, dim3(16, gy), dim3(BT), 0, s, desc, batch, A, B, D, Bd, nrhs);
  return hipGetLastError();
}
