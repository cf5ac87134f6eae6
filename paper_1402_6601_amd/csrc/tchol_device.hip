// Device side of tchol: one persistent kernel that executes a tile DAG.
//
// Worker loop (one workgroup = one worker, section 2.1 of the paper: a worker
// repeatedly takes a task, runs it, then activates its successors):
//   claim   ticket t = atomicAdd(ticket); (task, part) = items[t]
//   wait    until dep[task] == 0 (agent-scope acquire; bounded by a watchdog)
//   run     the work item (a POTRF tile, a TRSM row strip, a GEMM/SYRK
//           sub-tile, a solve block)
//   publish every global store of the item is a device-scope (write-through)
//           store (st_dev; no result may be written with a plain global
//           store); each wavefront waits for them (vmcnt(0)), then a barrier,
//           then done[task] += 1; the last work item of a task decrements
//           dep[s] of every successor s ("activate").  Readers acquire at
//           agent scope after their wait, so they see the written-through
//           results; no release fence (an L2 write-back) is needed.
// Tickets are handed out in a topological order, so the worker holding the
// oldest unfinished ticket always has its predecessors finished or held by
// running workers: the loop cannot deadlock, whatever the grid size.
//
// All matrices are column-major FP64 with leading dimension `ld`; tile (i, j)
// of the matrix starts at A + (j*nb)*ld + i*nb.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kargs.h"
#include <type_traits>
#include "tchol_kinds.h"

#define NT 256                 // threads per workgroup: 4 wavefronts of 64
#define LDS_DOUBLES 20352      // 162816 bytes of LDS per workgroup (gfx950 allows 163840)

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
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

// Value of v in lane l (l wave-uniform), as a scalar broadcast.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// ---------------------------------------------------------------------------
// Direct global -> LDS loads.  One instruction moves 16 (or 4) bytes per lane
// into LDS at a wave-uniform base (M0) + lane * size, without passing through
// registers, so the K panels stream in while the matrix cores run.
//
// They are issued as inline assembly rather than through the compiler's
// builtin: for the builtin, the compiler cannot tell which LDS stage a load
// writes, so it waits for every outstanding load (vmcnt(0)) before the next
// LDS read, which serialises each chunk's load with the previous chunk's
// products.  Issued this way the compiler does not track them at all, and
// every consumer waits for them explicitly (vmcnt counts, then a workgroup
// barrier) before reading the stage they fill.  M0 is set in the same
// statement, right before the load; it is a reserved register the compiler
// sets itself before each of its own uses (these kernels have none).
typedef __attribute__((address_space(3))) void lds_void_t;

__device__ __forceinline__ uint32_t lds_addr(double* l) {
  return __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void_t*)l);
}
__device__ __forceinline__ void dma16(const void* g, double* l) {
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off" : : "s"(lds_addr(l)), "v"(g) : "memory");
}
__device__ __forceinline__ void dma4(const void* g, double* l) {
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dword %1, off" : : "s"(lds_addr(l)), "v"(g) : "memory");
}
// The same from a wave-uniform base (scalar registers) plus a per-lane byte
// offset below 4 GB: one 32-bit register per lane instead of a 64-bit address.
__device__ __forceinline__ const void* uniform_ptr(const void* p) {
  const uint64_t v = (uint64_t)(uintptr_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const void*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ void dma16s(const void* base, uint32_t off, double* l) {
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, %2" : : "s"(lds_addr(l)), "v"(off), "s"(uniform_ptr(base))
               : "memory");
}
__device__ __forceinline__ void dma4s(const void* base, uint32_t off, double* l) {
  asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dword %1, %2" : : "s"(lds_addr(l)), "v"(off), "s"(uniform_ptr(base))
               : "memory");
}

constexpr int imin_c(int a, int b) { return a < b ? a : b; }

// Makes every value of v available at this point (the compiler waits for
// their loads here).  A value loaded only to be used under a condition would
// otherwise have its load moved under that condition, one load and one wait
// per value; issued unconditionally before this point, the loads overlap.
template <int C>
__device__ __forceinline__ void materialize(double (&v)[C]) {
#pragma unroll
  for (int c = 0; c < C; ++c) asm volatile("" : : "v"(v[c]));
}
template <int R, int C>
__device__ __forceinline__ void materialize(double (&v)[R][C]) {
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < C; ++c) asm volatile("" : : "v"(v[r][c]));
}

// Store with device (agent) scope: it is written through to the device's
// point of coherence instead of staying dirty in this XCD's L2.  All results
// a work item publishes to other workgroups are written this way.
__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(float* p, float v) {
  __hip_atomic_store(reinterpret_cast<uint32_t*>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

typedef float f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_dev(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// BF16 (the upper half of an FP32 word) rounded to nearest even, and back.
__device__ __forceinline__ uint32_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ double bf16_val(uint32_t h) { return (double)__uint_as_float(h << 16); }
// x as hi + mid + lo, three BF16 terms of decreasing magnitude (each the
// rounded remainder of the previous ones; the remainders are exact in FP64),
// good to about 2^-24 relative, i.e. FP32 level.
__device__ __forceinline__ void split3(double x, uint32_t& h, uint32_t& m, uint32_t& l) {
  h = bf16_rne((float)x);
  const double r1 = x - bf16_val(h);
  m = bf16_rne((float)r1);
  l = bf16_rne((float)(r1 - bf16_val(m)));
}

// s_waitcnt vmcnt(N) with the other counters left alone (gfx9 encoding).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// ---------------------------------------------------------------------------
// Matrix-core tile product used by every update:
//     C[M x N] -= Ap[M x K] * Bp[N x K]^T,   M <= BM, N <= BN, K % KC == 0.
// The four wavefronts form a WGM x (4/WGM) grid; each owns a (BM/WGM) x
// (BN*WGM/4) piece of C as 16x16 MFMA blocks held in registers from the load
// of C to the final store.  K is streamed in chunks of KC
// columns through NST LDS stages filled by direct-to-LDS loads, NST-1 chunks
// ahead of the matrix cores.  SEG = 128 moves 16 bytes per lane (rows in
// pairs) and needs even ld, 16-byte aligned panels, and, when M or N is odd,
// one readable row after the panel; SEG = 32 moves 4 bytes per lane and has
// no such needs.  Row indices are clamped into the panel
// (rows past M hold copies and only feed outputs that are never stored).  With lower_only, entries of C above its diagonal are untouched.
// With Cl set, the result goes to LDS at Cl (column-major, leading dimension
// ldl; it must not overlap the NST stages) instead of back to C.
//
// The chunk loop is kept free of branches in its steady state (the transfer
// width is fixed per kernel instance, a transfer slot's panel is known at
// compile time, and the last NST-1 chunks are peeled off), so that the
// accumulators stay in the matrix-core registers across chunks.
template <int BM, int BN, int KC, int WGM, int NST, int PAD>
struct GemmShape {
  static constexpr int WGN = 4 / WGM;
  static constexpr int WTM = BM / WGM, WTN = BN / WGN;
  static constexpr int RB = WTM / 16, CB = WTN / 16;
  // LDS rows of the staged panels (one k index each) may be padded
  static constexpr int ALD = BM + PAD, BLD = BN + PAD;
  static constexpr int STAGE = KC * (ALD + BLD);  // doubles per stage
  static_assert(NST * STAGE <= LDS_DOUBLES, "stages must fit the workgroup LDS");
  static_assert(BM % 128 == 0 || 128 % BM == 0, "a 1 KB segment must cover whole rows or a row part");
  static_assert(BN % 128 == 0 || 128 % BN == 0, "a 1 KB segment must cover whole rows or a row part");
  static_assert(PAD == 0 || (BM % 128 == 0 && BN % 128 == 0), "padded rows need segments that stay within a row");
};

// K loop with SEG-double transfers per wavefront instruction (128: 16-byte
// lanes, 32: 4-byte lanes).
template <int BM, int BN, int KC, int WGM, int NST, int PAD, int SEG, int RB, int CB>
__device__ __forceinline__ void gemm_kloop(d4 (&acc)[RB][CB], const double* __restrict__ Ap,
                                           const double* __restrict__ Bp, int64_t ld, int M, int N, int K,
                                           double* lds, int64_t ldb_ = -1) {
  const int64_t ldB = ldb_ < 0 ? ld : ldb_;  // the B panel's leading dimension (default: A's)
  using S = GemmShape<BM, BN, KC, WGM, NST, PAD>;
  static_assert(RB == S::RB && CB == S::CB, "accumulator shape");
  constexpr int ALD = S::ALD, BLD = S::BLD, STAGE = S::STAGE;
  constexpr int QA = KC * BM / SEG, QB = KC * BN / SEG;  // transfers per stage
  static_assert(QA * SEG == KC * BM && QB * SEG == KC * BN, "stage must be whole segments");
  // When both counts divide by four, transfer slot j of every wavefront
  // serves the same panel and every wavefront issues the same number.
  constexpr bool UNIFORM = (QA % 4 == 0) && (QB % 4 == 0);
  constexpr int J = (QA + QB + 3) / 4;  // transfer slots per wavefront
  constexpr int W = (QA + QB) / 4;      // fewest transfers per wavefront and chunk
  static_assert(W >= 1, "every wavefront must issue transfers for every chunk");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / S::WGN, wn = wave % S::WGN;
  const int l16 = lane & 15, lg = lane >> 4;

  // One transfer: segment q of panel X (rows R = BM or BN, valid rows V) of
  // chunk ch.  A segment covers consecutive doubles of the column-major
  // panel: part of one k row, or whole k rows when the row is shorter than
  // the segment (then the rows are unpadded and contiguous).  Each 16-byte
  // lane moves rows (r, r + 1); each 4-byte lane half of one double.
  //
  // The address is split into a wave-uniform base and a per-lane offset.
  // Either a segment lies within one k row (R a multiple of SEG; it starts at
  // row u = e0 % R of k row e0 / R) or it covers whole k rows (R divides
  // SEG, u = 0; lane element le falls in k row e0 / R + le / R).  Rows are
  // clamped to the last valid start row Vc; the base takes min(u, Vc), so
  // the lane offsets are never negative.
  auto xfer = [&](const double* X, int64_t ld, int R, int XLD, int V, int q, int k0, double* dst)
                  __attribute__((always_inline)) {
    const int e0 = q * SEG;
    const int le = SEG == 128 ? 2 * lane : (lane >> 1);
    // a pair starts at an even row no later than V - 1; for odd V the pair
    // (V - 1, V) reads the row after the panel, which the launch contract
    // guarantees to exist (leading dimension above the order)
    const int Vc = SEG == 128 ? ((V - 1) & ~1) : V - 1;
    const int u = e0 % R, cu = e0 / R, ru = imin(u, Vc);
    const int cl = (R % SEG == 0) ? 0 : le / R;
    const int rl = ((R % SEG == 0) ? imin(u + le, Vc) : imin(le % R, Vc)) - ru;
    const double* base = X + (int64_t)(k0 + cu) * ld + ru;
    const uint32_t off = (uint32_t)(((int64_t)cl * ld + rl) * 8);
    if (SEG == 128)
      dma16s(base, off, dst + cu * XLD + u);
    else
      dma4s(base, off + 4 * (lane & 1), dst + cu * XLD + u);
  };
  auto slot = [&](int j, int k0, double* As, double* Bs) __attribute__((always_inline)) {
    const int q = wave + 4 * j;
    if (UNIFORM) {
      if (j < QA / 4) xfer(Ap, ld, BM, ALD, M, q, k0, As);
      else xfer(Bp, ldB, BN, BLD, N, q - QA, k0, Bs);
    } else {
      if (q < QA) xfer(Ap, ld, BM, ALD, M, q, k0, As);
      else if (q < QA + QB) xfer(Bp, ldB, BN, BLD, N, q - QA, k0, Bs);
    }
  };
  auto issue = [&](int ch) __attribute__((always_inline)) {
    double* As = lds + (ch % NST) * STAGE;
    double* Bs = As + KC * ALD;
    const int k0 = ch * KC;
    if constexpr (SEG == 128) {
#pragma unroll
      for (int j = 0; j < J; ++j) slot(j, k0, As, Bs);
    } else {  // many narrow transfers: a rolled loop keeps their addresses out of registers
#pragma unroll 2
      for (int j = 0; j < J; ++j) slot(j, k0, As, Bs);
    }
  };
  // compute(ch, nx): the products of chunk ch; with nx >= 0 the transfers of
  // chunk nx are issued along the way, a few per k-step, so that the matrix
  // cores are not idle while a whole chunk's transfers are issued
  auto compute = [&](int ch, int nx) __attribute__((always_inline)) {
    const double* as = lds + (ch % NST) * STAGE;
    const double* bs = as + KC * ALD;
    double* nAs = lds + ((nx < 0 ? 0 : nx) % NST) * STAGE;
    double* nBs = nAs + KC * ALD;
    constexpr int PER = (J + KC / 4 - 1) / (KC / 4);  // transfer slots per k-step
    // fragments of k-step ks + 1 are read while the MFMAs of ks run
    double fa[2][RB], fb[2][CB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) fa[0][rb] = as[lg * ALD + wm * S::WTM + rb * 16 + l16];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) fb[0][cb] = bs[lg * BLD + wn * S::WTN + cb * 16 + l16];
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int cur = ks & 1, nxt = cur ^ 1;
      if (nx >= 0) {
#pragma unroll
        for (int jj = 0; jj < PER; ++jj)
          if (ks * PER + jj < J) slot(ks * PER + jj, nx * KC, nAs, nBs);
      }
      if (ks + 1 < KC / 4) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) fa[nxt][rb] = as[((ks + 1) * 4 + lg) * ALD + wm * S::WTM + rb * 16 + l16];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) fb[nxt][cb] = bs[((ks + 1) * 4 + lg) * BLD + wn * S::WTN + cb * 16 + l16];
      }
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          acc[rb][cb] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(fb[cur][cb], fa[cur][rb], acc[rb][cb], 0, 0, 2 /* neg B */);
    }
  };

  // Chunk ch has landed once no more than the later chunks' transfers are
  // outstanding.  A wavefront issues W (or, when not UNIFORM, W + 1)
  // transfers per chunk; waiting for "at most W per later chunk" (capped at
  // the counter's range) is exact or stricter, never short.
  //
  // The first chunk waits for everything outstanding: the caller's loads of
  // C are then known complete, and the compiler (which tracks those loads but
  // not the direct-to-LDS ones) inserts no waits of its own into the loop.
  const int nch = K / KC;
  if (nch <= 0) return;
#pragma unroll
  for (int p = 0; p < NST - 1; ++p)
    if (p < nch) issue(p);
  wait_vmcnt<0>();
  __syncthreads();
  compute(0, NST - 1 < nch ? NST - 1 : -1);
  int ch = 1;
  for (; ch + NST - 1 < nch; ++ch) {  // steady state: NST - 2 later chunks in flight
    wait_vmcnt<imin_c((NST - 2) * W, 63)>();
    __syncthreads();
    compute(ch, ch + NST - 1);
  }
  for (; ch < nch; ++ch) {  // the last NST - 1 chunks: nothing more to issue
    const int later = nch - 1 - ch;
    if (later >= 2) wait_vmcnt<imin_c(2 * W, 63)>();
    else if (later == 1) wait_vmcnt<imin_c(W, 63)>();
    else wait_vmcnt<0>();
    __syncthreads();
    compute(ch, -1);
  }
}

// ldc: leading dimension of C when it differs from the panels' (< 0: ld);
// zero_c: start from C = 0 instead of loading C; ldb: the B panel's leading
// dimension when it differs from A's (< 0: ld); neg: store -C.  CF32: the
// initial C is read from the FP32 matrix Cf (leading dimension ldcf) instead.
template <int SEG, int BM, int BN, int KC, int WGM, int NST, int PAD = 8, bool CF32 = false>
__device__ __forceinline__ void gemm_core(double* __restrict__ C, const double* __restrict__ Ap,
                                          const double* __restrict__ Bp, int64_t ld, int M, int N, int K,
                                          bool lower_only, double* lds, double* Cl = nullptr, int ldl = 0,
                                          int64_t ldc = -1, bool zero_c = false, int64_t ldb = -1,
                                          bool neg = false, const float* __restrict__ Cf = nullptr,
                                          int64_t ldcf = 0) {
  const int64_t ldC = ldc < 0 ? ld : ldc;
  using S = GemmShape<BM, BN, KC, WGM, NST, PAD>;
  constexpr int RB = S::RB, CB = S::CB;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / S::WGN, wn = wave % S::WGN;
  const int l16 = lane & 15, lg = lane >> 4;

  d4 acc[RB][CB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * S::WTM + rb * 16 + l16, col = wn * S::WTN + cb * 16 + 4 * i + lg;
        if constexpr (CF32)
          acc[rb][cb][i] = (double)Cf[(int64_t)imin(col, N - 1) * ldcf + imin(row, M - 1)];
        else
          acc[rb][cb][i] = zero_c ? 0.0 : C[(int64_t)imin(col, N - 1) * ldC + imin(row, M - 1)];
      }

  gemm_kloop<BM, BN, KC, WGM, NST, PAD, SEG>(acc, Ap, Bp, ld, M, N, K, lds, ldb);
  __syncthreads();  // every wavefront is done with the stages before LDS is reused

#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * S::WTM + rb * 16 + l16, col = wn * S::WTN + cb * 16 + 4 * i + lg;
        if (row < M && col < N && (!lower_only || row >= col)) {
          const double v = neg ? -acc[rb][cb][i] : acc[rb][cb][i];
          if (Cl)
            Cl[col * ldl + row] = v;  // result kept in LDS (column-major, ld ldl)
          else
            st_dev(C + (int64_t)col * ldC + row, v);
        }
      }
}

// GEMM / SYRK work item: a 128 x 128 sub-tile of C, K = nb.  Chunks of 32
// columns through two stages need half the workgroup barriers of chunks of
// 16 through four; a K that is only a multiple of 16 takes the latter.
#define GB 128
template <int SEG>
__device__ __forceinline__ void gemm_nt(double* C, const double* Ap, const double* Bp, int64_t ld, int M, int N,
                                        int K, bool lower_only, double* lds) {
  if (K % 32 == 0)
    gemm_core<SEG, GB, GB, 32, 2, 2>(C, Ap, Bp, ld, M, N, K, lower_only, lds);
  else
    gemm_core<SEG, GB, GB, 16, 2, 4>(C, Ap, Bp, ld, M, N, K, lower_only, lds);
}

// The same product with C at its own leading dimension ldc (the panels at
// ld), optionally starting from C = 0.
__device__ __forceinline__ void gemm_nt_ex(double* C, int64_t ldc, const double* Ap, const double* Bp, int64_t ld,
                                           int M, int N, int K, bool lower_only, bool zero_c, double* lds) {
  if (K % 32 == 0)
    gemm_core<128, GB, GB, 32, 2, 2>(C, Ap, Bp, ld, M, N, K, lower_only, lds, nullptr, 0, ldc, zero_c);
  else
    gemm_core<128, GB, GB, 16, 2, 4>(C, Ap, Bp, ld, M, N, K, lower_only, lds, nullptr, 0, ldc, zero_c);
}

// ---------------------------------------------------------------------------
// FP32 tile product for the mixed-precision factorization:
//     C[M x N] -= Ap[M x K] * Bp[N x K]^T in FP32 storage, FP32 MFMA
// (v_mfma_f32_16x16x4f32, the FP64 instruction's shape and operand layout)
// with FP32 accumulation; 128 x 128 outputs, K % KC == 0.  A stage holds KC
// k-rows laid out as [A row (128) | B row (128) | 16 pad] floats, so one
// 16-byte-per-lane transfer moves one k-row of both panels (lanes 0..31: A,
// lanes 32..63: B) and the padded rows keep the fragment reads free of bank
// conflicts.  Rows are moved four at a time: the row group of the last valid
// row may read up to three rows past the panel, which the mixed working copy
// provides (its leading dimension exceeds the order by at least three).
// The f32 MFMA has no operand negation, so the A fragment is negated.  Its
// 16 x 16 result differs in layout from the f64 instruction's: element i of
// lane l holds row 4 (l / 16) + i (not 4 i + l / 16) of column l % 16.
// CD: the product is added to an FP64 C (Cd, ld ldcd) instead: the diagonal
// tiles of the mixed-precision factorization stay in FP64 throughout.
#define F32_LD 272
template <int KC, int NST, bool CD = false>
__device__ __forceinline__ void gemm_f32_core(float* __restrict__ C, const float* __restrict__ Ap,
                                              const float* __restrict__ Bp, int64_t ld, int M, int N, int K,
                                              bool lower_only, double* lds_d, double* __restrict__ Cd = nullptr,
                                              int64_t ldcd = 0) {
  constexpr int STAGE = KC * F32_LD;  // floats per stage
  constexpr int W = KC / 4;           // transfers per wavefront and chunk
  static_assert(NST * STAGE <= 2 * LDS_DOUBLES, "stages must fit the workgroup LDS");
  static_assert(KC % 4 == 0 && W >= 1, "every wavefront transfers whole k-rows");
  float* lds = reinterpret_cast<float*>(lds_d);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;  // 2 x 2 wavefronts, 64 x 64 each
  const int l16 = lane & 15, lg = lane >> 4;
  const bool arow = lane < 32;
  const float* src0 = arow ? Ap + imin(4 * lane, (M - 1) & ~3) : Bp + imin(4 * (lane - 32), (N - 1) & ~3);

  f4 acc[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * 64 + rb * 16 + l16, col = wn * 64 + cb * 16 + 4 * lg + i;
        acc[rb][cb][i] = CD ? 0.f : C[(int64_t)imin(col, N - 1) * ld + imin(row, M - 1)];
      }

  static_assert(STAGE % 2 == 0 && F32_LD % 2 == 0, "destinations are addressed in doubles");
  auto issue = [&](int ch) __attribute__((always_inline)) {
    // destinations as double pointers into the shared array (stage and row offsets are even)
    double* st = lds_d + (ch % NST) * (STAGE / 2);
    const int k0 = ch * KC;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int q = wave + 4 * j;  // k-row of the chunk
      dma16(src0 + (int64_t)(k0 + q) * ld, st + q * (F32_LD / 2));
    }
  };
  // as in gemm_kloop: the transfers of chunk nx (if any) are issued along the
  // products of chunk ch, one k-row per k-step
  auto compute = [&](int ch, int nx) __attribute__((always_inline)) {
    const float* st = lds + (ch % NST) * STAGE;
    double* nst = lds_d + ((nx < 0 ? 0 : nx) % NST) * (STAGE / 2);
    constexpr int PER = (W + KC / 4 - 1) / (KC / 4);
    float fa[2][4], fb[2][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) fa[0][rb] = -st[lg * F32_LD + wm * 64 + rb * 16 + l16];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) fb[0][cb] = st[lg * F32_LD + 128 + wn * 64 + cb * 16 + l16];
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int cur = ks & 1, nxt = cur ^ 1;
      if (nx >= 0) {
#pragma unroll
        for (int jj = 0; jj < PER; ++jj)
          if (ks * PER + jj < W) {
            const int q = wave + 4 * (ks * PER + jj);
            dma16(src0 + (int64_t)(nx * KC + q) * ld, nst + q * (F32_LD / 2));
          }
      }
      if (ks + 1 < KC / 4) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) fa[nxt][rb] = -st[((ks + 1) * 4 + lg) * F32_LD + wm * 64 + rb * 16 + l16];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          fb[nxt][cb] = st[((ks + 1) * 4 + lg) * F32_LD + 128 + wn * 64 + cb * 16 + l16];
      }
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(fb[cur][cb], fa[cur][rb], acc[rb][cb], 0, 0, 0);
    }
  };
  // as in gemm_kloop: the first chunk waits for everything, the loads of C included
  const int nch = K / KC;
#pragma unroll
  for (int p = 0; p < NST - 1; ++p)
    if (p < nch) issue(p);
  if (nch > 0) {  // (every loop below is reached only through the first chunk's full wait)
    wait_vmcnt<0>();
    __syncthreads();
    compute(0, NST - 1 < nch ? NST - 1 : -1);
    int ch = 1;
    for (; ch + NST - 1 < nch; ++ch) {
      wait_vmcnt<imin_c((NST - 2) * W, 63)>();
      __syncthreads();
      compute(ch, ch + NST - 1);
    }
    for (; ch < nch; ++ch) {
      const int later = nch - 1 - ch;
      if (later >= 2) wait_vmcnt<imin_c(2 * W, 63)>();
      else if (later == 1) wait_vmcnt<imin_c(W, 63)>();
      else wait_vmcnt<0>();
      __syncthreads();
      compute(ch, -1);
    }
  }
  __syncthreads();
  if constexpr (CD) {
    // read-modify-write of the FP64 tile, two row blocks at a time: the 32
    // old values are requested together (clamped into the tile, which is
    // nb x nb in full) and all taken before the first store, one memory
    // round trip per pair instead of one per value
#pragma unroll
    for (int rp = 0; rp < 4; rp += 2) {
      double old[2][16];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = wm * 64 + (rp + h) * 16 + l16, col = wn * 64 + cb * 16 + 4 * lg + i;
            old[h][4 * cb + i] = Cd[(int64_t)imin(col, N - 1) * ldcd + imin(row, M - 1)];
          }
      materialize(old);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = wm * 64 + (rp + h) * 16 + l16, col = wn * 64 + cb * 16 + 4 * lg + i;
            if (row < M && col < N && (!lower_only || row >= col))
              st_dev(Cd + (int64_t)col * ldcd + row, old[h][4 * cb + i] + (double)acc[rp + h][cb][i]);
          }
    }
  } else {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = wm * 64 + rb * 16 + l16, col = wn * 64 + cb * 16 + 4 * lg + i;
          if (row < M && col < N && (!lower_only || row >= col)) st_dev(C + (int64_t)col * ld + row, acc[rb][cb][i]);
        }
  }
}

__device__ __forceinline__ void gemm_nt_f32(float* C, const float* Ap, const float* Bp, int64_t ld, int M, int N,
                                            int K, bool lower_only, double* lds) {
  if (K % 32 == 0)
    gemm_f32_core<32, 4>(C, Ap, Bp, ld, M, N, K, lower_only, lds);
  else
    gemm_f32_core<16, 4>(C, Ap, Bp, ld, M, N, K, lower_only, lds);
}

// FP32 GEMM item with a 256 x 128 output, C[M x N] -= Ap[M x K] Bp[N x K]^T,
// M <= 256, N <= 128 (the mixed-precision factorization's GEMM items): the
// scheme of gemm_f32_core with twice the rows per wavefront (2 x 2
// wavefronts of 128 x 64).  Per k-row of a chunk one 16-byte transfer of all
// 64 lanes moves the 256 A rows and one of lanes 0-31 the 128 B rows into an
// LDS row [A 256 | B 128 | 16 pad]; three stages of 32 k-rows.
#define F32W_LD 400
template <int KC, int NST>
__device__ __forceinline__ void gemm_f32_wide(float* __restrict__ C, const float* __restrict__ Ap,
                                              const float* __restrict__ Bp, int64_t ld, int M, int N, int K,
                                              double* lds_d) {
  constexpr int STAGE = KC * F32W_LD;  // floats per stage
  constexpr int W = 2 * (KC / 4);      // transfers per wavefront and chunk: two per k-row, KC / 4 k-rows
  static_assert(NST * STAGE <= 2 * LDS_DOUBLES, "stages must fit the workgroup LDS");
  static_assert(KC % 4 == 0 && W <= 63, "every wavefront transfers whole k-rows");
  float* lds = reinterpret_cast<float*>(lds_d);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;  // 2 x 2 wavefronts, 128 x 64 each
  const int l16 = lane & 15, lg = lane >> 4;
  const float* srcA = Ap + imin(4 * lane, (M - 1) & ~3);
  const float* srcB = Bp + imin(4 * (lane & 31), (N - 1) & ~3);

  f4 acc[8][4];
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * 128 + rb * 16 + l16, col = wn * 64 + cb * 16 + 4 * lg + i;
        acc[rb][cb][i] = C[(int64_t)imin(col, N - 1) * ld + imin(row, M - 1)];
      }

  static_assert(STAGE % 2 == 0 && F32W_LD % 2 == 0, "destinations are addressed in doubles");
  // the two transfers of k-row q of chunk ch (doubles: a row is F32W_LD / 2, B starts at 128)
  auto xfer = [&](int ch, int q) __attribute__((always_inline)) {
    double* st = lds_d + (ch % NST) * (STAGE / 2) + q * (F32W_LD / 2);
    const int64_t k = (int64_t)(ch * KC + q) * ld;
    dma16(srcA + k, st);
    if (lane < 32) dma16(srcB + k, st + 128);
  };
  auto issue = [&](int ch) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < KC / 4; ++j) xfer(ch, wave + 4 * j);
  };
  // the products of chunk ch; the transfers of chunk nx (if any) go out along
  // them, one k-row per k-step
  auto compute = [&](int ch, int nx) __attribute__((always_inline)) {
    const float* st = lds + (ch % NST) * STAGE;
    float fa[2][8], fb[2][4];
#pragma unroll
    for (int rb = 0; rb < 8; ++rb) fa[0][rb] = -st[lg * F32W_LD + wm * 128 + rb * 16 + l16];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) fb[0][cb] = st[lg * F32W_LD + 256 + wn * 64 + cb * 16 + l16];
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int cur = ks & 1, nxt = cur ^ 1;
      if (nx >= 0) xfer(nx, wave + 4 * ks);
      if (ks + 1 < KC / 4) {
#pragma unroll
        for (int rb = 0; rb < 8; ++rb)
          fa[nxt][rb] = -st[((ks + 1) * 4 + lg) * F32W_LD + wm * 128 + rb * 16 + l16];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) fb[nxt][cb] = st[((ks + 1) * 4 + lg) * F32W_LD + 256 + wn * 64 + cb * 16 + l16];
      }
#pragma unroll
      for (int rb = 0; rb < 8; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(fb[cur][cb], fa[cur][rb], acc[rb][cb], 0, 0, 0);
    }
  };
  // as in gemm_kloop: the first chunk waits for everything, the loads of C included
  const int nch = K / KC;
#pragma unroll
  for (int p = 0; p < NST - 1; ++p)
    if (p < nch) issue(p);
  if (nch > 0) {  // (every loop below is reached only through the first chunk's full wait)
    wait_vmcnt<0>();
    __syncthreads();
    compute(0, NST - 1 < nch ? NST - 1 : -1);
    int ch = 1;
    for (; ch + NST - 1 < nch; ++ch) {
      wait_vmcnt<imin_c((NST - 2) * W, 63)>();
      __syncthreads();
      compute(ch, ch + NST - 1);
    }
    for (; ch < nch; ++ch) {
      const int later = nch - 1 - ch;
      if (later >= 2) wait_vmcnt<imin_c(2 * W, 63)>();
      else if (later == 1) wait_vmcnt<imin_c(W, 63)>();
      else wait_vmcnt<0>();
      __syncthreads();
      compute(ch, -1);
    }
  }
  __syncthreads();
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * 128 + rb * 16 + l16, col = wn * 64 + cb * 16 + 4 * lg + i;
        if (row < M && col < N) st_dev(C + (int64_t)col * ld + row, acc[rb][cb][i]);
      }
}

// The same with the result added to an FP64 C (Cd, ld ldcd).
__device__ __forceinline__ void gemm_nt_f32_d(double* Cd, int64_t ldcd, const float* Ap, const float* Bp, int64_t ld,
                                              int M, int N, int K, bool lower_only, double* lds) {
  if (K % 32 == 0)
    gemm_f32_core<32, 4, true>(nullptr, Ap, Bp, ld, M, N, K, lower_only, lds, Cd, ldcd);
  else
    gemm_f32_core<16, 4, true>(nullptr, Ap, Bp, ld, M, N, K, lower_only, lds, Cd, ldcd);
}

// ---------------------------------------------------------------------------
// BF16 GEMM item of the BF16-update factorization: C[M x N] (FP32, ld ldc)
// -= A B^T with A (M x K) and B (N x K) each given as three BF16 terms
// (hi + mid + lo, split3) in K-contiguous rows (row stride hld, terms hterm
// apart; K beyond one column block of kb columns continues in the next
// block, hblk further); M <= 256, N <= 128, K % 32 == 0, kb % 32 == 0.  The six products of terms whose
// orders add up to at most two (hh, hm, mh, mm, hl, lh) run on the BF16
// matrix cores (v_mfma_f32_16x16x32_bf16) with FP32 accumulation; the
// terms left out are below 2^-24 of the product, so the update keeps FP32
// accuracy.  2 x 2 wavefronts of 128 x 64.  A chunk of 32 k holds, per
// term, 64-byte rows of A (256) and B (128) in LDS, filled by direct
// 16-byte transfers (16 rows per wavefront instruction); the four 16-byte
// quarters of a row are XOR-swizzled by bits 2-3 of the row, so the
// fragment reads of 16 consecutive rows hit distinct banks.  Two stages;
// the next chunk's 72 transfers go out at the start of the current chunk's
// products.  The instruction has no operand negation: the accumulators
// start from -C and -acc is stored.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
#define BW_SLOTS_A 1024                               // 16-byte slots per term of A: 256 rows x 4
#define BW_SLOTS_B 512                                // of B: 128 rows x 4
#define BW_STAGE_BYTES (3 * (BW_SLOTS_A + BW_SLOTS_B) * 16)

__device__ __forceinline__ int bw_slot(int row, int q) { return row * 4 + (q ^ ((row >> 2) & 3)); }

__device__ __forceinline__ void gemm_bf16x6_wide(float* __restrict__ C, int64_t ldc, const uint16_t* __restrict__ Ha,
                                                 const uint16_t* __restrict__ Hb, int64_t hld, int64_t hterm,
                                                 int64_t hblk, int kb, int M, int N, int K, double* lds_d) {
  constexpr int KC = 32;
  static_assert(2 * BW_STAGE_BYTES <= 8 * LDS_DOUBLES, "two stages must fit the workgroup LDS");
  char* lds = reinterpret_cast<char*>(lds_d);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, lg = lane >> 4;

  f4 acc[8][4];
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * 128 + rb * 16 + l16, col = wn * 64 + cb * 16 + 4 * lg + i;
        acc[rb][cb][i] = -C[(int64_t)imin(col, N - 1) * ldc + imin(row, M - 1)];
      }
  // transfer j (0..71) of chunk ch: A term j / 16, rows 16 (j % 16) ..; then B term (j - 48) / 8
  auto xfer = [&](int ch, int j) __attribute__((always_inline)) {
    char* st = lds + (ch & 1) * BW_STAGE_BYTES;
    const bool isa = j < 48;
    const int term = isa ? j >> 4 : (j - 48) >> 3, grp = isa ? j & 15 : (j - 48) & 7;
    const int row = grp * 16 + (lane >> 2);
    const int q = (lane & 3) ^ ((row >> 2) & 3);
    const int kk = ch * KC;  // k of the chunk: column kk % kb of column block kk / kb
    const uint16_t* g = (isa ? Ha : Hb) + term * hterm + (int64_t)(kk / kb) * hblk +
                        (int64_t)imin(row, (isa ? M : N) - 1) * hld + kk % kb + 8 * q;
    char* dst = st + (isa ? term * BW_SLOTS_A : 3 * BW_SLOTS_A + term * BW_SLOTS_B) * 16 + grp * 64 * 16;
    dma16(g, reinterpret_cast<double*>(dst));
  };
  auto issue = [&](int ch) __attribute__((always_inline)) {
#pragma unroll
    for (int jj = 0; jj < 18; ++jj) xfer(ch, wave + 4 * jj);
  };
  auto compute = [&](int ch, int nx) __attribute__((always_inline)) {
    const char* st = lds + (ch & 1) * BW_STAGE_BYTES;
    if (nx >= 0) issue(nx);
    bf16x8 fb[3][4];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        fb[t][cb] = *reinterpret_cast<const bf16x8*>(
            st + (3 * BW_SLOTS_A + t * BW_SLOTS_B + bw_slot(wn * 64 + cb * 16 + l16, lg)) * 16);
    // the A fragments of row block rb + 1 are read while the products of rb run
    bf16x8 fan[2][3];
#pragma unroll
    for (int t = 0; t < 3; ++t)
      fan[0][t] = *reinterpret_cast<const bf16x8*>(st + (t * BW_SLOTS_A + bw_slot(wm * 128 + l16, lg)) * 16);
#pragma unroll
    for (int rb = 0; rb < 8; ++rb) {
      if (rb + 1 < 8) {
#pragma unroll
        for (int t = 0; t < 3; ++t)
          fan[(rb + 1) & 1][t] = *reinterpret_cast<const bf16x8*>(
              st + (t * BW_SLOTS_A + bw_slot(wm * 128 + (rb + 1) * 16 + l16, lg)) * 16);
      }
      const bf16x8* fa = fan[rb & 1];
      // term pairs (B term, A term) from the smallest: h l, l h, m m, h m, m h, h h;
      // consecutive instructions go to the four independent accumulators
      // of the row block, so none waits for the previous one's result
      constexpr int PB[6] = {2, 0, 1, 1, 0, 0}, PA[6] = {0, 2, 1, 0, 1, 0};
#pragma unroll
      for (int pr = 0; pr < 6; ++pr)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[PB[pr]][cb], fa[PA[pr]], acc[rb][cb], 0, 0, 0);
    }
  };
  const int nch = K / KC;
  if (nch > 0) {
    issue(0);
    wait_vmcnt<0>();  // the loads of C and chunk 0
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
      compute(ch, ch + 1 < nch ? ch + 1 : -1);
      if (ch + 1 < nch) {
        wait_vmcnt<0>();
        __syncthreads();
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int rb = 0; rb < 8; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * 128 + rb * 16 + l16, col = wn * 64 + cb * 16 + 4 * lg + i;
        if (row < M && col < N) st_dev(C + (int64_t)col * ldc + row, -acc[rb][cb][i]);
      }
}

// ---------------------------------------------------------------------------
// Panel constants of the diagonal tile's adjoint (panels of PW columns).
#define PW 16
#define PPLD 516                              // LDS leading dimension of the panel
#define P_STAGE_DOUBLES (272 * 8 * 4)         // stages of gemm_core<SEG, 256, 16, 8, 4, 4, 0>

// ---------------------------------------------------------------------------
// POTRF of a tile of order m <= 128 held in LDS for the whole factorization:
// loaded once, factored right-looking by 16-column panels, stored once.  Per
// panel: the 16 x 16 diagonal block is factored on wavefront 0 in registers
// (diag16_x), every thread solves one row below it, and the trailing
// lower blocks take the panel's update on the matrix cores (16 x 16 blocks,
// K = 16); wavefront 0 updates and factors the next diagonal block first,
// while the other wavefronts update the rest.  Returns 0, or the 1-based
// column (within the tile) whose pivot is not positive.
#define SLD 132   // LDS leading dimension of the resident tile

// Factors the 16 x 16 (w x w, rows and columns past w padded with the
// identity) diagonal block at (off, off) of an LDS matrix X (leading
// dimension LDX) on one wavefront: lane r holds row r in registers, the
// pivot and the column entries are broadcast across lanes (readlane), so no
// barrier is needed.  With extra > 0, lanes 16 .. 16 + extra - 1 hold the
// rows off + 16 .. below the block, which the same steps solve against it
// (X := X L_dd^{-T}) at no extra cost.  l = sqrt(d) and 1/l come from the
// hardware reciprocal square root and two Newton steps (y to about an ulp;
// then l = d y with one residual correction), a far shorter dependent chain
// than a correctly rounded square root and division, and exact for powers
// of four; pivots below 2^-900 are scaled by 2^1000 first (exactly), and
// the results back.  No step branches, so the updates of one column overlap
// the next pivot's chain.  Writes L_dd back (and the solved rows below), a
// copy to Ldd[r * LDD + c] (r < 16 + extra) and the reciprocal pivots to
// Linv.  Returns 0, or ibase + the 1-based column of the first pivot that
// is not positive (zero, negative or NaN; the arithmetic goes on and its
// results are discarded).
template <int LDX, int LDD>
__device__ __forceinline__ int diag16_x(double* X, int off, int w, double* Ldd, double* Linv, int lane, int ibase,
                                        int extra = 0) {
  double* As = X;
  const int c0 = off;
  const bool below = lane >= PW && lane < PW + extra;  // a row below the block
  double x[PW];
  const int r = below ? lane : imin(lane, w - 1);
  // every load is issued before any is used (and kept out of the selects below)
  double v[PW];
#pragma unroll
  for (int c = 0; c < PW; ++c) v[c] = As[(c0 + imin(c, w - 1)) * LDX + c0 + r];
  materialize(v);
#pragma unroll
  for (int c = 0; c < PW; ++c)
    x[c] = below ? ((c < w) ? v[c] : 0.0)
                 : ((lane < w) ? (((c <= lane) & (c < w)) ? v[c] : 0.0) : (c == lane ? 1.0 : 0.0));
  int info = 0;
  double pinv[PW];
#pragma unroll
  for (int cc = 0; cc < PW; ++cc) {
    const double d = readlane_f64(x[cc], cc);
    info = (info == 0 && !(d > 0.0)) ? ibase + cc + 1 : info;
    const bool tiny = d < 0x1p-900;
    const double ds = tiny ? d * 0x1p+1000 : d;
    double y = __builtin_amdgcn_rsq(ds);
    y = fma(0.5 * y, fma(-ds, y * y, 1.0), y);
    y = fma(0.5 * y, fma(-ds, y * y, 1.0), y);
    double l = ds * y;
    l = fma(fma(-l, l, ds), 0.5 * y, l);
    l = tiny ? l * 0x1p-500 : l;
    const double inv = tiny ? y * 0x1p+500 : y;
    pinv[cc] = inv;
    // the scaled column is broadcast before the pivot itself is set, which
    // keeps l off the chain to the next pivot; entries above the diagonal
    // (lane < column) are updated too, without a select: they are never
    // read, and the identity padding stays exact
    const double sc = x[cc] * inv;
#pragma unroll
    for (int c2 = cc + 1; c2 < PW; ++c2) {
      const double vv = readlane_f64(sc, c2);
      x[c2] -= sc * vv;
    }
    x[cc] = (lane == cc) ? l : sc;
  }
  if (lane < w) {
#pragma unroll
    for (int c = 0; c < PW; ++c)
      if (c <= lane) As[(c0 + c) * LDX + c0 + lane] = x[c];
  }
  if (below) {
#pragma unroll
    for (int c = 0; c < PW; ++c) {
      As[(c0 + c) * LDX + c0 + lane] = x[c];
      Ldd[lane * LDD + c] = x[c];
    }
  }
  if (lane < PW) {
#pragma unroll
    for (int c = 0; c < PW; ++c) Ldd[lane * LDD + c] = (c <= lane) ? x[c] : 0.0;
    double li = pinv[0];
#pragma unroll
    for (int c = 1; c < PW; ++c) li = (lane == c) ? pinv[c] : li;
    Linv[lane] = li;
  }
  return info;
}

__device__ __forceinline__ int diag16_lds(double* As, int c0, int w, double* Ldd, double* Linv, int lane) {
  return diag16_x<SLD, PW + 1>(As, c0, w, Ldd, Linv, lane, c0);
}

// Block (bi, bj) of the resident tile -= P(bi) P(bj)^T, P the 16 columns of
// the panel at c0.  A operand: P(bi) (rows on lanes % 16), B operand: P(bj)^T;
// element v of lane l is then row 4v + l/16, column l%16 of the block.
__device__ __forceinline__ void upd16_lds(double* As, int c0, int bi, int bj, int lane) {
  const int l16 = lane & 15, lg = lane >> 4;
  d4 acc;
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = As[(bj * 16 + l16) * SLD + bi * 16 + 4 * v + lg];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double fa = As[(c0 + 4 * s + lg) * SLD + bi * 16 + l16];
    const double fb = As[(c0 + 4 * s + lg) * SLD + bj * 16 + l16];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, fb, acc, 0, 0, 2 /* neg B */);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) As[(bj * 16 + l16) * SLD + bi * 16 + 4 * v + lg] = acc[v];
}

__device__ __forceinline__ int potrf_small(double* __restrict__ Akk, int64_t ld, int m, double* lds) {
  double* As = lds;                      // [128][SLD]
  double* Ldd = As + 128 * SLD;          // [PW][PW + 1]
  double* Linv = Ldd + PW * (PW + 1);    // [PW]
  __shared__ int s_sinfo;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nblk = (m + 15) >> 4;
  // the lower triangle into LDS, 16 loads in flight per thread; rows and
  // columns past m hold the identity
  {
    constexpr int PER = 128 * 128 / NT, BATCH = 16;
#pragma unroll 1
    for (int u0 = 0; u0 < PER; u0 += BATCH) {
      double v[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int idx = tid + (u0 + u) * NT, c = idx >> 7, r = idx & 127;
        v[u] = Akk[(int64_t)imin(c, m - 1) * ld + imin(imax(r, c), m - 1)];
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int idx = tid + (u0 + u) * NT, c = idx >> 7, r = idx & 127;
        if (c < nblk * 16 && r < nblk * 16) As[c * SLD + r] = (r < m && c < m && r >= c) ? v[u] : (r == c ? 1.0 : 0.0);
      }
    }
  }
  __syncthreads();
  if (wave == 0) {
    const int info = diag16_lds(As, 0, imin(16, m), Ldd, Linv, lane);
    if (lane == 0) s_sinfo = info;
  }
  __syncthreads();
  for (int j = 0; j < nblk; ++j) {
    const int c0 = j * 16;
    const int info = __builtin_amdgcn_readfirstlane(s_sinfo);
    if (info != 0) return info;
    // rows below the diagonal block: y := y L_dd^{-T}, one row per thread
#pragma unroll 1
    for (int r = c0 + 16 + tid; r < nblk * 16; r += NT) {
      double y[PW];
#pragma unroll
      for (int c = 0; c < PW; ++c) y[c] = As[(c0 + c) * SLD + r];
#pragma unroll
      for (int c = 0; c < PW; ++c) {
        y[c] *= Linv[c];
#pragma unroll
        for (int c2 = c + 1; c2 < PW; ++c2) y[c2] -= y[c] * Ldd[c2 * (PW + 1) + c];
      }
#pragma unroll
      for (int c = 0; c < PW; ++c) As[(c0 + c) * SLD + r] = y[c];
    }
    __syncthreads();
    if (j + 1 >= nblk) break;
    // the panel's update of the trailing lower blocks; wavefront 0 first
    // updates and factors the next diagonal block (the critical path)
    const int nb2 = nblk - j - 1;
    const int npair = nb2 * (nb2 + 1) / 2;
    if (wave == 0) {
      upd16_lds(As, c0, j + 1, j + 1, lane);
      const int info2 = diag16_lds(As, c0 + 16, imin(16, m - c0 - 16), Ldd, Linv, lane);
      if (lane == 0) s_sinfo = info2;
    }
    // block pairs p >= 1 in column-major order of (bi >= bj), after (j+1, j+1),
    // on the other three wavefronts (wavefront 0 is busy with the diagonal)
#pragma unroll 1
    for (int p = (wave == 0 ? npair : wave); p < npair; p += 3) {
      int cj = 0, rem = p;
      while (rem >= nb2 - cj) {
        rem -= nb2 - cj;
        ++cj;
      }
      const int bj = j + 1 + cj;
      upd16_lds(As, c0, bj + rem, bj, lane);
    }
    __syncthreads();
  }
  // the factor to the tile, lower triangle only
  for (int idx = tid; idx < m * 128; idx += NT) {
    const int c = idx >> 7, r = idx & 127;
    if (r < m && r >= c) st_dev(Akk + (int64_t)c * ld + r, As[c * SLD + r]);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// POTRF work item for a tile of order m <= 512 on one workgroup:
// Akk := chol(Akk), lower, in place.  Left-looking by panels of PT_W = 32
// columns, each taken in slabs of up to PT_SLAB = 256 rows that stay in LDS
// from their update to their store:
//  1. the matrix cores apply every earlier column to the slab (256 x 32
//     outputs per K step, the result written to LDS);
//  2. in the first slab, wavefront 0 factors the 32 x 32 diagonal block: its
//     leading 16 x 16 block in registers (diag16_x, which also solves the 16
//     rows below it), their product subtracted from the trailing 16 x 16
//     block on the matrix cores, then that block factored;
//  3. every thread solves one row of the slab below the block against L_dd;
//  4. the slab goes to the tile (write-through stores), where the next
//     panel's update reads it.
// Panels of 32 columns halve the number of panels and the re-reads of the
// factored columns relative to the 16 of the diagonal blocks, and give the
// updates enough outputs per K step to keep the matrix cores busy.
// SLAB = 128: slabs of 128 rows in a compact layout of 81024 bytes (two
// workgroups per compute unit): L_dd and the reciprocal pivots live in the
// update's staging area (free once the product is in the slab), the columns
// of L_dd below the diagonal packed.  With Bf (compact layout only) the
// forward solve L y = b of nrhs <= 4 right-hand sides (column-major at Bf,
// leading dimension ldbf) rides along, right-looking by panels: in the first
// slab of a panel, thread 128 + j solves the panel's rows of column j
// against L_dd (the same substitution as the rows below the block, on the
// values the earlier panels left) and stores them, final, to Bf and to Yp;
// when a slab is stored, each of its rows below the block takes
// b -= L(row, panel) y_panel.  Bf then holds y.
// Returns 0, or the 1-based column (within the tile) whose pivot is not
// positive (zero, negative or NaN).
#define PT_W 32
#define PT_SLAB 256
#define PT_LT 36                               // stride of the columns of L_dd
#define PT_LT_PACKED (PT_W * (PT_W + 1) / 2)   // the packed columns (c2 >= c)
#define PT_FWD 4                               // right-hand sides of the fused forward solve
#define PT_LDS_COMPACT (2 * 16 * (128 + PT_W) + PT_W * 136 + PT_LT_PACKED + PT_W * PT_FWD)
#define FRB_COMPACT_DOUBLES (32 * 4 * 64 + 2 * 4 * 64)  // tile_solve<true>

// IN32 (compact layout): the tile's values are read from the FP32 matrix A32
// (leading dimension ld32) instead of Akk, and L is written to both (Akk in
// FP64 for the later panels' products, A32 rounded to FP32).
template <int SEG, int SLAB = PT_SLAB, bool IN32 = false>
__device__ __forceinline__ int potrf_tile(double* __restrict__ Akk, int64_t ld, int m, double* lds,
                                          double* Bf = nullptr, int64_t ldbf = 0, int nrhs = 0,
                                          float* __restrict__ A32 = nullptr, int64_t ld32 = 0) {
  static_assert(!IN32 || SLAB == 128, "FP32 input in the compact layout only");
  static_assert(SLAB == 256 || SLAB == 128, "slab height");
  constexpr bool PACKED = SLAB < PT_SLAB;
  constexpr int LDP = SLAB + 8;                        // LDS leading dimension of a slab
  constexpr int STAGE = 2 * 16 * (SLAB + PT_W);        // stages of gemm_core<SEG, SLAB, 32, 16, 4, 2, 0>
  static_assert(PACKED ? (STAGE + PT_W * LDP + PT_LT_PACKED + PT_W * PT_FWD == PT_LDS_COMPACT &&
                          PT_W * (PT_W + 1) + PT_W <= STAGE)
                       : STAGE + PT_W * LDP + PT_W * (PT_W + 1) + PT_W + PT_W * PT_LT <= LDS_DOUBLES,
                "LDS budget");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* Ps = lds + STAGE;                                 // [PT_W][LDP] the slab
  double* Ldd = PACKED ? lds : Ps + PT_W * LDP;             // [PT_W][PT_W + 1] the diagonal block (lower)
  double* Linv = Ldd + PT_W * (PT_W + 1);                   // [PT_W] reciprocal pivots
  double* LT = PACKED ? Ps + PT_W * LDP : Linv + PT_W;      // L_dd by columns
  double* Yp = LT + PT_LT_PACKED;                           // [PT_W][PT_FWD] the panel's rows of y (Bf)
  const bool fwd = PACKED && Bf != nullptr;
  // column c of L_dd from its diagonal down (c2 >= c): LT[lt(c) + c2]
  auto lt = [](int c) __attribute__((always_inline)) { return PACKED ? c * PT_W - c * (c + 1) / 2 : c * PT_LT; };
  __shared__ int s_info;
  for (int c0 = 0; c0 < m; c0 += PT_W) {
    const int w = imin(PT_W, m - c0);
    const int R = m - c0;
    double* P = Akk + (int64_t)c0 * ld + c0;
    float* const P32 = IN32 ? A32 + (int64_t)c0 * ld32 + c0 : nullptr;
    for (int s0 = 0; s0 < R; s0 += SLAB) {
      const int S = imin(SLAB, R - s0);
      if (c0 > 0) {
        // the slab - L[c0 + s0 :, 0 : c0] L[c0 : c0 + w, 0 : c0]^T into LDS,
        // on a product no taller than the slab needs
        if (SLAB > 128 && S > 128)
          gemm_core<SEG, SLAB, PT_W, 16, 4, 2, 0, IN32>(P + s0, Akk + c0 + s0, Akk + c0, ld, S, w, c0, false, lds, Ps,
                                                        LDP, -1, false, -1, false, IN32 ? P32 + s0 : nullptr, ld32);
        else if (S > 64)
          gemm_core<SEG, 128, PT_W, 16, 4, 2, 0, IN32>(P + s0, Akk + c0 + s0, Akk + c0, ld, S, w, c0, false, lds, Ps,
                                                       LDP, -1, false, -1, false, IN32 ? P32 + s0 : nullptr, ld32);
        else
          gemm_core<SEG, 64, PT_W, 16, 4, 2, 0, IN32>(P + s0, Akk + c0 + s0, Akk + c0, ld, S, w, c0, false, lds, Ps,
                                                      LDP, -1, false, -1, false, IN32 ? P32 + s0 : nullptr, ld32);
      } else if (tid < S) {
        double v[PT_W];
#pragma unroll
        for (int c = 0; c < PT_W; ++c)
          v[c] = IN32 ? (double)P32[(int64_t)imin(c, w - 1) * ld32 + s0 + tid] : P[(int64_t)imin(c, w - 1) * ld + s0 + tid];
#pragma unroll
        for (int c = 0; c < PT_W; ++c) Ps[c * LDP + tid] = v[c];
      }
      __syncthreads();
      if (s0 == 0) {
        if (wave == 0) {
          // the leading 16 x 16 block, the rows 16 .. w-1 below it solved in the same steps
          int info = diag16_x<LDP, PT_W + 1>(Ps, 0, imin(16, w), Ldd, Linv, lane, c0, imax(w - 16, 0));
          if (w > 16) {
            const int wb = w - 16;
            // trailing block -= (those rows)(those rows)^T: element v of lane
            // l is row 16 + 4v + l/16, column 16 + l%16 (rows and columns past
            // w only meet each other and are never read)
            {
              const int l16 = lane & 15, lg = lane >> 4;
              d4 acc;
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[v] = Ps[(16 + l16) * LDP + 16 + 4 * v + lg];
#pragma unroll
              for (int s = 0; s < 4; ++s) {
                const double f = Ps[(4 * s + lg) * LDP + 16 + l16];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(f, f, acc, 0, 0, 2 /* neg B */);
              }
#pragma unroll
              for (int v = 0; v < 4; ++v) Ps[(16 + l16) * LDP + 16 + 4 * v + lg] = acc[v];
            }
            const int info_b =
                diag16_x<LDP, PT_W + 1>(Ps, 16, wb, Ldd + 16 * (PT_W + 1) + 16, Linv + 16, lane, c0 + 16);
            info = info != 0 ? info : info_b;
          }
          if (lane == 0) s_info = info;
        }
        __syncthreads();
        const int info = __builtin_amdgcn_readfirstlane(s_info);
        if (info != 0) return info;
        // L_dd by columns for the rows below: column c at LT[c * PT_LT + c2]
        // (c2 > c), the reciprocal pivot at c2 = c
        for (int idx = tid; idx < PT_W * PT_W; idx += NT) {
          const int c = idx / PT_W, c2 = idx - c * PT_W;
          if (!PACKED || c2 >= c) LT[lt(c) + c2] = c2 == c ? Linv[c] : (c2 > c ? Ldd[c2 * (PT_W + 1) + c] : 0.0);
        }
        __syncthreads();
      }
      // rows below the diagonal block: y := y L_dd^{-T}, one row per thread
      // (there are such rows only when the panel is 32 wide); each column's
      // entries of L_dd are loaded together before they are used.  With Bf,
      // threads 128 + j of the first slab take the panel's rows of column j
      // of b (rows of the compact slab never reach thread 128)
      {
        const int r = (s0 == 0 ? w : 0) + tid;
        const int j = tid - 128;
        const bool rhs = fwd && s0 == 0 && j >= 0 && j < nrhs;
        if (r < S || rhs) {
          double y[PT_W];
          if (rhs) {
#pragma unroll
            for (int c = 0; c < PT_W; ++c) y[c] = c < w ? Bf[(int64_t)j * ldbf + c0 + c] : 0.0;
          } else {
#pragma unroll
            for (int c = 0; c < PT_W; ++c) y[c] = Ps[c * LDP + r];
          }
#pragma unroll
          for (int c = 0; c < PT_W; ++c) {
            double l[PT_W];
#pragma unroll
            for (int c2 = c; c2 < PT_W; ++c2) l[c2] = LT[lt(c) + c2];
#pragma unroll
            for (int c2 = c; c2 < PT_W; ++c2) asm volatile("" : : "v"(l[c2]));
            y[c] *= l[c];
#pragma unroll
            for (int c2 = c + 1; c2 < PT_W; ++c2) y[c2] -= y[c] * l[c2];
          }
          if (rhs) {
#pragma unroll
            for (int c = 0; c < PT_W; ++c) {
              Yp[c * PT_FWD + j] = y[c];
              if (c < w) st_dev(Bf + (int64_t)j * ldbf + c0 + c, y[c]);
            }
          } else {
#pragma unroll
            for (int c = 0; c < PT_W; ++c) Ps[c * LDP + r] = y[c];
          }
        }
      }
      __syncthreads();
      // the slab (lower part) to the tile, one row per thread; the next slab
      // reuses the LDS
      if (tid < S) {
#pragma unroll
        for (int c = 0; c < PT_W; ++c)
          if (c < w && s0 + tid >= c) {
            st_dev(P + (int64_t)c * ld + s0 + tid, Ps[c * LDP + tid]);
            if constexpr (IN32) st_dev(P32 + (int64_t)c * ld32 + s0 + tid, (float)Ps[c * LDP + tid]);
          }
        if (fwd && s0 + tid >= w) {
          // b(row) -= L(row, panel) y_panel for the rows below the block
          double* const bp = Bf + c0 + s0 + tid;
          double bv[PT_FWD];
#pragma unroll
          for (int jj = 0; jj < PT_FWD; ++jj) bv[jj] = jj < nrhs ? bp[(int64_t)jj * ldbf] : 0.0;
#pragma unroll
          for (int c = 0; c < PT_W; ++c) {
            if (c < w) {
              const double lv = Ps[c * LDP + tid];
#pragma unroll
              for (int jj = 0; jj < PT_FWD; ++jj) bv[jj] -= lv * Yp[c * PT_FWD + jj];
            }
          }
#pragma unroll
          for (int jj = 0; jj < PT_FWD; ++jj)
            if (jj < nrhs) st_dev(bp + (int64_t)jj * ldbf, bv[jj]);
        }
      }
      __syncthreads();
    }
    // the panel must be visible to every wavefront before the next panel's
    // update reads it
    wait_vmcnt<0>();
    __syncthreads();
  }
  return 0;
}

// ---------------------------------------------------------------------------
// TRSM work item: a strip of S <= 32 rows of A_ik, X := X L_kk^{-T}
// (mk = order of L_kk, a multiple of 16; X in FP64 or, in the mixed-precision
// factorization, FP32 storage, computed in FP64 either way).  Transposed, X^T := L_kk^{-1} X^T
// is a forward solve with the strip's rows as 32 right-hand sides (two
// groups of 16).  The strip lives in LDS as Xs[g][c][16] (row 16g + j,
// column c), which the MFMA fragments read without bank conflicts.  For
// each block of 16 columns, wavefronts 0 and 1 solve the block for their
// row group in four 4-column sub-steps on the matrix cores (the exact 4x4
// inverse of the diagonal block's sub-block applied by one MFMA, then one
// MFMA for the columns after it), then every wavefront subtracts the block's
// contribution from its later column blocks.  The solver's L data for the
// next step is requested one step ahead; the update fragments at the start
// of the step, to land during the solve.
//
// REV = 2: the same solve, also storing P^T at Qb (ld ldq): the explicit
// inverse of the mixed-precision solve, from identity strips.
#define TS 32

// Hs (non-null): the solved strip is also stored as three BF16 terms
// (split3) in K-contiguous rows: strip row r, column c of term t at
// Hs[t * hterm + r * hld + c] (the BF16 panels of the BF16-update factorization).
template <typename TX, int REV = 0>
__device__ __forceinline__ void trsm_strip(TX* __restrict__ X, int64_t ldx, const double* __restrict__ Lkk, int64_t ld,
                                           int S, int mk, double* lds, double* Qb = nullptr,
                                           int64_t ldq = 0, uint16_t* Hs = nullptr, int64_t hld = 0,
                                           int64_t hterm = 0) {
  double* Xs = lds;  // [2][512][16]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, lg = lane >> 4;
  const int nblk = mk >> 4;
  // L(row, col) of the operator the forward solve applies
  auto lat = [&](int row, int col) __attribute__((always_inline)) { return Lkk[(int64_t)col * ld + row]; };
  // the strip: thread (r, c0) moves rows r of columns c0 + 8u, 16 loads in flight
  {
    const int r = tid & 31, c0 = tid >> 5, rr = imin(r, S - 1);
#pragma unroll 1
    for (int part = 0; part < 4; ++part) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = (double)X[(int64_t)imin(c0 + 8 * (u + 16 * part), mk - 1) * ldx + rr];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int c = c0 + 8 * (u + 16 * part);
        if (c < mk) Xs[(r >> 4) * 8192 + c * 16 + (r & 15)] = (r < S) ? v[u] : 0.0;
      }
    }
  }
  // Step data.  Solver lanes (wavefronts 0, 1): the 4x4 sub-block entries
  // d[a][b] (a >= b) of sub-block s* = l16 / 4 and the update entries
  // L[q0 + l16][q0 + 4s + lg], requested one step ahead; every wavefront:
  // the fragments L[later column block rows, q0 + 4kk + lg], requested at
  // the start of the step and used after the block's solve.
  struct SolveData {
    double d[10];
    double fd[4];
  };
  auto fetch_solve = [&](int rb, SolveData& sd) __attribute__((always_inline)) {
    const int q0 = rb * 16;
    const int sb = q0 + 4 * (l16 >> 2);
    int n = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int bq = 0; bq <= a; ++bq) sd.d[n++] = lat(sb + a, sb + bq);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) sd.fd[s4] = lat(q0 + l16, q0 + 4 * s4 + lg);
  };
  auto step = [&](int rb, const SolveData& sd, SolveData& sdn) __attribute__((always_inline)) {
    const int q0 = rb * 16;
    __syncthreads();  // the block's columns are final (and, first time, the strip is staged)
    double fl[8][4];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int crow = imin(q0 + 16 + (wave + 4 * t) * 16 + l16, mk - 1);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) fl[t][kk] = lat(crow, q0 + kk * 4 + lg);
    }
    if (wave < 2) {
      if (rb + 1 < nblk) fetch_solve(rb + 1, sdn);
      const int g = wave;
      // column lg of the inverse of sub-block s* = l16 / 4; this lane's A entry is row l16 % 4
      double dd[4][4];
      {
        int n = 0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int bq = 0; bq < 4; ++bq) dd[a][bq] = (bq <= a) ? sd.d[n++] : 0.0;
      }
      double w[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        double t = (a == lg) ? 1.0 : 0.0;
#pragma unroll
        for (int bq = 0; bq < a; ++bq) t -= dd[a][bq] * w[bq];
        w[a] = (a < lg) ? 0.0 : t * (1.0 / dd[a][a]);
      }
      const int i4 = l16 & 3;
      const double wmine = (i4 == 0) ? w[0] : (i4 == 1) ? w[1] : (i4 == 2) ? w[2] : w[3];
      d4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = Xs[g * 8192 + (q0 + 4 * v + lg) * 16 + l16];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const double fw = ((l16 >> 2) == s4) ? wmine : 0.0;
        const d4 z = __builtin_amdgcn_mfma_f64_16x16x4f64(fw, acc[s4], d4{0.0, 0.0, 0.0, 0.0}, 0, 0, 0);
        acc[s4] = z[s4];
        const double fdv = (l16 >= 4 * s4 + 4) ? sd.fd[s4] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fdv, z[s4], acc, 0, 0, 2 /* neg B */);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) Xs[g * 8192 + (q0 + 4 * v + lg) * 16 + l16] = acc[v];
    }
    __syncthreads();
    // X^T[later column blocks] -= L[those rows, q0:q0+16] X^T[q0:q0+16] for both row groups
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int cb = rb + 1 + wave + 4 * t;
      if (cb < nblk) {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          d4 acc;
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[v] = Xs[g * 8192 + (cb * 16 + 4 * v + lg) * 16 + l16];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const double fx = Xs[g * 8192 + (q0 + kk * 4 + lg) * 16 + l16];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fl[t][kk], fx, acc, 0, 0, 2 /* neg B */);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) Xs[g * 8192 + (cb * 16 + 4 * v + lg) * 16 + l16] = acc[v];
        }
      }
    }
  };
  SolveData sa, sb;
  if (wave < 2) fetch_solve(0, sa);
  for (int rb = 0; rb < nblk; rb += 2) {
    step(rb, sa, sb);
    if (rb + 1 < nblk) step(rb + 1, sb, sa);
  }
  __syncthreads();
  const int r = tid & 31, c0 = tid >> 5;
  if (r < S)
    for (int c = c0; c < mk; c += 8) st_dev(X + (int64_t)c * ldx + r, (TX)Xs[(r >> 4) * 8192 + c * 16 + (r & 15)]);
  if (Hs) {
    // runs of 4 columns (8 bytes per term): lane l of wavefront w takes row
    // 16 (w & 1) + l % 16 (consecutive rows: conflict-free reads of Xs) and
    // runs 4 u + l / 16 of its half of the columns (w / 2); a store
    // instruction then writes 32-byte pieces of 16 rows
    const int hr = 16 * (wave & 1) + l16, half = mk >> 3;  // runs of 4 per half of the columns
    if (hr < S) {
#pragma unroll 1
      for (int u = 0; 4 * u + lg < half; ++u) {
        const int c0 = (wave >> 1) * (mk >> 1) + 4 * (4 * u + lg);
        uint64_t t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          uint32_t a0, a1, a2;
          split3(Xs[(hr >> 4) * 8192 + (c0 + e) * 16 + (hr & 15)], a0, a1, a2);
          t0 |= (uint64_t)a0 << (16 * e);
          t1 |= (uint64_t)a1 << (16 * e);
          t2 |= (uint64_t)a2 << (16 * e);
        }
        uint16_t* h = Hs + (int64_t)hr * hld + c0;
        st_dev(reinterpret_cast<uint64_t*>(h), t0);
        st_dev(reinterpret_cast<uint64_t*>(h + hterm), t1);
        st_dev(reinterpret_cast<uint64_t*>(h + 2 * hterm), t2);
      }
    }
  }
  if constexpr (REV == 2) {
    for (int idx = tid; idx < S * mk; idx += NT) {
      const int rr = idx / mk, c = idx - rr * mk;
      st_dev(Qb + (int64_t)rr * ldq + c, Xs[(rr >> 4) * 8192 + c * 16 + (rr & 15)]);
    }
  }
}

// ---------------------------------------------------------------------------
// TRSM work item through the diagonal tile's explicit inverse (FP64 launches
// that compute it, TRTRI(k) before TRSM(i, k)): rows of A_ik, X := X L_kk^{-T}
// = X (L_kk^{-1})^T, one 128-row block per item, as products with L_kk^{-1}
// (Linv, column-major, ld nb; entry (c, t) is zero for t > c) on the matrix
// cores.  Column block c of the result reads the columns of X up to the
// block's end, so the blocks go from the right to the left, each written
// after its own product has read it; no other item touches these rows.
template <int SEG>
__device__ __forceinline__ void trsm_inv_rows(double* __restrict__ X, int64_t ld, const double* __restrict__ Linv,
                                              int64_t nb, int M, int mk, double* lds) {
  for (int c0 = ((mk - 1) / GB) * GB; c0 >= 0; c0 -= GB) {
    const int N = imin(GB, mk - c0), K = c0 + N;
    // C = 0 - X Linv^T over K, stored negated
    if (K % 32 == 0)
      gemm_core<SEG, GB, GB, 32, 2, 2>(X + (int64_t)c0 * ld, X, Linv + c0, ld, M, N, K, false, lds, nullptr, 0, -1,
                                       true, nb, true);
    else
      gemm_core<SEG, GB, GB, 16, 2, 4>(X + (int64_t)c0 * ld, X, Linv + c0, ld, M, N, K, false, lds, nullptr, 0, -1,
                                       true, nb, true);
  }
}

// ---------------------------------------------------------------------------
// Solve work items.  Right-hand sides are processed 16 columns at a time
// (the N of an MFMA block).  MFMA layout used here: A operand = L fragment
// (rows of L on lanes % 16), B operand = right-hand-side fragment
// (right-hand sides on lanes % 16); a lane then holds rows 4i + lane/16 of
// one right-hand side (lane % 16) of the 16x16 result.

// Tile solves, register resident.  The tile's rows form blocks of 16
// (nblk <= 32); wavefront w owns blocks w, w + 4, ..., and keeps their
// right-hand sides in registers in the layout of an MFMA result: element v
// of lane l holds row 4v + l/16 of right-hand side l%16.  That is also the
// layout of the B operand of an MFMA's k-step v, so a solved block feeds the
// updates of the other blocks without leaving registers.
//
// Block rb is solved by its owner in four dependent 4-row sub-steps:
// y_s := W_s r_s with W_s the inverse of the s-th 4x4 diagonal block of L
// (one MFMA whose A operand is W_s in rows 4s..4s+3 and zero elsewhere),
// then the rows below lose L[rows, 4s..4s+3] y_s (one MFMA).  The 4x4
// inverses are formed once per task by substitution; a 4x4 inverse of an
// integer factor with power-of-two pivots is exact, so such systems are
// still solved exactly.  The solved block is published through LDS (two
// buffers, one barrier per block) and every wavefront subtracts its
// contribution from the blocks it owns; the owner of the next block
// updates and solves that block first.  The L fragments of block rb's
// updates are requested one block ahead.
//
// LDS: Fr[blk][s][f][64] the A-operand fragments of the sub-steps (f = 0:
// inverse, f = 1: update), then two 16 x 16 exchange buffers.
#define FR_SLOT(blk, s, f) ((((blk) * 4 + (s)) * 2 + (f)) * 64)
#define FR0_SLOT(blk, s) (((blk) * 4 + (s)) * 64)  // COMPACT: the inverses only

// Builds Fr for the forward (trans = false) or backward (trans = true)
// solve of the nblk diagonal 16-blocks of L_kk (m rows).  Rows and columns
// past m behave as the identity.  COMPACT: only the inverse fragments (the
// update fragments are read from L_kk by the solve).
template <bool COMPACT = false>
__device__ __forceinline__ void build_block_fragments(const double* __restrict__ Lkk, int64_t ld, int m,
                                                      bool trans, double* Fr) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int s = tid >> 6;  // wavefront w builds sub-step w of every block
  const int l16 = lane & 15, lg = lane >> 4;
  const int nblk = (m + 15) >> 4;
  auto slot0 = [](int blk, int s4) __attribute__((always_inline)) {
    return COMPACT ? FR0_SLOT(blk, s4) : FR_SLOT(blk, s4, 0);
  };
  if constexpr (COMPACT) {
    for (int blk = 0; blk < nblk; ++blk) Fr[FR0_SLOT(blk, s) + lane] = 0.0;
  } else {
    // update fragments (and zeros in the inverse slots): all 32 loads are
    // requested before any is used.  Forward: A[i][k] = L[r0+i][r0+4s+k] for
    // i >= 4s+4; backward: A[i][k] = L[r0+4s+k][r0+i] for i < 4s.
    const int row = trans ? 4 * s + lg : l16, col = trans ? l16 : 4 * s + lg;
    const bool live = trans ? (l16 < 4 * s) : (l16 >= 4 * s + 4);
    double v[32];
#pragma unroll
    for (int blk = 0; blk < 32; ++blk) {
      const int r0 = imin(blk, nblk - 1) * 16, bw = imin(16, m - r0);
      v[blk] = Lkk[(int64_t)(r0 + imin(col, bw - 1)) * ld + r0 + imin(row, bw - 1)];
    }
#pragma unroll
    for (int blk = 0; blk < 32; ++blk) {
      if (blk < nblk) {
        const int bw = imin(16, m - blk * 16);
        Fr[FR_SLOT(blk, s, 1) + lane] = (live & (row < bw) & (col < bw)) ? v[blk] : 0.0;
        Fr[FR_SLOT(blk, s, 0) + lane] = 0.0;
      }
    }
  }
  __syncthreads();
  // column c of the inverse of the 4x4 block (blk, s), by substitution; a
  // thread takes blocks tid/16 and tid/16 + 16
  {
    const int c = tid & 3, s4 = (tid >> 2) & 3;
    double d[2][4][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int blk = imin((tid >> 4) + 16 * h, nblk - 1);
      const int r0 = blk * 16 + 4 * s4, bw = imin(4, m - r0);  // bw may be <= 0: identity
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double x = Lkk[(int64_t)(imin(m - 1, r0 + j)) * ld + imin(m - 1, r0 + i)];
          d[h][i][j] = ((j <= i) & (i < bw) & (j < bw)) ? x : (i == j ? 1.0 : 0.0);
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int blk = (tid >> 4) + 16 * h;
      if (blk < nblk) {
        double w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          double t = (i == c) ? 1.0 : 0.0;
#pragma unroll
          for (int j = 0; j < i; ++j) t -= d[h][i][j] * w[j];
          w[i] = (i < c) ? 0.0 : t * (1.0 / d[h][i][i]);
        }
        // forward A[i'][k'] = W[i'-4s][k'] (i' in 4s..4s+3) -> lane k'*16 + i';
        // backward A[i'][k'] = W[k'][i'-4s] -> lane i*16 + 4s + c
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i >= c) Fr[slot0(blk, s4) + (trans ? i * 16 + 4 * s4 + c : c * 16 + 4 * s4 + i)] = w[i];
      }
    }
  }
  __syncthreads();
}

// Solves the owner's block in place (acc: the block's right-hand sides).
__device__ __forceinline__ void solve_block(d4& acc, const double* Fr, int blk, bool trans, int lane) {
#pragma unroll
  for (int ss = 0; ss < 4; ++ss) {
    const int s = trans ? 3 - ss : ss;
    const d4 z = __builtin_amdgcn_mfma_f64_16x16x4f64(Fr[FR_SLOT(blk, s, 0) + lane], acc[s], d4{0.0, 0.0, 0.0, 0.0},
                                                     0, 0, 0);
    acc[s] = z[s];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Fr[FR_SLOT(blk, s, 1) + lane], z[s], acc, 0, 0, 2 /* neg B */);
  }
}

// The same with the inverse fragments of the compact layout and the update
// fragments fu (sub-step order ss) read from L_kk: entry (row, col) of the
// block's sub-step s = trans ? 3 - ss : ss, zero outside its live part.
__device__ __forceinline__ void solve_block_c(d4& acc, const double* Fr, int blk, const double (&fu)[4], int m,
                                              bool trans, int lane) {
  const int l16 = lane & 15, lg = lane >> 4;
  const int bw = imin(16, m - blk * 16);
#pragma unroll
  for (int ss = 0; ss < 4; ++ss) {
    const int s = trans ? 3 - ss : ss;
    const int row = trans ? 4 * s + lg : l16, col = trans ? l16 : 4 * s + lg;
    const bool live = (trans ? (l16 < 4 * s) : (l16 >= 4 * s + 4)) & (row < bw) & (col < bw);
    const d4 z = __builtin_amdgcn_mfma_f64_16x16x4f64(Fr[FR0_SLOT(blk, s) + lane], acc[s], d4{0.0, 0.0, 0.0, 0.0},
                                                     0, 0, 0);
    acc[s] = z[s];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(live ? fu[ss] : 0.0, z[s], acc, 0, 0, 2 /* neg B */);
  }
}

// trans = false: Y_k := L_kk^{-1} B_k; trans = true: X_k := L_kk^{-T} Y_k.
// COMPACT (the compact instance, 69632 bytes of LDS, 256 registers): Fr
// holds only the blocks' inverse fragments, the update fragments of the
// block a step solves are loaded from L_kk one step ahead, and the step's
// update fragments at its start (one buffer instead of two: the other
// workgroup on the compute unit covers the wait).
template <bool COMPACT = false>
__device__ __forceinline__ void tile_solve(const double* __restrict__ Lkk, int64_t ld, double* Bk, int64_t ldb,
                                           int m, int nrhs, bool trans, double* lds) {
  double* Fr = lds;                                      // [nblk][4][2][64] (COMPACT: [nblk][4][64])
  double* Ex = lds + 32 * 4 * (COMPACT ? 1 : 2) * 64;  // [2][4][64]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, lg = lane >> 4;
  const int nblk = (m + 15) >> 4;
  build_block_fragments<COMPACT>(Lkk, ld, m, trans, Fr);
  // COMPACT: the raw entries behind block blk's update fragments (sub-step
  // order), clamped into the tile; solve_block_c masks them
  auto fetch_fu = [&](int blk, double (&fu)[4]) __attribute__((always_inline)) {
    const int r0 = imin(imax(blk, 0), nblk - 1) * 16, bw = imin(16, m - r0);
#pragma unroll
    for (int ss = 0; ss < 4; ++ss) {
      const int s = trans ? 3 - ss : ss;
      const int row = trans ? 4 * s + lg : l16, col = trans ? l16 : 4 * s + lg;
      fu[ss] = Lkk[(int64_t)(r0 + imin(col, bw - 1)) * ld + r0 + imin(row, bw - 1)];
    }
  };
  // fragments of the updates by solved block rb of the owned blocks ub = wave + 4t:
  // forward L[ub rows][rb cols], backward L[rb rows][ub cols]^T
  // Only the blocks the solved block rb still updates are fetched (forward:
  // ub > rb, backward: ub < rb): the same blocks that use the fragments.
  auto fetch = [&](int rb, double (&fl)[8][4]) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int ub = wave + 4 * t;
      if (trans ? (ub < rb) : (ub > rb && ub < nblk)) {
        const int ur = imin(ub * 16 + l16, m - 1);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int q = imin(rb * 16 + 4 * kk + lg, m - 1);
          fl[t][kk] = trans ? Lkk[(int64_t)ur * ld + q] : Lkk[(int64_t)q * ld + ur];
        }
      }
    }
  };
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    const int jn = imin(16, nrhs - j0);
    const int jc = imin(l16, jn - 1);
    d4 acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = (wave + 4 * t) * 16 + 4 * v + lg;
        const double x = Bk[(int64_t)(j0 + jc) * ldb + imin(row, m - 1)];
        acc[t][v] = (row < m) ? x : 0.0;
      }
    const int first = trans ? nblk - 1 : 0;
    double fla[8][4], flb[8][4];
    double fua[4], fub[4];  // COMPACT: update fragments of the block a step solves
    if constexpr (COMPACT)
      fetch_fu(first, fub);
    else
      fetch(first, fla);
    // the first block: solved by its owner, published in buffer 0
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (wave + 4 * t == first) {
        if constexpr (COMPACT)
          solve_block_c(acc[t], Fr, first, fub, m, trans, lane);
        else
          solve_block(acc[t], Fr, first, trans, lane);
#pragma unroll
        for (int v = 0; v < 4; ++v) Ex[v * 64 + lane] = acc[t][v];
      }
    if constexpr (COMPACT) fetch_fu(trans ? first - 1 : first + 1, fua);
    __syncthreads();
    // one step: block rb is solved and published in buffer (step & 1); its
    // contribution goes to every block still to be solved, the next block first
    auto step = [&](int step_i, const double (&fl)[8][4], double (&fln)[8][4], const double (&fu)[4],
                    double (&fun)[4]) __attribute__((always_inline)) {
      const int rb = trans ? nblk - 1 - step_i : step_i;
      const int nx = trans ? rb - 1 : rb + 1;
      const bool has_next = trans ? (rb > 0) : (rb + 1 < nblk);
      const double* ex = Ex + (step_i & 1) * 256;
      double* exn = Ex + ((step_i + 1) & 1) * 256;
      d4 yb;
#pragma unroll
      for (int v = 0; v < 4; ++v) yb[v] = ex[v * 64 + lane];
      if constexpr (COMPACT) {
        // one buffer (fl and fln are the same array): this step's fragments
        // now, the next solved block's update fragments one step ahead
        fetch(rb, fln);
        if (has_next) fetch_fu(trans ? nx - 1 : nx + 1, fun);
      } else if (has_next) {
        fetch(nx, fln);
      }
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (has_next && wave + 4 * t == nx) {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(fl[t][kk], yb[kk], acc[t], 0, 0, 2 /* neg B */);
          if constexpr (COMPACT)
            solve_block_c(acc[t], Fr, nx, fu, m, trans, lane);
          else
            solve_block(acc[t], Fr, nx, trans, lane);
#pragma unroll
          for (int v = 0; v < 4; ++v) exn[v * 64 + lane] = acc[t][v];
        }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int ub = wave + 4 * t;
        if ((trans ? ub < nx : (ub > nx && ub < nblk))) {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(fl[t][kk], yb[kk], acc[t], 0, 0, 2 /* neg B */);
        }
      }
      __syncthreads();
    };
    for (int si = 0; si < nblk; si += 2) {
      if constexpr (COMPACT) {
        step(si, fla, fla, fua, fub);
        if (si + 1 < nblk) step(si + 1, fla, fla, fub, fua);
      } else {
        step(si, fla, flb, fua, fub);
        if (si + 1 < nblk) step(si + 1, flb, fla, fub, fua);
      }
    }
    if (l16 < jn) {
#pragma unroll
      for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = (wave + 4 * t) * 16 + 4 * v + lg;
          if (row < m) st_dev(Bk + (int64_t)(j0 + l16) * ldb + row, acc[t][v]);
        }
    }
  }
}

// The strip update of gemv_strip with 16-byte transfers (two FP64 values,
// or two FP32 values in 8 bytes, per lane and load): half the load
// instructions.  K is taken in pairs of k-steps: step u of a wavefront
// covers K index kw + 8 (u / 2) + 2 (lane / 16) + u % 2, so that a lane's two
// consecutive indices sit in steps 2j and 2j + 1.  Without TRANS a lane's
// rows of L are paired instead: block t holds the strip's rows 2 m + t
// (m = lane % 16), both loaded by one transfer.  Needs a full strip of 32
// rows, a K range whose length is a multiple of 8 and starts even, even
// leading dimensions and 16-byte aligned L and X; then every step of every
// wavefront lies inside K and nothing is masked.
template <typename TL, bool TRANS, bool ASSIGN>
__device__ __forceinline__ void gemv_strip_wide(const TL* __restrict__ L, int64_t ld, double* Y, const double* X,
                                                int64_t ldb, int k0, int k1, int nrhs, double* lds) {
  typedef TL TL2 __attribute__((ext_vector_type(2)));
  typedef const __attribute__((address_space(1))) char gchar;
  typedef const __attribute__((address_space(1))) TL2 gTL2;
  double* Ps = lds;  // [wavefront][8][64]: the partial products
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, lg = lane >> 4;
  const int nsteps = (k1 - k0) >> 2;                // even
  const int qs = (((nsteps + 3) >> 2) + 1) & ~1;    // per wavefront, even, at most 32
  const int ns = imax(0, imin(qs, nsteps - wave * qs));  // even
  const int kw = k0 + 4 * wave * qs + 2 * lg;      // this lane's first K index
  gchar* const Lu = (gchar*)uniform_ptr(L);
  const uint32_t es = sizeof(TL), lds_b = (uint32_t)ld * es;
  double fa[32], fb[32];
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (2 * j < ns) {
      const uint32_t c = (uint32_t)(kw + 8 * j);
      if (TRANS) {  // rows c, c + 1 of columns l16 and 16 + l16
        const TL2 va = *(gTL2*)(Lu + ((uint32_t)l16 * lds_b + c * es));
        const TL2 vb = *(gTL2*)(Lu + ((uint32_t)(16 + l16) * lds_b + c * es));
        fa[2 * j] = (double)va[0];
        fa[2 * j + 1] = (double)va[1];
        fb[2 * j] = (double)vb[0];
        fb[2 * j + 1] = (double)vb[1];
      } else {      // rows 2 l16, 2 l16 + 1 of columns c and c + 1
        const TL2 v0 = *(gTL2*)(Lu + (__umul24(c, lds_b) + (uint32_t)(2 * l16) * es));
        const TL2 v1 = *(gTL2*)(Lu + (__umul24(c + 1, lds_b) + (uint32_t)(2 * l16) * es));
        fa[2 * j] = (double)v0[0];
        fb[2 * j] = (double)v0[1];
        fa[2 * j + 1] = (double)v1[0];
        fb[2 * j + 1] = (double)v1[1];
      }
    }
  // output element (t, v) of a lane: strip row 2 (4 v + lg) + t (paired rows)
  // or 16 t + 4 v + lg (TRANS); this wavefront adds up two of the eight
  auto out_row = [&](int t, int v) __attribute__((always_inline)) {
    return TRANS ? 16 * t + 4 * v + lg : 2 * (4 * v + lg) + t;
  };
  const int ob = wave >> 1;
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    const int jn = imin(16, nrhs - j0);
    const int jc = j0 + imin(l16, jn - 1);
    const double* const Xj = X + (int64_t)jc * ldb + kw;
    double x[32];
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (2 * j < ns) {
        typedef double dd2 __attribute__((ext_vector_type(2)));
        const dd2 v = *reinterpret_cast<const dd2*>(Xj + 8 * j);
        x[2 * j] = v[0];
        x[2 * j + 1] = v[1];
      }
    double y[2] = {0.0, 0.0};
    if (!ASSIGN)
#pragma unroll
      for (int h = 0; h < 2; ++h) y[h] = Y[(int64_t)jc * ldb + out_row(ob, 2 * (wave & 1) + h)];
    d4 acc[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (2 * j < ns) {
#pragma unroll
        for (int u = 2 * j; u < 2 * j + 2; ++u) {
          acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[u], x[u], acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[u], x[u], acc[1], 0, 0, 0);
        }
      }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) Ps[(wave * 8 + 4 * t + v) * 64 + lane] = acc[t][v];
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = 4 * ob + 2 * (wave & 1) + h;
      double s = ASSIGN ? Ps[e * 64 + lane] : y[h] - Ps[e * 64 + lane];
#pragma unroll
      for (int w = 1; w < 4; ++w) s = ASSIGN ? s + Ps[(w * 8 + e) * 64 + lane] : s - Ps[(w * 8 + e) * 64 + lane];
      if (l16 < jn) st_dev(Y + (int64_t)(j0 + l16) * ldb + out_row(ob, e & 3), s);
    }
    __syncthreads();
  }
}

// Solve update on one strip of at most 32 output rows:
//     Y := Y - op(L) X     or, ASSIGN,     Y := op(L) X
// with op(L) = L (output row r, K index c at L[c ld + r]: the forward
// update, and the diagonal steps that apply an explicit inverse) or, TRANS,
// L^T (output row r, K index c at L[r ld + c]: the backward update).  K runs
// over [k0, k1) (row c of X at X[c]); right-hand side j at column j (ld ldb).
// These items sit on the solve's dependency chain and move little data, so
// their time is memory latency: the four wavefronts take a quarter of K each
// and request all of their L fragments (two 16-row blocks, up to 32 k-steps
// of 4) and right-hand-side fragments before the first product, one round
// trip per item.  The quarters' partial products meet in LDS and are added
// in wavefront order, so the result does not depend on timing.  L in FP64
// or FP32 (the mixed-precision working copy); X and Y in FP64.
template <typename TL, bool TRANS, bool ASSIGN>
__device__ __forceinline__ void gemv_strip(const TL* __restrict__ L, int64_t ld, double* Y, const double* X,
                                           int64_t ldb, int rows, int k0, int k1, int nrhs, double* lds) {
  if (rows == 32 && ((k1 - k0) & 7) == 0 && (k0 & 1) == 0 && ((ld | ldb) & 1) == 0 &&
      ((reinterpret_cast<uintptr_t>(L) | reinterpret_cast<uintptr_t>(X)) & 15) == 0) {
    gemv_strip_wide<TL, TRANS, ASSIGN>(L, ld, Y, X, ldb, k0, k1, nrhs, lds);
    return;
  }
  double* Ps = lds;  // [wavefront][8][64]: the partial products
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, lg = lane >> 4;
  const int nsteps = (k1 - k0 + 3) >> 2;  // k-steps of 4
  const int qs = (nsteps + 3) >> 2;       // per wavefront: at most 32 (K <= 512)
  const int ns = imax(0, imin(qs, nsteps - wave * qs));
  const int kw = k0 + 4 * wave * qs;
  const int kend = imin(k1, kw + 4 * ns);  // end of this wavefront's K
  const int ra = imin(l16, rows - 1), rb = imin(16 + l16, rows - 1);
  // L fragments by 32-bit byte offsets from a wave-uniform base (the item
  // spans less than 4 GB: at most 512 columns of at most 614400 rows), so
  // that a fragment's address costs a multiply-add instead of 64-bit
  // arithmetic.  Fragments of k-steps past this wavefront's quarter are
  // loaded (in bounds) but meet zeros in place of X, in groups of 8 k-steps.
  typedef const __attribute__((address_space(1))) char gchar;
  typedef const __attribute__((address_space(1))) TL gTL;
  gchar* const Lu = (gchar*)uniform_ptr(L);
  const uint32_t es = sizeof(TL), lds_b = (uint32_t)ld * es;
  const uint32_t offa = TRANS ? (uint32_t)ra * lds_b : (uint32_t)ra * es;
  const uint32_t offb = TRANS ? (uint32_t)rb * lds_b : (uint32_t)rb * es;
  double fa[32], fb[32];
#pragma unroll
  for (int g = 0; g < 4; ++g)
    if (8 * g < ns) {
#pragma unroll
      for (int u = 8 * g; u < 8 * g + 8; ++u) {
        const uint32_t c = (uint32_t)imin(kw + 4 * u + lg, k1 - 1);
        const uint32_t oc = TRANS ? c * es : __umul24(c, lds_b);
        fa[u] = (double)*(gTL*)(Lu + (offa + oc));
        fb[u] = (double)*(gTL*)(Lu + (offb + oc));
      }
    }
  // this wavefront's two outputs of the strip's eight per lane: block wave / 2,
  // rows 4 v + lg with v = 2 (wave % 2) + h
  const int ob = wave >> 1;
  for (int j0 = 0; j0 < nrhs; j0 += 16) {
    const int jn = imin(16, nrhs - j0);
    const int jc = j0 + imin(l16, jn - 1);
    const double* const Xj = X + (int64_t)jc * ldb;
    // loaded unconditionally (in bounds) and masked at their use: a select
    // between a loaded value and zero would be turned into a branch around
    // each load, with a wait for it at the join
    double x[32];
#pragma unroll
    for (int g = 0; g < 4; ++g)
      if (8 * g < ns) {
#pragma unroll
        for (int u = 8 * g; u < 8 * g + 8; ++u) x[u] = Xj[imin(kw + 4 * u + lg, k1 - 1)];
      }
    double y[2] = {0.0, 0.0};
    if (!ASSIGN)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = 16 * ob + 4 * (2 * (wave & 1) + h) + lg;
        y[h] = Y[(int64_t)jc * ldb + imin(r, rows - 1)];
      }
    d4 acc[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
    for (int g = 0; g < 4; ++g)
      if (8 * g < ns) {
#pragma unroll
        for (int u = 8 * g; u < 8 * g + 8; ++u) {
          const double xv = (kw + 4 * u + lg < kend) ? x[u] : 0.0;
          acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[u], xv, acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[u], xv, acc[1], 0, 0, 0);
        }
      }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) Ps[(wave * 8 + 4 * t + v) * 64 + lane] = acc[t][v];
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = 4 * ob + 2 * (wave & 1) + h;
      double s = ASSIGN ? Ps[e * 64 + lane] : y[h] - Ps[e * 64 + lane];
#pragma unroll
      for (int w = 1; w < 4; ++w) s = ASSIGN ? s + Ps[(w * 8 + e) * 64 + lane] : s - Ps[(w * 8 + e) * 64 + lane];
      const int r = 16 * ob + 4 * (e & 3) + lg;
      if (l16 < jn && r < rows) st_dev(Y + (int64_t)(j0 + l16) * ldb + r, s);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// POTRF of the mixed-precision factorization: the diagonal tiles live in
// FP64 in the workspace (Dk, ld nb) from the start (copied from A) and take
// their SYRK updates there, so the tile is factored in place by the FP64
// tile kernel.  Dk then holds L_kk for the TRSM strips of step k and the
// tile's inverses (TRTRI); the FP32 copy's diagonal tiles are never read.
__device__ __forceinline__ int potrf_tile_mixed(double* __restrict__ Dk, int64_t ldd, int m, double* lds) {
  const int tid = threadIdx.x;
  const int info = __builtin_amdgcn_readfirstlane(m <= 128 ? potrf_small(Dk, ldd, m, lds) : potrf_tile<128>(Dk, ldd, m, lds));
  // a ragged tile is padded to a multiple of 16 with the identity (for its
  // explicit inverse, which then holds L^{-1} in its leading m x m block)
  const int mpad = (m + 15) & ~15;
  for (int idx = tid; idx < mpad * mpad; idx += NT) {
    const int c = idx / mpad, r = idx - c * mpad;
    if (r >= c && (r >= m || c >= m)) st_dev(Dk + (int64_t)c * ldd + r, r == c ? 1.0 : 0.0);
  }
  return info;
}

// ---------------------------------------------------------------------------
// DRED work item: rows [r0, r0 + 16) of the diagonal tile's Lbar (ld) get
// the tile's partial products added, slot by slot in a fixed order (each slot
// holds -tril(P_ik^T L_ik), nb x nb at stride slot_stride, ld ldslot; only
// the lower triangle is read and written).  Eight entries per thread and
// four slots per round keep 32 loads in flight.  With LbT set, the strip's
// rows also go transposed into columns [r0, r0 + 16) of LbT (ld ldt), zero
// below the diagonal: Lbar_kk^T for the closed-form tile adjoint.
__device__ __forceinline__ void dred_strip(double* __restrict__ Bkk, int64_t ld, const double* __restrict__ slots,
                                           int64_t slot_stride, int nslots, int64_t ldslot, int m, int r0,
                                           double* __restrict__ LbT = nullptr, int64_t ldt = 0) {
  const int tid = threadIdx.x;
  const int ncol = imin(r0 + 16, m);          // columns that hold lower entries of these rows
  const int tot = 16 * ncol;                  // (row, column) pairs, rows fastest
  for (int base = 0; base < tot; base += 8 * NT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = imin(base + u * NT + tid, tot - 1), c = idx >> 4, r = imin(r0 + (idx & 15), m - 1);
      v[u] = Bkk[(int64_t)c * ld + r];
    }
    for (int s0 = 0; s0 < nslots; s0 += 4) {
      double t[4][8];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int idx = imin(base + u * NT + tid, tot - 1), c = idx >> 4, r = imin(r0 + (idx & 15), m - 1);
          t[q][u] = (s0 + q < nslots) ? slots[(int64_t)(s0 + q) * slot_stride + (int64_t)c * ldslot + r] : 0.0;
        }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] += t[q][u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * NT + tid, c = idx >> 4, r = r0 + (idx & 15);
      if (idx < tot && r < m && r >= c) {
        st_dev(Bkk + (int64_t)c * ld + r, v[u]);
        if (LbT) st_dev(LbT + (int64_t)r * ldt + c, v[u]);
      }
      if (LbT && idx < tot && r < m && r < c) st_dev(LbT + (int64_t)r * ldt + c, 0.0);
    }
  }
  if (LbT) {  // the transposed rows below the strip's columns: zero
    const int rows = imin(r0 + 16, m) - r0, below = m - ncol;
    for (int idx = tid; idx < rows * below; idx += NT) {
      const int rr = idx / below, c = ncol + idx - rr * below;
      st_dev(LbT + (int64_t)(r0 + rr) * ldt + c, 0.0);
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the factorization of a diagonal tile.  In lower-parameter form
// (the derivative with respect to the entries the factorization reads, the
// lower triangle; Q = P + P^T is twice the symmetric adjoint), the reverse of
// a right-looking tile factorization with tiles of w has, per step k taken
// from the last to the first,
//   Lbar_ik -= sum_{j > k} Q_ij L_jk             (i > k)
//   P_ik     = Lbar_ik L_kk^{-1}                 (i > k)
//   Lbar_kk -= tril(sum_{i > k} P_ik^T L_ik)
//   P_kk     = the adjoint of the w x w factorization:
//              tril(G + G^T) - diag(G),  G = L_kk^{-T} Phi(L_kk^T Lbar_kk) L_kk^{-1}
//              (Phi: lower triangle with the diagonal halved).
// The tile's own adjoint applies this with w = 16 inside the tile, panels
// from the right: the matrix cores form the first line for the panel's rows
// below its diagonal block (Q of the tile as far as it is known, from the
// workspace), one thread per row solves the second, every thread takes one
// entry of the 16 x 16 third and fourth (the 16 x 16 inverse by substitution),
// and the panel's P is written to Q in both orientations and, halved off the
// diagonal (the symmetric adjoint), over Lbar.  Before the panels, the
// partial products of the tile's column are applied to Lbar_kk in a fixed
// order; each slot holds -tril(P_ik^T L_ik) (the tile product subtracts from
// a zero start), so they are added.  Lkk, Bkk: the factor and Lbar tiles (ld);
// LTkk, Qkk: the transposed factor and Q tiles (ldq, zero beyond the order).
__device__ __forceinline__ void prev_tile(const double* __restrict__ Lkk, const double* __restrict__ LTkk,
                                          double* __restrict__ Bkk, int64_t ld, double* __restrict__ Qkk, int64_t ldq,
                                          int m, const double* __restrict__ slots, int64_t slot_stride, int nslots,
                                          int64_t ldslot, double* lds) {
  const int tid = threadIdx.x;
  double* Ps = lds + P_STAGE_DOUBLES;  // [PW][PPLD] the panel's rows below its diagonal block
  double* Ls = Ps + PW * PPLD;         // [16][17] L of the diagonal block, identity-padded
  double* Bs = Ls + 16 * 17;           // [16][17] its Lbar
  double* Ms = Bs + 16 * 17;
  double* Is = Ms + 16 * 17;           // L^{-1} of the block
  double* Ys = Is + 16 * 17;
  double* Gs = Ys + 16 * 17;
  const int ta = tid >> 4, tb = tid & 15;  // the entry (row, column) a thread owns in 16 x 16 steps

  // Lbar_kk -= tril(P_ik^T L_ik), slot by slot (each slot holds the negated product)
  if (nslots > 0) {
    const int tot = m * m;
    for (int base = 0; base < tot; base += 16 * NT) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int idx = imin(base + u * NT + tid, tot - 1), c = idx / m, r = idx - c * m;
        v[u] = Bkk[(int64_t)c * ld + r];
      }
      for (int sl = 0; sl < nslots; ++sl) {
        const double* S0 = slots + (int64_t)sl * slot_stride;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int idx = imin(base + u * NT + tid, tot - 1), c = idx / m, r = idx - c * m;
          v[u] += (r >= c) ? S0[(int64_t)c * ldslot + r] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int idx = base + u * NT + tid, c = idx / m, r = idx - c * m;
        if (idx < tot && r >= c) st_dev(Bkk + (int64_t)c * ld + r, v[u]);
      }
    }
    wait_vmcnt<0>();
    __syncthreads();
  }
  const int mpad = (m + 15) & ~15;
  for (int c0 = ((m - 1) >> 4) << 4; c0 >= 0; c0 -= PW) {
    const int w = imin(PW, m - c0), R = m - c0;
    // (1) rows below the block: Lbar - Q L over the columns right of the panel, into LDS
    for (int s0 = 16; s0 < R; s0 += 256) {
      gemm_core<128, 256, PW, 8, 4, 4, 0>(Bkk + (int64_t)c0 * ld + c0 + s0, Qkk + (int64_t)(c0 + 16) * ldq + c0 + s0,
                                          LTkk + (int64_t)(c0 + 16) * ldq + c0, ldq, imin(256, R - s0), w,
                                          mpad - c0 - 16, false, lds, Ps + s0, PPLD, ld);
      __syncthreads();
    }
    {
      const bool in = ta < w && tb < w;
      Ls[ta * 17 + tb] = in ? (ta >= tb ? Lkk[(int64_t)(c0 + tb) * ld + c0 + ta] : 0.0) : (ta == tb ? 1.0 : 0.0);
      Bs[ta * 17 + tb] = (in && ta >= tb) ? Bkk[(int64_t)(c0 + tb) * ld + c0 + ta] : 0.0;
    }
    // the panel's L rows below the block, for the diagonal block's update (stage area is free)
    for (int idx = tid; idx < w * (R - 16); idx += NT) {
      const int c = idx / (R - 16), r = 16 + idx - c * (R - 16);
      lds[c * PPLD + r] = Lkk[(int64_t)(c0 + c) * ld + c0 + r];
    }
    __syncthreads();
    // (2) P rows := Lbar rows L_dd^{-1}: back substitution over the block's columns
    for (int r = 16 + tid; r < R; r += NT) {
      double y[PW];
#pragma unroll
      for (int c = 0; c < PW; ++c) y[c] = (c < w) ? Ps[c * PPLD + r] : 0.0;
#pragma unroll
      for (int c = PW - 1; c >= 0; --c) {
#pragma unroll
        for (int c2 = c + 1; c2 < PW; ++c2) y[c] -= y[c2] * Ls[c2 * 17 + c];
        y[c] = y[c] / Ls[c * 17 + c];
      }
#pragma unroll
      for (int c = 0; c < PW; ++c) Ps[c * PPLD + r] = y[c];
    }
    __syncthreads();
    // (3) Lbar_dd -= tril(P^T L) over the rows below the block
    if (ta >= tb && ta < w) {
      double acc = 0.0;
      for (int r = 16; r < R; ++r) acc += Ps[ta * PPLD + r] * lds[tb * PPLD + r];
      Bs[ta * 17 + tb] -= acc;
    }
    __syncthreads();
    // (4) the 16 x 16 adjoint
    {
      double acc = 0.0;
      if (ta >= tb)
        for (int t = ta; t < 16; ++t) acc += Ls[t * 17 + ta] * Bs[t * 17 + tb];
      Ms[ta * 17 + tb] = (ta == tb) ? 0.5 * acc : acc;
    }
    if (tid < 16) {
      const int c = tid;
      for (int r = 0; r < 16; ++r) {
        double v = (r == c) ? 1.0 : 0.0;
        for (int t = c; t < r; ++t) v -= Ls[r * 17 + t] * Is[t * 17 + c];
        Is[r * 17 + c] = (r < c) ? 0.0 : v / Ls[r * 17 + r];
      }
    }
    __syncthreads();
    {
      double acc = 0.0;
      for (int t = 0; t < 16; ++t) acc += Ms[ta * 17 + t] * Is[t * 17 + tb];
      Ys[ta * 17 + tb] = acc;
    }
    __syncthreads();
    {
      double acc = 0.0;
      for (int t = 0; t < 16; ++t) acc += Is[t * 17 + ta] * Ys[t * 17 + tb];
      Gs[ta * 17 + tb] = acc;
    }
    __syncthreads();
    // (5) write: Q (both orientations) and the symmetric adjoint over Lbar
    if (ta < w && tb < w) {
      const double g = Gs[ta * 17 + tb] + Gs[tb * 17 + ta];  // P_ab + P_ba off the diagonal, 2 P_aa on it
      st_dev(Qkk + (int64_t)(c0 + tb) * ldq + c0 + ta, g);
      if (ta >= tb) st_dev(Bkk + (int64_t)(c0 + tb) * ld + c0 + ta, (ta == tb) ? Gs[ta * 17 + ta] : 0.5 * g);
    }
    for (int idx = tid; idx < w * (R - 16); idx += NT) {
      const int c = idx / (R - 16), r = 16 + idx - c * (R - 16);
      const double v = Ps[c * PPLD + r];
      st_dev(Qkk + (int64_t)(c0 + c) * ldq + c0 + r, v);
      st_dev(Bkk + (int64_t)(c0 + c) * ld + c0 + r, 0.5 * v);
    }
    for (int idx = tid; idx < w * (R - 16); idx += NT) {
      const int r = 16 + idx / w, c = idx - (r - 16) * w;
      st_dev(Qkk + (int64_t)(c0 + r) * ldq + c0 + c, Ps[c * PPLD + r]);
    }
    wait_vmcnt<0>();
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Adjoint of a diagonal tile in closed form.  For the tile factorization
// L_kk L_kk^T = A_kk and the adjoint Lbar_kk of its factor (after the
// partial products of its column), the adjoint with respect to the tile is
// the symmetric matrix S / 2 with
//     S = L^{-T} (M + M^T) L^{-1} = L^{-T} Y + Y^T L^{-1},   Y = M L^{-1},
// M = Phi(L^T Lbar) (Phi: the lower triangle with its diagonal halved); in
// lower-parameter form P_kk = tril(S) - diag(S) / 2, so Q_kk = S, and the
// output over Lbar_kk is tril(S) / 2.
// This is the panel recursion of the tile's adjoint summed in closed form
// (the same linear map; only the rounding differs), and it turns the long
// chain of 16-column panels into three products over TCHOL_PRB-order blocks
// that many workgroups share:
//   PADJM: Mn = -M by lower blocks, from LT (L^T) and Lbar_kk^T (which
//          DRED(k) leaves in the Q_kk tile)
//   PADJY: Y^T = L^{-T} Mn^T negated, i.e. (M L^{-1})^T, by upper blocks
//   PADJS: S by lower blocks, stored to Q_kk in both orientations and,
//          halved, to the lower triangle of Lbar_kk
// L^{-T} comes from TRTRI(k) (upper triangular, exact zeros below).  Every
// product is C = -A B^T from a zero start (the matrix cores' primitive);
// the negated M absorbs the first sign, the second cancels it, and the
// third is undone at the store.  Zero regions: the products' K ranges
// skip the blocks that vanish by triangularity, and inside the diagonal
// blocks the stored zeros (of Mn above its diagonal, of L^{-T} below, of
// Lbar^T below) make the rest exact.
#define PRB TCHOL_PRB

// C = -(A0 B0^T [+ A1 B1^T]) for one PRB x PRB block (M, N <= PRB, K a multiple
// of 16; the A panels at ld, the B panels at ldb, default ld); with Cinit the
// products are subtracted from C (read at ldc) instead of from zero.
// epi(row, col, value) stores each entry.  SEG as for gemm_core (128 needs
// even leading dimensions and 16-byte aligned panels).
template <int SEG = 128, class Epi>
__device__ __forceinline__ void padj_block(const double* A0, const double* B0, const double* A1, const double* B1,
                                           int64_t ld, int M, int N, int K, double* lds, Epi epi, int64_t ldb = -1,
                                           const double* Cinit = nullptr, int64_t ldc = 0) {
  using S = GemmShape<PRB, PRB, 16, 2, 4, 0>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / S::WGN, wn = wave % S::WGN;
  const int l16 = lane & 15, lg = lane >> 4;
  d4 acc[S::RB][S::CB];
#pragma unroll
  for (int rb = 0; rb < S::RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < S::CB; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * S::WTM + rb * 16 + l16, col = wn * S::WTN + cb * 16 + 4 * i + lg;
        acc[rb][cb][i] = Cinit ? Cinit[(int64_t)imin(col, N - 1) * ldc + imin(row, M - 1)] : 0.0;
      }
  gemm_kloop<PRB, PRB, 16, 2, 4, 0, SEG>(acc, A0, B0, ld, M, N, K, lds, ldb);
  if (A1 != nullptr) {
    __syncthreads();  // the stages are refilled only after every wavefront's last reads
    gemm_kloop<PRB, PRB, 16, 2, 4, 0, SEG>(acc, A1, B1, ld, M, N, K, lds, ldb);
  }
  __syncthreads();
#pragma unroll
  for (int rb = 0; rb < S::RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < S::CB; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * S::WTM + rb * 16 + l16, col = wn * S::WTN + cb * 16 + 4 * i + lg;
        if (row < M && col < N) epi(row, col, acc[rb][cb][i]);
      }
}

// TREV(i, k) work item through the tile's explicit inverse: rows r0 ..
// r0 + M - 1 of P_ik = Lbar_ik L_kk^{-1}, with L_kk^{-T} (IT, ld nb, upper
// triangular) from TRTRI(k).  Lb: those rows of Lbar_ik (ld); P(:, c) reads
// the columns of Lbar from c on, so the column blocks go left to right and
// each is written (P / 2 over Lbar, P into Q_ik at Qik and P^T into Q_ki at
// Qki, both ld ldq) after its own product has read it.  SEG = 128 needs Lb
// 16-byte aligned with an even ld; 32 serves the rest.
template <int SEG>
__device__ __forceinline__ void trev_rows(double* __restrict__ Lb, int64_t ld, const double* __restrict__ IT, int64_t nb,
                                          int M, int m, double* __restrict__ Qik, double* __restrict__ Qki,
                                          int64_t ldq, double* lds) {
  for (int c0 = 0; c0 < m; c0 += PRB) {
    padj_block<SEG>(Lb + (int64_t)c0 * ld, IT + (int64_t)c0 * nb + c0, nullptr, nullptr, ld, M, imin(PRB, m - c0),
                    m - c0, lds,
                    [&](int r, int c, double v) __attribute__((always_inline)) {
                      const double p = -v;
                      st_dev(Lb + (int64_t)(c0 + c) * ld + r, 0.5 * p);
                      st_dev(Qik + (int64_t)(c0 + c) * ldq + r, p);
                      st_dev(Qki + (int64_t)r * ldq + c0 + c, p);
                    },
                    nb);
  }
}

// Block (bi, bj), bi >= bj, of the lower triangle from a work item's part.
__device__ __forceinline__ void lower_block(int part, int& bi, int& bj) {
  bi = 0;
  while ((bi + 1) * (bi + 2) / 2 <= part) ++bi;
  bj = part - bi * (bi + 1) / 2;
}

// One work item of PADJM / PADJY / PADJS on tile k of order m (a multiple of
// 16).  LTkk, Qkk: the tile of L^T and of Q (ld ldq); Bkk: Lbar_kk (ld);
// IT: L_kk^{-T}, Mn and YT: the tile's scratch blocks (ld nb).
__device__ __forceinline__ void padj_item(int kind, int part, int m, const double* __restrict__ LTkk,
                                          double* __restrict__ Qkk, int64_t ldq, double* __restrict__ Bkk, int64_t ld,
                                          const double* __restrict__ IT, double* __restrict__ Mn,
                                          double* __restrict__ YT, int64_t nb, double* lds) {
  int bi, bj;
  lower_block(part, bi, bj);
  const int i0 = bi * PRB, j0 = bj * PRB;
  const int Mi = imin(PRB, m - i0), Nj = imin(PRB, m - j0);
  if (kind == TK_PADJM) {
    // Mn(i, j) = -sum_{t >= i} L^T(i, t) Lbar^T(j, t), diagonal halved, zero above it
    padj_block(LTkk + (int64_t)i0 * ldq + i0, Qkk + (int64_t)i0 * ldq + j0, nullptr, nullptr, ldq, Mi, Nj, m - i0,
               lds, [&](int r, int c, double v) __attribute__((always_inline)) {
                 if (bi == bj) v = r > c ? v : (r == c ? 0.5 * v : 0.0);
                 st_dev(Mn + (int64_t)(j0 + c) * nb + i0 + r, v);
               });
  } else if (kind == TK_PADJY) {
    // Y^T(j, i) = -sum_{j <= t <= i} L^{-T}(j, t) Mn(i, t), the block of rows j0 and columns i0
    const int kend = imin(i0 + PRB, m);
    padj_block(IT + (int64_t)j0 * nb + j0, Mn + (int64_t)j0 * nb + i0, nullptr, nullptr, nb, Nj, Mi, kend - j0, lds,
               [&](int r, int c, double v) __attribute__((always_inline)) {
                 st_dev(YT + (int64_t)(i0 + c) * nb + j0 + r, v);
               });
  } else {
    // S(i, j) = sum_{t >= i} L^{-T}(i, t) Y^T(j, t) + Y^T(i, t) L^{-T}(j, t), lower entries
    padj_block(IT + (int64_t)i0 * nb + i0, YT + (int64_t)i0 * nb + j0, YT + (int64_t)i0 * nb + i0,
               IT + (int64_t)i0 * nb + j0, nb, Mi, Nj, m - i0, lds,
               [&](int r, int c, double v) __attribute__((always_inline)) {
                 const int i = i0 + r, j = j0 + c;
                 if (i >= j) {
                   const double s = -v;
                   st_dev(Qkk + (int64_t)j * ldq + i, s);
                   st_dev(Qkk + (int64_t)i * ldq + j, s);
                   st_dev(Bkk + (int64_t)j * ld + i, 0.5 * s);
                 }
               });
  }
}

// Adjoint preparation: LT := L^T over the padded order np (LT(c, t) = L(t, c)
// at t * ldq + c, zero outside the lower triangle of the n x n factor), and
// the padding rows and columns of Q set to zero.  32 x 32 tiles through LDS.
__global__ void tchol_backward_prep(const double* __restrict__ L, int64_t n, double* __restrict__ LT,
                                    double* __restrict__ Q, int64_t ldq, int64_t np) {
  __shared__ double t32[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
  const int64_t c0 = (int64_t)blockIdx.x * 32, t0 = (int64_t)blockIdx.y * 32;
  // read L(t0 + j, c0 + i) for i = row of the transposed tile: columns c of L, rows t contiguous
  for (int i = ty; i < 32; i += 8) {
    const int64_t c = c0 + i, t = t0 + tx;
    t32[i][tx] = (c < n && t < n && t >= c) ? L[c * n + t] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t t = t0 + j, c = c0 + tx;
    if (t < np && c < np) LT[t * ldq + c] = t32[tx][j];
  }
  // Q padding: rows or columns at or past n
  for (int j = ty; j < 32; j += 8) {
    const int64_t t = t0 + j, r = c0 + tx;
    if (t < np && r < np && (t >= n || r >= n)) Q[t * ldq + r] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// scheduler
__device__ __forceinline__ int ld_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t tile_size(int64_t n, int64_t nb, int t) {
  const int64_t r = n - (int64_t)t * nb;
  return r < nb ? r : nb;
}

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Executed by a whole wavefront with every decision made wave-uniform
// (readfirstlane), so the compiler keeps the control flow scalar: a barrier
// must never end up inside lane-masked loop structure.  Waits until the
// task's counter reaches zero; false when the run is being aborted or the
// wait exceeded its bound.
__device__ __forceinline__ bool wait_ready(const KArgs& a, int task, int lane) {
  const int dep0 = ld_relaxed(&a.dep[task]), abort0 = ld_relaxed(&a.hdr[HDR_ABORT]);  // both in flight at once
  if (uniform_i(dep0) == 0) return uniform_i(abort0) == 0;
  const uint64_t t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(2);
    // the counter and the abort flag in flight together: one round trip per poll
    const int d = ld_relaxed(&a.dep[task]), ab = uniform_i(ld_relaxed(&a.hdr[HDR_ABORT]));
    if (uniform_i(d) == 0) return ab == 0;
    if (ab != 0) return false;
    if ((int64_t)(wall_clock64() - t0) > a.wait_limit) {
      if (lane == 0) {
        __hip_atomic_store(&a.hdr[HDR_ERROR], DEV_ERR_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.hdr[HDR_ABORT], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      return false;
    }
  }
}

// Stops every worker with a runtime error code (the first one is kept).
__device__ __forceinline__ void raise_error(const KArgs& a, int code) {
  if (threadIdx.x == 0) {
    int expected = 0;
    __hip_atomic_compare_exchange_strong(&a.hdr[HDR_ERROR], &expected, code, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&a.hdr[HDR_ABORT], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// POTRF split over several workgroups.  A diagonal tile of order m > 128 is
// factored as its own small tile Cholesky DAG over 128 x 128 sub-blocks
// (T2 = ceil(m / 128) per side):
//   P(b)        chol of sub-block (b, b)                  (potrf_small)
//   S(r, b, s)  32-row strip s of sub-block (r, b) := . L_bb^{-T}, r > b   (trsm_strip)
//   U(r, c, b)  sub-block (r, c) -= L_rb L_cb^T, r >= c > b  (SYRK / GEMM core)
// The POTRF task has several work items; each one that starts joins the
// tile's pool: the worker takes the next sub-unit from a counter in the
// workspace, waits for that unit's predecessors through per-sub-block
// counters, runs it through the same tile bodies as whole tasks and
// publishes it (write-through stores, then the counter), until no unit is
// left; then its work item is done.  Units are handed out in a topological order, so the oldest
// unfinished unit always has its predecessors finished or running, and a
// single work item drains the pool alone if no other joins: no workgroup
// ever waits for one that has not started.  Updates of a sub-block are
// applied in order of b, so the factor does not depend on which workgroup
// runs what.
#define PSB 128        // sub-block order
#define PL_NEXT 0      // next unit to hand out
#define PL_P 2         // + b: P(b) done
#define PL_S 8         // + 4 r + b: strips of S(r, b) done
#define PL_U 24        // + 4 r + c: updates applied to sub-block (r, c)

struct PoolUnit {
  int type, b, r, c, s;  // type 0: P(b); 1: S(r, b, s); 2: U(r, c, b); -1: none left
};

__device__ __forceinline__ int psb_size(int m, int i) { return imin(PSB, m - i * PSB); }
__device__ __forceinline__ int psb_strips(int m, int i) { return (psb_size(m, i) + TS - 1) / TS; }

// Unit u of the sub-DAG in claim order: step by step, P(b), then the strips
// of each sub-block row below it, then its updates column by column (the
// next diagonal sub-block's first: it leads to P(b + 1)).
__device__ __forceinline__ PoolUnit pool_unit(int m, int u) {
  const int T2 = (m + PSB - 1) / PSB;
  for (int b = 0; b < T2; ++b) {
    if (u == 0) return {0, b, b, b, 0};
    --u;
    for (int r = b + 1; r < T2; ++r) {
      const int ns = psb_strips(m, r);
      if (u < ns) return {1, b, r, b, u};
      u -= ns;
    }
    for (int c = b + 1; c < T2; ++c)
      for (int r = c; r < T2; ++r) {
        if (u == 0) return {2, b, r, c, 0};
        --u;
      }
  }
  return {-1, 0, 0, 0, 0};
}

// Wavefront 0: waits until pool[q0] >= v0, pool[q1] >= v1 and pool[q2] >= v2
// (agent-scope loads, s_sleep back-off); false on abort or when the wait
// exceeds its bound (which then raises TCHOL_E_TIMEOUT like a task wait).
__device__ __forceinline__ bool pool_wait(const KArgs& a, const int32_t* pool, int q0, int v0, int q1, int v1, int q2,
                                          int v2, int lane) {
  // the three counters and the abort flag in flight together: one round trip per poll
  int ab = 0;
  auto met = [&]() __attribute__((always_inline)) {
    const int x0 = ld_relaxed(pool + q0), x1 = ld_relaxed(pool + q1), x2 = ld_relaxed(pool + q2);
    ab = uniform_i(ld_relaxed(&a.hdr[HDR_ABORT]));
    return uniform_i((x0 >= v0) & (x1 >= v1) & (x2 >= v2)) != 0;
  };
  if (met()) return ab == 0;
  const uint64_t t0 = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(2);
    if (met()) return ab == 0;
    if (ab != 0) return false;
    if ((int64_t)(wall_clock64() - t0) > a.wait_limit) {
      if (lane == 0) {
        __hip_atomic_store(&a.hdr[HDR_ERROR], DEV_ERR_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.hdr[HDR_ABORT], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      return false;
    }
  }
}

// Wavefront 0: waits for the predecessors of pool unit pu of a tile of order m.
__device__ __forceinline__ bool pool_wait_unit(const KArgs& a, const int32_t* pool, int m, const PoolUnit& pu,
                                               int lane) {
  if (pu.type == 0)  // P(b): the diagonal sub-block has taken its b updates
    return pool_wait(a, pool, PL_U + 5 * pu.b, pu.b, PL_U + 5 * pu.b, pu.b, PL_U + 5 * pu.b, pu.b, lane);
  if (pu.type == 1)  // S(r, b, s): L_bb factored, sub-block (r, b) updated b times
    return pool_wait(a, pool, PL_P + pu.b, 1, PL_U + 4 * pu.r + pu.b, pu.b, PL_P + pu.b, 1, lane);
  // U(r, c, b): every strip of (r, b) and (c, b) solved, (r, c) updated b times
  return pool_wait(a, pool, PL_S + 4 * pu.r + pu.b, psb_strips(m, pu.r), PL_S + 4 * pu.c + pu.b,
                   psb_strips(m, pu.c), PL_U + 4 * pu.r + pu.c, pu.b, lane);
}

// SEG = 128: the launch guarantees even leading dimensions, 16-byte aligned
// matrices and, for odd orders, a leading dimension above the order, so
// every panel the updates stream is 16-byte transferable; SEG = 32 serves
// every other case.  One transfer width per kernel instance keeps the
// update loops free of per-item branches.
// MODE 4: the batched FP32 launch: the mixed-precision factor kinds and
// the solve kinds with substitution against the FP64 diagonal tiles (one
// solve of a few right-hand sides does not repay explicit inverses).
// MODE 0: FP64 factorization and solve.  MODE 1 / 2: the mixed-precision
// factorization / its solves: the matrix is the FP32 working copy (a.A points
// to it), factored with FP32 MFMA updates and FP64 diagonal tiles kept in
// a.D; solves run in FP64 reading L in FP32 off the diagonal and in FP64 on
// it.  MODE 5: the mixed-precision factorization with BF16 updates: as
// MODE 1, with the TRSM strips also storing their results as three BF16
// terms (a.H) and the GEMM items running on the BF16 matrix cores over them.
// A mixed launch runs only its own task kinds (keeping each instance small)
// and is always a 16-byte one.
template <int SEG, int MODE>
__global__ void __launch_bounds__(NT, MODE >= 6 ? 2 : 1) tchol_persistent(KArgs a) {
  constexpr bool MIXED = MODE == 1 || MODE == 2 || MODE == 4 || MODE == 5;
  constexpr bool FACTOR_KINDS = MODE == 0 || MODE == 1 || MODE == 4 || MODE == 5;
  constexpr bool SOLVE_KINDS = MODE == 0 || MODE == 2 || MODE == 4;
  constexpr bool ADJOINT_KINDS = MODE == 3;
  // The FP64 and mixed-precision factorizations split large POTRF tasks
  // over their work items (the tile's pool of sub-units; the mixed one on
  // its FP64 diagonal tile); the batched FP32 instance factors each diagonal
  // tile on one workgroup (only part 0 of a POTRF task works)
  constexpr bool POOLED = MODE == 0 || MODE == 1 || MODE == 5;
  // MODE 6 (batched systems of one tile each): the compact POTRF and tile
  // solves only, in half the LDS, two workgroups per compute unit; MODE 7 the
  // same with each system's matrix read from and L written to FP32 storage
  // (A32, the FP64 tile in A for the products and the solves)
  static_assert(FRB_COMPACT_DOUBLES <= PT_LDS_COMPACT, "compact LDS budget");
  constexpr bool COMPACT = MODE == 6 || MODE == 7;
  __shared__ double lds[COMPACT ? PT_LDS_COMPACT : LDS_DOUBLES];
  __shared__ int s_claim[4];
  __shared__ int32_t s_desc[DESC_WORDS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = uniform_i(tid >> 6);
  // wavefront 0's record of the work item it ran last, published at the
  // start of the next claim, and of the items this worker completed
  int p_task = -1, p_ticket = 0, p_parts = 0, p_e0 = 0, p_e1 = 0, ndone = 0;
  uint64_t p_end = 0;
  // wavefront 0: the POTRF pool this worker serves (pl_task < 0: none) and
  // the POTRF work item's record, published when the pool has run dry
  int pl_task = -1, pl_m = 0, pl_ticket = 0, pl_parts = 0, pl_e0 = 0, pl_e1 = 0;
  int32_t* pl_pool = nullptr;
  for (;;) {
    // publish + claim: wavefront 0 marks the previous item done and takes the
    // next ticket in the same round trip, then waits for the new task while
    // its descriptor is fetched.  A worker in a POTRF pool takes the pool's
    // next sub-unit instead, and returns to the tickets when none is left.
    if (wave == 0) {
      int task = -1, part = 0, unit = -1, t = 0;
      bool claimed = false;
      uint64_t tw = 0;
      if (POOLED && pl_task >= 0) {
        int u = 0;
        if (lane == 0) u = __hip_atomic_fetch_add(pl_pool + PL_NEXT, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        u = uniform_i(u);
        const PoolUnit pu = pool_unit(pl_m, u);
        if (pu.type >= 0) {
          claimed = true;
          task = pl_task;
          t = pl_ticket;
          unit = u;
          if (!pool_wait_unit(a, pl_pool, pl_m, pu, lane)) task = -1;
        } else {
          // the pool has run dry: this worker's POTRF work item is complete
          p_task = pl_task;
          p_ticket = pl_ticket;
          p_parts = pl_parts;
          p_e0 = pl_e0;
          p_e1 = pl_e1;
          if (a.trace) p_end = wall_clock64();
          pl_task = -1;
        }
      }
      if (!claimed) {
        int prev = 0;
        if (lane == 0) {
          if (p_task >= 0)
            prev = __hip_atomic_fetch_add(&a.done[p_task], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          t = __hip_atomic_fetch_add(&a.hdr[HDR_TICKET], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (p_task >= 0) {
          // the last work item of a task activates its successors
          if (uniform_i(prev) == p_parts - 1)
            for (int e = p_e0 + lane; e < p_e1; e += 64)
              __hip_atomic_fetch_sub(&a.dep[a.succ[e]], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ++ndone;
          if (a.trace && lane == 0) {
            a.trace[4 * (int64_t)p_ticket + 2] = p_end;
            a.trace[4 * (int64_t)p_ticket + 3] = (uint64_t)(uint32_t)p_task | ((uint64_t)(uint32_t)blockIdx.x << 32);
          }
          p_task = -1;
        }
        t = uniform_i(t);
        if (t < a.nitem) {
          task = uniform_i(a.items[2 * t]);
          part = uniform_i(a.items[2 * t + 1]);
          if (a.trace) tw = wall_clock64();
          const int dv = lane < DESC_WORDS ? a.desc[DESC_WORDS * (int64_t)task + lane] : 0;
          if (!wait_ready(a, task, lane)) task = -1;
          if (lane < DESC_WORDS) s_desc[lane] = dv;
          const int kd = uniform_i(__builtin_amdgcn_readlane(dv, 0)), pd = uniform_i(__builtin_amdgcn_readlane(dv, 4));
          if (POOLED && task >= 0 && kd == TK_POTRF && pd > 1) {
            // a work item of a split POTRF: join the tile's pool
            const int tkd = uniform_i(__builtin_amdgcn_readlane(dv, 3)), sd = uniform_i(__builtin_amdgcn_readlane(dv, 7));
            const int64_t* srd = a.sys + SYS_WORDS * (int64_t)sd;
            pl_task = task;
            pl_m = (int)tile_size(srd[2], srd[3], tkd);
            pl_pool = a.pool + POOL_WORDS * (srd[6] + tkd);
            pl_ticket = t;
            pl_parts = pd;
            pl_e0 = uniform_i(__builtin_amdgcn_readlane(dv, 5));
            pl_e1 = uniform_i(__builtin_amdgcn_readlane(dv, 6));
            int u = 0;
            if (lane == 0) u = __hip_atomic_fetch_add(pl_pool + PL_NEXT, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            u = uniform_i(u);
            const PoolUnit pu = pool_unit(pl_m, u);
            if (pu.type >= 0) {
              unit = u;
              if (!pool_wait_unit(a, pl_pool, pl_m, pu, lane)) task = -1;
            } else {
              unit = -2;  // the pool ran dry before this item started: nothing to do
              pl_task = -1;
            }
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (lane == 0) {
        s_claim[0] = task;
        s_claim[1] = part;
        s_claim[2] = t;
        s_claim[3] = unit;
        if (a.trace && task >= 0 && !claimed) {
          a.trace[4 * (int64_t)t + 0] = tw;
          a.trace[4 * (int64_t)t + 1] = wall_clock64();
        }
        // the completed-item count, added once per worker
        if (task < 0 && ndone > 0)
          __hip_atomic_fetch_add(&a.hdr[HDR_DONE], ndone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
    const int task = uniform_i(s_claim[0]), part = uniform_i(s_claim[1]), ticket = uniform_i(s_claim[2]);
    const int unit = uniform_i(s_claim[3]);
    if (task < 0) break;
    const int kind = uniform_i(s_desc[0]), ti = uniform_i(s_desc[1]), tj = uniform_i(s_desc[2]),
              tk = uniform_i(s_desc[3]);
    const int d_parts = uniform_i(s_desc[4]), d_e0 = uniform_i(s_desc[5]), d_e1 = uniform_i(s_desc[6]);
    // the task's system: base pointers, order, tile size, leading dimension
    const int sid = uniform_i(s_desc[7]);
    const int64_t* sr = a.sys + SYS_WORDS * (int64_t)sid;
    using E = typename std::conditional<MIXED, float, double>::type;
    E* const Abase = reinterpret_cast<E*>(a.A) + sr[0];
    double* const Bbase = a.B + sr[1];
    const int64_t sn = sr[2], nb = sr[3], ld = sr[4], ldb = sn;
    // mixed precision: the system's FP64 diagonal tiles and their inverses
    double* const Dsys = a.D + (MIXED ? sr[5] : 0);
    double* const DinvSys = a.Dinv + sr[5];
    double* const DinvTSys = a.DinvT + sr[5];
    auto tsz = [&](int t) __attribute__((always_inline)) { return (int)tile_size(sn, nb, t); };
    // the solve's diagonal step on tile t applies explicit inverses (and keeps
    // y in the scratch vector): always in the mixed-precision solves; in the
    // FP64 solve of a launch that computes them (their tiles' orders are
    // multiples of 16), else substitution in place
    auto inv_tile = [&](int t) __attribute__((always_inline)) {
      return MODE == 2 || (MODE == 0 && a.inv != 0 && (tsz(t) & 15) == 0);
    };
    // in a batched launch a system whose factorization failed only passes
    // its remaining tasks on, so that the DAG drains
    const bool skip = a.batched && uniform_i(ld_relaxed(&a.sinfo[sid])) != 0;
    int ok = 1;
    // A unit of a POTRF pool runs the POTRF, TRSM or GEMM body on sub-blocks
    // of the diagonal tile (tk, tk): po_* give the sub-block offsets (rows,
    // columns, panel columns) and sizes; whole tasks take the tile's.
    int body = kind;
    int po_r = 0, po_c = 0, po_k = 0, po_m = 0, po_n = 0, po_kk = 0, po_s = 0;
    PoolUnit pu = {-1, 0, 0, 0, 0};
    if (POOLED && unit >= 0) {
      const int m = tsz(tk);
      pu = pool_unit(m, unit);
      body = pu.type == 0 ? TK_POTRF : (pu.type == 1 ? TK_TRSM : TK_GEMM);
      po_r = pu.r * PSB;
      po_c = pu.c * PSB;
      po_k = pu.b * PSB;
      po_m = psb_size(m, pu.r);
      po_n = psb_size(m, pu.c);
      po_kk = psb_size(m, pu.b);
      po_s = pu.s;
    } else if (POOLED && unit == -2) {
      body = -1;
    }
    if constexpr (COMPACT) {
      const bool fuse_fwd = a.nrhs > 0 && a.nrhs <= PT_FWD;
      if (skip) {
      } else if (kind == TK_POTRF) {
        // up to PT_FWD right-hand sides: the forward solve rides along (its FTRSV task only passes the completion on)
        // MODE 7: the system's FP32 matrix at A32 + sr[5], leading dimension sr[7]
        const int info = uniform_i(potrf_tile<SEG, 128, MODE == 7>(
            Abase + (tk * nb) * ld + tk * nb, ld, tsz(tk), lds, fuse_fwd ? Bbase + tk * nb : nullptr, ldb,
            (int)a.nrhs, MODE == 7 ? a.A32 + sr[5] + (tk * nb) * sr[7] + tk * nb : nullptr, sr[7]));
        if (info != 0 && tid == 0)
          __hip_atomic_store(&a.sinfo[sid], (int)(tk * nb) + info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (kind == TK_BTRSV || (kind == TK_FTRSV && !fuse_fwd)) {
        tile_solve<true>(Abase + (tk * nb) * ld + tk * nb, ld, Bbase + tk * nb, ldb, tsz(tk), (int)a.nrhs,
                         kind == TK_BTRSV, lds);
      } else if (kind != TK_FTRSV) {
        ok = 0;
      }
    } else switch (skip ? -1 : body) {
      case -1:
        break;
      case TK_POTRF: {
        if constexpr (!FACTOR_KINDS) {
          ok = 0;
          break;
        }
        // tiles of order <= 128 are factored by one workgroup in LDS; larger
        // ones through the tile's pool of sub-units when the task has several
        // work items (the plan's choice), else by the one-workgroup kernel
        int info;
        if constexpr (MIXED) {
          double* const Dk = Dsys + (int64_t)tk * nb * nb;
          if (POOLED && unit >= 0) {
            // P(b) on the FP64 diagonal tile; the last one pads a ragged tile
            // to a multiple of 16 with the identity (for its inverse)
            info = uniform_i(potrf_small(Dk + (int64_t)po_k * nb + po_k, nb, po_m, lds));
            if (info != 0) {
              info += po_k;
            } else if (po_k + po_m == tsz(tk)) {
              const int m = tsz(tk), mpad = (m + 15) & ~15;
              for (int idx = tid; idx < mpad * mpad; idx += NT) {
                const int c = idx / mpad, r = idx - c * mpad;
                if (r >= c && (r >= m || c >= m)) st_dev(Dk + (int64_t)c * nb + r, r == c ? 1.0 : 0.0);
              }
            }
          } else {
            if (part > 0) break;  // one workgroup factors the tile
            info = uniform_i(potrf_tile_mixed(Dk, nb, tsz(tk), lds));
          }
        } else {
          const bool sub = unit >= 0;
          const int m = sub ? po_m : tsz(tk);
          E* Akk = Abase + (tk * nb + po_k) * ld + tk * nb + po_k;
          if (m <= PSB)
            info = uniform_i(potrf_small(Akk, ld, m, lds));
          else
            info = uniform_i(potrf_tile<SEG>(Akk, ld, m, lds));
          if (info != 0) info += po_k;
        }
        if (info != 0 && tid == 0) {
          if (a.batched) {
            __hip_atomic_store(&a.sinfo[sid], (int)(tk * nb) + info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } else {
            __hip_atomic_store(&a.hdr[HDR_INFO], (int)(tk * nb) + info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.hdr[HDR_ABORT], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
        if (info != 0 && !a.batched) ok = 0;
        break;
      }
      case TK_TRSM: {
        if constexpr (!FACTOR_KINDS) {
          ok = 0;
          break;
        }
        if constexpr (MIXED) {
          double* const Dk = Dsys + (int64_t)tk * nb * nb;
          if (POOLED && unit >= 0) {
            // strip of sub-block (r, b) of the FP64 diagonal tile
            const int r0 = po_s * TS;
            trsm_strip(Dk + (int64_t)po_k * nb + po_r + r0, nb, Dk + (int64_t)po_k * nb + po_k, nb,
                       imin(TS, po_m - r0), po_kk, lds);
          } else {
            const int r0 = part * a.trsm_rows;
            const int S = imin(a.trsm_rows, tsz(ti) - r0);
            if constexpr (MODE == 5)  // the strip also as BF16 terms, for the BF16 updates
              trsm_strip(Abase + (tk * nb) * ld + ti * nb + r0, ld, Dk, nb, S, tsz(tk), lds, nullptr, 0,
                         a.H + ((int64_t)tk * a.hrows + (int64_t)ti * nb + r0) * nb, nb, (int64_t)a.T * a.hrows * nb);
            else
              trsm_strip(Abase + (tk * nb) * ld + ti * nb + r0, ld, Dk, nb, S, tsz(tk), lds);
          }
        } else if (a.inv != 0 && unit < 0) {
          // a 128-row block of A_ik through L_kk^{-1} (the launch's TRTRI(k))
          const int r0 = part * GB;
          trsm_inv_rows<SEG>(Abase + (tk * nb) * ld + ti * nb + r0, ld, DinvSys + (int64_t)tk * nb * nb, nb,
                             imin(GB, tsz(ti) - r0), tsz(tk), lds);
        } else {
          // a strip of A_ik, or of sub-block (r, b) of the diagonal tile for a pool unit
          const bool sub = unit >= 0;
          const int rs = sub ? TS : a.trsm_rows;
          const int r0 = (sub ? po_s : part) * rs;
          const int64_t row0 = sub ? (int64_t)tk * nb + po_r + r0 : (int64_t)ti * nb + r0;
          const int S = imin(rs, (sub ? po_m : tsz(ti)) - r0);
          const int64_t col0 = (int64_t)tk * nb + po_k;
          trsm_strip(Abase + col0 * ld + row0, ld, Abase + col0 * ld + col0, ld, S, sub ? po_kk : tsz(tk), lds);
        }
        break;
      }
      case TK_SYRK:
      case TK_GEMM:
      case TK_GEMM2: {
        if constexpr (!FACTOR_KINDS) {
          ok = 0;
          break;
        }
        // the work item's output sub-tile: row block si of bm rows, column block sj of bn
        int si, sj, bm, bn;
        if (kind == TK_SYRK) {
          si = 0;
          while ((si + 1) * (si + 2) / 2 <= part) ++si;
          sj = part - si * (si + 1) / 2;
          bm = bn = a.syrk_b;
        } else {
          const int ncj = (tsz(tj) + a.gemm_n - 1) / a.gemm_n;
          si = part / ncj;
          sj = part % ncj;
          bm = a.gemm_m;
          bn = a.gemm_n;
        }
        int M = imin(bm, tsz(ti) - si * bm);
        int N = imin(bn, tsz(tj) - sj * bn);
        // a double update streams the panel columns of steps k and k + 1,
        // which are adjacent in the matrix: one product with K = 2 nb
        int K = kind == TK_GEMM2 ? tsz(tk) + tsz(tk + 1) : tsz(tk);
        bool lower = kind == TK_SYRK && si == sj;
        int64_t crow = (int64_t)ti * nb + si * bm, ccol = (int64_t)tj * nb + sj * bn, kcol = (int64_t)tk * nb;
        int64_t brow = (int64_t)tj * nb + sj * bn;
        if (POOLED && unit >= 0) {
          // sub-block (r, c) of the diagonal tile -= L_rb L_cb^T
          M = po_m;
          N = po_n;
          K = po_kk;
          lower = po_r == po_c;
          crow = (int64_t)tk * nb + po_r;
          ccol = (int64_t)tk * nb + po_c;
          kcol = (int64_t)tk * nb + po_k;
          brow = ccol;
        }
        E* C = Abase + ccol * ld + crow;
        const E* Ap = Abase + kcol * ld + crow;
        const E* Bp = Abase + kcol * ld + brow;
        const bool misaligned = ((reinterpret_cast<uintptr_t>(Ap) | reinterpret_cast<uintptr_t>(Bp)) & 15) != 0;
        if constexpr (MIXED) {
          if (POOLED && unit >= 0) {
            // sub-block (r, c) of the FP64 diagonal tile -= L_rb L_cb^T, in FP64
            double* const Dk = Dsys + (int64_t)tk * nb * nb;
            gemm_nt<128>(Dk + (int64_t)po_c * nb + po_r, Dk + (int64_t)po_k * nb + po_r,
                         Dk + (int64_t)po_k * nb + po_c, nb, M, N, K, lower, lds);
            break;
          }
          // four rows per 16-byte lane: ld a multiple of 4 and three rows after the order
          if ((((int)ld & 3) != 0) || ld < sn + 3 || misaligned) {
            raise_error(a, DEV_ERR_LAYOUT);  // unreachable when the host honours the launch contract
            ok = 0;
            break;
          }
          if (kind == TK_SYRK)
            gemm_nt_f32_d(Dsys + (int64_t)ti * nb * nb + (int64_t)(sj * bn) * nb + si * bm, nb, Ap, Bp, ld, M, N,
                          tsz(tk), si == sj, lds);
          else if (MODE == 5 && bm == 256 && bn == 128 && tsz(tk) % 32 == 0)
            gemm_bf16x6_wide(C, ld, a.H + ((int64_t)tk * a.hrows + crow) * nb, a.H + ((int64_t)tk * a.hrows + brow) * nb,
                             nb, (int64_t)a.T * a.hrows * nb, a.hrows * nb, (int)nb, M, N, K, lds);
          else if (bm == 256 && bn == 128 && tsz(tk) % 32 == 0)
            gemm_f32_wide<32, 3>(C, Ap, Bp, ld, M, N, K, lds);
          else  // 128-row products (a 256-row item whose K is not a multiple of 32 takes two)
            for (int r0 = 0; r0 < M; r0 += 128)
              gemm_nt_f32(C + r0, Ap + r0, Bp, ld, imin(128, M - r0), N, K, false, lds);
        } else {
          if (SEG == 128 && (((int)ld & 1) != 0 || (((M | N) & 1) != 0 && ld <= sn) || misaligned)) {
            raise_error(a, DEV_ERR_LAYOUT);  // unreachable when the host honours the launch contract
            ok = 0;
            break;
          }
          gemm_nt<SEG>(C, Ap, Bp, ld, M, N, K, lower, lds);
        }
        break;
      }
      case TK_FTRSV:
      case TK_BTRSV:
        if constexpr (!SOLVE_KINDS) {
          ok = 0;
        } else if constexpr (MODE == 4) {
          // batched FP32 systems: substitution against the FP64 diagonal tile, in place
          tile_solve(Dsys + (int64_t)tk * nb * nb, nb, Bbase + tk * nb, ldb, tsz(tk), (int)a.nrhs, kind == TK_BTRSV,
                     lds);
        } else if (inv_tile(tk)) {
          // explicit inverses, by row strips: forward y_k := L_kk^{-1} b_k into
          // the scratch vector (its rows r0.. need columns up to r0 + rows), backward
          // x_k := L_kk^{-T} y_k back into B (rows r0.. need columns from r0)
          const int m = tsz(tk);
          const int r0 = part * a.gemv_rows;
          const int rows = imin(a.gemv_rows, m - r0);
          double* const Sbase = a.S + sr[1];
          if (kind == TK_FTRSV && MODE == 0)  // L_kk^{-1} = (L_kk^{-T})^T: rows of it are columns of DinvT
            gemv_strip<double, true, true>(DinvTSys + (int64_t)tk * nb * nb + (int64_t)r0 * nb, nb,
                                           Sbase + tk * nb + r0, Bbase + tk * nb, ldb, rows, 0, imin(m, r0 + rows),
                                           (int)a.nrhs, lds);
          else if (kind == TK_FTRSV)
            gemv_strip<double, false, true>(DinvSys + (int64_t)tk * nb * nb + r0, nb, Sbase + tk * nb + r0,
                                            Bbase + tk * nb, ldb, rows, 0, imin(m, r0 + rows), (int)a.nrhs, lds);
          else
            gemv_strip<double, false, true>(DinvTSys + (int64_t)tk * nb * nb + r0, nb, Bbase + tk * nb + r0,
                                            Sbase + tk * nb, ldb, rows, r0, m, (int)a.nrhs, lds);
        } else if constexpr (MODE == 0) {
          // substitution against L_kk, in place (batched systems; an order not a multiple of 16)
          tile_solve(Abase + (tk * nb) * ld + tk * nb, ld, Bbase + tk * nb, ldb, tsz(tk), (int)a.nrhs,
                     kind == TK_BTRSV, lds);
        } else {
          ok = 0;
        }
        break;
      case TK_FGEMV: {
        if constexpr (!SOLVE_KINDS) {
          ok = 0;
          break;
        }
        const int r0 = part * a.gemv_rows;
        const int rows = imin(a.gemv_rows, tsz(ti) - r0);
        // y_k is in the scratch vector when the diagonal step applied an inverse
        const double* Yk = inv_tile(tk) ? a.S + sr[1] + tk * nb : Bbase + tk * nb;
        gemv_strip<E, false, false>(Abase + (tk * nb) * ld + ti * nb + r0, ld, Bbase + ti * nb + r0, Yk, ldb, rows,
                                    0, tsz(tk), (int)a.nrhs, lds);
        break;
      }
      case TK_BGEMV: {
        if constexpr (!SOLVE_KINDS) {
          ok = 0;
          break;
        }
        const int c0 = part * a.gemv_rows;
        const int cols = imin(a.gemv_rows, tsz(ti) - c0);
        double* Yi = inv_tile(ti) ? a.S + sr[1] + ti * nb + c0 : Bbase + ti * nb + c0;
        gemv_strip<E, true, false>(Abase + (ti * nb + c0) * ld + tk * nb, ld, Yi, Bbase + tk * nb, ldb, cols, 0,
                                   tsz(tk), (int)a.nrhs, lds);
        break;
      }
      case TK_TRTRI: {
        if constexpr (MODE != 0 && MODE != 1 && MODE != 3 && MODE != 5) {
          ok = 0;
        } else {
          // L_kk^{-T} by 32-row strips: identity rows solved in place (into DinvT, ld nb).
          // The mixed-precision factorization reads its FP64 diagonal tile,
          // identity-padded when ragged, and also stores the transposes as
          // L_kk^{-1} (Dinv); the FP64 launches read L_kk in A (its order is
          // then a multiple of 16) and keep L_kk^{-1} as well (for the TRSM
          // items), the adjoint L_kk^{-T} only.
          const int mpad = (tsz(tk) + 15) & ~15;
          const int r0 = part * a.trsm_rows;
          const int S = imin(a.trsm_rows, mpad - r0);
          double* X = DinvTSys + (int64_t)tk * nb * nb + r0;
          for (int idx = tid; idx < S * mpad; idx += NT) {
            const int c = idx / S, r = idx - c * S;
            st_dev(X + (int64_t)c * nb + r, (r0 + r == c) ? 1.0 : 0.0);
          }
          wait_vmcnt<0>();
          __syncthreads();
          if constexpr (MODE == 0)  // with L_kk^{-1} too (Dinv), which the TRSM items apply
            trsm_strip<double, 2>(X, nb, Abase + (tk * nb) * ld + tk * nb, ld, S, mpad, lds,
                                  DinvSys + (int64_t)tk * nb * nb + (int64_t)r0 * nb, nb);
          else if constexpr (MODE == 3)  // the adjoint: L (its A) is the factor
            trsm_strip<double>(X, nb, Abase + (tk * nb) * ld + tk * nb, ld, S, mpad, lds);
          else
            trsm_strip<double, 2>(X, nb, Dsys + (int64_t)tk * nb * nb, nb, S, mpad, lds,
                                  DinvSys + (int64_t)tk * nb * nb + (int64_t)r0 * nb, nb);
        }
        break;
      }
      case TK_GREV:
      case TK_GREV2:
      case TK_TREV:
      case TK_DPART:
      case TK_DRED:
      case TK_PREV:
      case TK_PADJM:
      case TK_PADJY:
      case TK_PADJS: {
        if constexpr (!ADJOINT_KINDS) {
          ok = 0;
        } else {
          // A = L, B = Lbar (both at ld); Q and LT at ldq, zero past the order
          // (padded to a multiple of 16, so every K below is one)
          const int64_t ldq = a.ldq;
          const int T = (int)((sn + nb - 1) / nb);
          const int64_t np = (sn + 15) & ~(int64_t)15;
          if ((ldq & 1) != 0 || ldq < np) {
            raise_error(a, DEV_ERR_LAYOUT);  // unreachable when the host honours the launch contract
            ok = 0;
            break;
          }
          // partial-product slots, column k after column k - 1: S_ik at base(k) + i - k - 1
          auto slot = [&](int i, int k) __attribute__((always_inline)) {
            return (int64_t)k * (T - 1) - (int64_t)k * (k - 1) / 2 + (i - k - 1);
          };
          if (kind == TK_GREV) {
            // a single link (the last of its chain, on the critical path): 64 x 64 blocks
            const int ncj = (tsz(tk) + PRB - 1) / PRB;
            const int si = part / ncj, sj = part % ncj;
            const int M = imin(PRB, tsz(ti) - si * PRB), N = imin(PRB, tsz(tk) - sj * PRB);
            const int K = (int)(np - (int64_t)tj * nb < nb ? np - (int64_t)tj * nb : nb);
            double* C = Bbase + (tk * nb + sj * PRB) * ld + ti * nb + si * PRB;
            padj_block(a.Q + (tj * nb) * ldq + ti * nb + si * PRB, a.LT + (tj * nb) * ldq + tk * nb + sj * PRB, nullptr,
                       nullptr, ldq, M, N, K, lds,
                       [&](int r, int c, double v) __attribute__((always_inline)) {
                         st_dev(C + (int64_t)c * ld + r, v);
                       },
                       -1, C, ld);
          } else if (kind == TK_GREV2) {
            // the links j = tj and tj + 1 as one product over their
            // consecutive columns of Q and L^T (K = 2 nb, less at the padded end)
            const int ncj = (tsz(tk) + a.gemm_n - 1) / a.gemm_n;
            const int si = part / ncj, sj = part % ncj;
            const int M = imin(a.gemm_m, tsz(ti) - si * a.gemm_m);
            const int N = imin(a.gemm_n, tsz(tk) - sj * a.gemm_n);
            const int64_t kw = 2 * nb;
            const int K = (int)(np - (int64_t)tj * nb < kw ? np - (int64_t)tj * nb : kw);
            gemm_nt_ex(Bbase + (tk * nb + sj * a.gemm_n) * ld + ti * nb + si * a.gemm_m, ld,
                       a.Q + (tj * nb) * ldq + ti * nb + si * a.gemm_m, a.LT + (tj * nb) * ldq + tk * nb + sj * a.gemm_n,
                       ldq, M, N, K, false, false, lds);
          } else if (kind == TK_TREV) {
            // 64-row blocks of P_ik through L_kk^{-T} from TRTRI(k) (tile k is
            // never the ragged last one, so its order is a multiple of 16)
            const int r0 = part * PRB;
            double* Lb = Bbase + (tk * nb) * ld + ti * nb + r0;
            const int M = imin(PRB, tsz(ti) - r0);
            double* Qik = a.Q + (tk * nb) * ldq + ti * nb + r0;
            double* Qki = a.Q + (ti * nb + r0) * ldq + tk * nb;
            const double* IT = DinvTSys + (int64_t)tk * nb * nb;
            if ((ld & 1) == 0 && (reinterpret_cast<uintptr_t>(Bbase) & 15) == 0)
              trev_rows<128>(Lb, ld, IT, nb, M, tsz(tk), Qik, Qki, ldq, lds);
            else
              trev_rows<32>(Lb, ld, IT, nb, M, tsz(tk), Qik, Qki, ldq, lds);
          } else if (kind == TK_DPART) {
            // 64 x 64 block (bi, bj) of the lower triangle of the slot, -(P_ik^T L_ik)
            int bi, bj;
            lower_block(part, bi, bj);
            const int M = imin(PRB, tsz(tk) - bi * PRB), N = imin(PRB, tsz(tk) - bj * PRB);
            const int K = (int)(np - (int64_t)ti * nb < nb ? np - (int64_t)ti * nb : nb);
            double* Sk = a.D + slot(ti, tk) * nb * nb + (int64_t)(bj * PRB) * nb + bi * PRB;
            padj_block(a.Q + (ti * nb) * ldq + tk * nb + bi * PRB, a.LT + (ti * nb) * ldq + tk * nb + bj * PRB, nullptr,
                       nullptr, ldq, M, N, K, lds, [&](int r, int c, double v) __attribute__((always_inline)) {
                         if (bi != bj || r >= c) st_dev(Sk + (int64_t)c * nb + r, v);
                       });
          } else if (kind == TK_DRED) {
            // a tile whose order is a multiple of 16 takes the closed-form adjoint,
            // which reads Lbar_kk^T from the Q_kk tile
            const bool closed = (tsz(tk) & 15) == 0;
            dred_strip(Bbase + (tk * nb) * ld + tk * nb, ld, a.D + slot(tk + 1, tk) * nb * nb, nb * nb, T - 1 - tk, nb,
                       tsz(tk), part * 16, closed ? a.Q + (tk * nb) * ldq + tk * nb : nullptr, ldq);
          } else if (kind != TK_PREV) {
            // the closed-form tile adjoint: L_kk^{-T} in DinvT, two scratch
            // blocks (Mn, Y^T) per diagonal tile in Dinv
            const int64_t nb2 = nb * nb;
            padj_item(kind, part, tsz(tk), a.LT + (tk * nb) * ldq + tk * nb, a.Q + (tk * nb) * ldq + tk * nb, ldq,
                      Bbase + (tk * nb) * ld + tk * nb, ld, DinvTSys + tk * nb2, DinvSys + 2 * tk * nb2,
                      DinvSys + (2 * tk + 1) * nb2, nb, lds);
          } else {
            // the partial products were applied by DRED(k)
            prev_tile(Abase + (tk * nb) * ld + tk * nb, a.LT + (tk * nb) * ldq + tk * nb,
                      Bbase + (tk * nb) * ld + tk * nb, ld, a.Q + (tk * nb) * ldq + tk * nb, ldq, tsz(tk), a.D,
                      nb * nb, 0, nb, lds);
          }
        }
        break;
      }
      default:
        ok = 0;
        break;
    }
    // Publish.  Every global store of a work item is a device-scope store
    // (st_dev), written through to the device's point of coherence; once
    // each wavefront has seen its stores complete (vmcnt 0) the item's
    // results are visible to any CU that invalidates its caches before
    // reading them (the acquire after each wait).  This replaces an
    // agent-scope release fence, whose L2 write-back costs tens of
    // microseconds per work item on this part.  The completion counter is
    // incremented at the start of the next claim.
    wait_vmcnt<0>();
    __syncthreads();
    if (POOLED && unit >= 0) {
      // a pool unit: its sub-block counter tells the units that wait for it
      if (tid == 0) {
        const int ctr = pu.type == 0 ? PL_P + pu.b : (pu.type == 1 ? PL_S + 4 * pu.r + pu.b : PL_U + 4 * pu.r + pu.c);
        __hip_atomic_fetch_add(a.pool + POOL_WORDS * (sr[6] + tk) + ctr, 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
    } else if (wave == 0) {
      p_task = ok ? task : -1;
      p_ticket = ticket;
      p_parts = d_parts;
      p_e0 = d_e0;
      p_e1 = d_e1;
      if (a.trace) p_end = wall_clock64();
    }
  }
}

// Clears the header and the per-task completion counters and copies the
// initial dependency counters; the plan's constant part is copied by the host.
__global__ void tchol_reset(int32_t* hdr, int32_t* dep, int32_t* done, const int32_t* dep0, int32_t ntask,
                            int32_t* sinfo, int32_t nsys, int32_t* pool, int64_t npool) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < HDR_WORDS) hdr[i] = 0;
  if (i < ntask) {
    dep[i] = dep0[i];
    done[i] = 0;
  }
  if (i < nsys) sinfo[i] = 0;
  if (i < npool) pool[i] = 0;
}

// wide: every panel the launch streams is 16-byte transferable (even
// leading dimensions, 16-byte aligned matrices), decided by the host.
// npool: words of the POTRF pools (all zeroed by the reset kernel).
extern "C" hipError_t tchol_dev_launch(const KArgs* a, int32_t ntask, const int32_t* dep0, int64_t npool, int grid,
                                       int wide, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1) {
  const int rb = 256;
  int64_t cover = ntask > HDR_WORDS ? ntask : HDR_WORDS;
  if (a->nsys > cover) cover = a->nsys;
  if (npool > cover) cover = npool;
  hipLaunchKernelGGL(tchol_reset, dim3((unsigned)((cover + rb - 1) / rb)), dim3(rb), 0, stream, a->hdr, a->dep,
                     a->done, dep0, ntask, a->sinfo, a->nsys, a->pool, npool);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev0) {
    e = hipEventRecord(ev0, stream);
    if (e != hipSuccess) return e;
  }
  if (a->mixed == 5)
    hipLaunchKernelGGL((tchol_persistent<128, 5>), dim3(grid), dim3(NT), 0, stream, *a);
  else if (a->mixed == 4)
    hipLaunchKernelGGL((tchol_persistent<128, 4>), dim3(grid), dim3(NT), 0, stream, *a);
  else if (a->mixed == 3)
    hipLaunchKernelGGL((tchol_persistent<128, 3>), dim3(grid), dim3(NT), 0, stream, *a);
  else if (a->mixed == 1)
    hipLaunchKernelGGL((tchol_persistent<128, 1>), dim3(grid), dim3(NT), 0, stream, *a);
  else if (a->mixed == 2)
    hipLaunchKernelGGL((tchol_persistent<128, 2>), dim3(grid), dim3(NT), 0, stream, *a);
  else if (a->mixed == 6)
    hipLaunchKernelGGL((tchol_persistent<128, 6>), dim3(grid), dim3(NT), 0, stream, *a);
  else if (a->mixed == 7)
    hipLaunchKernelGGL((tchol_persistent<128, 7>), dim3(grid), dim3(NT), 0, stream, *a);
  else if (wide)
    hipLaunchKernelGGL((tchol_persistent<128, 0>), dim3(grid), dim3(NT), 0, stream, *a);
  else
    hipLaunchKernelGGL((tchol_persistent<32, 0>), dim3(grid), dim3(NT), 0, stream, *a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev1) e = hipEventRecord(ev1, stream);
  return e;
}

// The adjoint's preparation (LT and the padding of Q), before its persistent launch.
extern "C" hipError_t tchol_dev_backward_prep(const double* L, int64_t n, double* LT, double* Q, int64_t ldq,
                                              int64_t np, hipStream_t stream) {
  if (np == 0) return hipSuccess;
  const unsigned g = (unsigned)((np + 31) / 32);
  hipLaunchKernelGGL(tchol_backward_prep, dim3(g, g), dim3(256), 0, stream, L, n, LT, Q, ldq, np);
  return hipGetLastError();
}

// Workgroups of the compact instance (batched systems of one tile each) that
// the device holds at once.
extern "C" hipError_t tchol_dev_compact_grid(int device, int* grid) {
  int cus = 0, occ = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, tchol_persistent<128, 6>, NT, 0);
  if (e != hipSuccess) return e;
  int occ7 = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ7, tchol_persistent<128, 7>, NT, 0);
  if (e != hipSuccess) return e;
  occ = occ < occ7 ? occ : occ7;
  *grid = cus * (occ > 0 ? occ : 1);
  return hipSuccess;
}

extern "C" hipError_t tchol_dev_max_grid(int device, int* grid) {
  int cus = 0, occ = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  // both instances share the LDS size and launch bounds; take the smaller occupancy
  int occ32 = 0;
  int occm = 0, occs = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, tchol_persistent<128, 0>, NT, 0);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ32, tchol_persistent<32, 0>, NT, 0);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occm, tchol_persistent<128, 1>, NT, 0);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occs, tchol_persistent<128, 2>, NT, 0);
  if (e != hipSuccess) return e;
  int occa = 0, occb = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occa, tchol_persistent<128, 3>, NT, 0);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occb, tchol_persistent<128, 4>, NT, 0);
  if (e != hipSuccess) return e;
  int occf = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occf, tchol_persistent<128, 5>, NT, 0);
  if (e != hipSuccess) return e;
  occ = occ < occf ? occ : occf;
  occ = occ < occa ? occ : occa;
  occ = occ < occb ? occ : occb;
  occ = occ < occ32 ? occ : occ32;
  occ = occ < occm ? occ : occm;
  occ = occ < occs ? occ : occs;
  *grid = cus * (occ > 0 ? occ : 1);
  return hipSuccess;
}
