// Host planner for the tile DAGs run by the persistent kernel.
//
// Factorization (right-looking tile Cholesky of Buttari et al., the PLASMA
// DPOTRF the paper schedules, section 4.1 "Benchmarks"), T = ceil(n / nb):
//   POTRF(k)        preds: SYRK(k, k-1)                  succs: TRSM(i, k), i > k
//   TRSM(i, k)      preds: POTRF(k), GEMM(i, k, k-1)     succs: SYRK(i, k), GEMM(i, j, k) k<j<i,
//                                                               GEMM(m, i, k) m > i
//   SYRK(i, k)      preds: TRSM(i, k), SYRK(i, k-1)      succs: SYRK(i, k+1) or POTRF(i)
//   GEMM(i, j, k)   preds: TRSM(i,k), TRSM(j,k), GEMM(i,j,k-1)
//                                                        succs: GEMM(i, j, k+1) or TRSM(i, j)
// These edges are exactly the read-after-write and write-after-write
// conflicts on tiles that a data-flow runtime detects (section 2); the
// k-ascending chain of updates into each tile is kept, so every tile sees its
// updates in a fixed order and the result does not depend on the schedule.
//
// Solve L L^T X = B (B split into row blocks like the tiles of L):
//   FTRSV(k)        Y_k = L_kk^{-1} B_k       after FGEMV(k, k-1)
//   FGEMV(i, k)     B_i -= L_ik Y_k, i > k    after FTRSV(k), FGEMV(i, k-1)
//   BTRSV(k)        X_k = L_kk^{-T} Y_k       after FTRSV(T-1) (k = T-1) or BGEMV(k, k+1)
//   BGEMV(i, k)     Y_i -= L_ki^T X_k, i < k  after BTRSV(k), BGEMV(i, k+1)
// The diagonal steps either substitute against L_kk (one work item, in
// place) or apply the explicit inverses L_kk^{-1}, L_kk^{-T} by row strips
// (as many work items as the updates), with Y kept in a scratch vector.
// The FP64 solve computes those inverses itself:
//   TRTRI(k)        L_kk^{-1}, L_kk^{-T}      after POTRF(k) (merged launch)
// and FTRSV(k) then also waits for TRTRI(k).
//
// Batched plans hold several systems (each with its own order and tile
// size); each system's solve follows its factorization through the edges
// POTRF(k) -> FTRSV(k) and TRSM(i, k) -> FGEMV(i, k).
//
// Priority: the upward rank of HEFT (section 3.1): rank(t) = w(t) + max over
// successors s of rank(s), with w HEFT's computation cost of the task: the
// time of its work items summed over its parts, in units of about 200 us at
// nb = 512 on this part (POTRF 5, TRSM 10, SYRK 4, GEMM 6; TRSV 1, GEMV 2,
// and the solve's TRTRI as long as a TRSM, 10),
// and no communication term (one device).  Flop counts (1, 3, 3, 6) would
// undervalue POTRF and TRSM, whose tile kernels run far below the GEMM's
// efficiency, and start the critical path late.  Every weight is positive, so
// a task's rank exceeds each successor's and the decreasing-rank order is
// topological.
#include "plan.hpp"

#include <algorithm>
#include <queue>
#include <map>
#include <mutex>
#include <numeric>
#include <stdexcept>
#include <tuple>

#include "../../include/tchol.h"

namespace tchol {

namespace {

// Adds the tasks of one system to the plan (successor lists kept as
// vectors, indexed by global task id, turned into CSR afterwards).
struct Builder {
  Plan& p;
  const Split& s;
  std::vector<std::vector<int32_t>>& succ;
  int32_t sys;
  int64_t n, nb;
  int32_t T;
  Builder(Plan& plan, const Split& split, std::vector<std::vector<int32_t>>& succ_lists, int32_t system)
      : p(plan), s(split), succ(succ_lists), sys(system), n(plan.systems[system].n), nb(plan.systems[system].nb),
        T(plan.systems[system].T) {}

  int64_t tile_size(int32_t t) const { return std::min<int64_t>(nb, n - (int64_t)t * nb); }

  int32_t add(int32_t kind, int32_t i, int32_t j, int32_t k, int32_t parts) {
    p.kind.push_back(kind);
    p.ti.push_back(i);
    p.tj.push_back(j);
    p.tk.push_back(k);
    p.sys.push_back(sys);
    p.parts.push_back(parts);
    succ.emplace_back();
    return (int32_t)p.kind.size() - 1;
  }

  static int32_t cdiv(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }
};

// ids of one system's tasks, for the edges between its factor and solve DAGs
struct FactorIds {
  std::vector<int32_t> potrf, trsm;  // trsm[i * T + k]
  std::vector<int32_t> trtri;        // inverse-TRSM factorizations: TRTRI(k) for k < T-1, else -1
};

// The mixed-precision factorization (OP_FACTOR_INV) has its own costs: its
// GEMM items are FP32 products (256 x 128 sub-tiles), its TRTRI tasks as
// long as a TRSM: POTRF 5, TRSM 11, SYRK 4, GEMM 4, TRTRI 11.
int64_t weight(int32_t kind, int32_t op) {
  if (op == OP_FACTOR_INV) {
    switch (kind) {
      case TK_POTRF: return 5;
      case TK_TRSM: return 11;
      case TK_SYRK: return 4;
      case TK_GEMM: return 4;
      case TK_GEMM2: return 8;
      case TK_TRTRI: return 11;
      default: break;
    }
  }
  switch (kind) {
    case TK_POTRF: return 5;
    case TK_TRSM: return 10;
    case TK_SYRK: return 4;
    case TK_GEMM: return 6;
    case TK_GEMM2: return 12;
    case TK_FTRSV: case TK_BTRSV: return 1;
    case TK_GREV: return 6;
    case TK_TREV: return 3;
    case TK_DPART: return 3;
    case TK_PREV: return 4;
    case TK_TRTRI: return op == TCHOL_OP_BACKWARD ? 40 : 10;
    case TK_DRED: return 1;
    case TK_GREV2: return 11;
    case TK_PADJM: case TK_PADJY: return 1;
    case TK_PADJS: return 2;
    default: return 2;
  }
}

// Work items of the POTRF of a tile of order m in a system of several tiles
// (on the critical path of the tile DAG).  Tiles above 128 are factored as a
// small tile DAG over 128 x 128 sub-blocks whose sub-units the task's work
// items share (the kernel's POTRF pool); as many items as the widest step of
// that DAG offers (the strips of the sub-blocks below the first one), at
// most 8.  Smaller tiles take one work item.
int32_t potrf_parts(int64_t m) {
  if (m <= 128) return 1;
  int32_t strips = 0;
  for (int64_t r0 = 128; r0 < m; r0 += 128) strips += (int32_t)((std::min<int64_t>(128, m - r0) + 31) / 32);
  return std::min<int32_t>(8, strips);
}

// trtri: add TRTRI(k) after POTRF(k) (explicit inverses for the
// mixed-precision solve; no task of the factorization waits for them).
// inv_trsm: TRSM(i, k) applies L_kk^{-1} from TRTRI(k), which runs between
// POTRF(k) and the step's TRSMs (k < T-1: every tile with a TRSM below it is
// a full one), by 128-row blocks on the matrix cores.
void build_factor(Builder& b, FactorIds* ids = nullptr, bool trtri = false, bool inv_trsm = false) {
  auto& succ = b.succ;
  const int32_t T = b.T;
  std::vector<int32_t> id_potrf(T, -1), id_trsm((size_t)T * T, -1), id_syrk((size_t)T * T, -1);
  std::vector<int32_t> id_inv(T, -1);
  std::vector<int32_t> id_gemm((size_t)T * T * T, -1);
  auto ix2 = [T](int32_t i, int32_t k) { return (size_t)i * T + k; };
  auto ix3 = [T](int32_t i, int32_t j, int32_t k) { return ((size_t)k * T + i) * T + j; };
  // The updates of tile (i, j), k = 0 .. j-1, are chained in k.  Every pair
  // (k, k+1) with k even that does not contain the last update (k+1 <= j-2)
  // is one GEMM2 task (K = 2 nb: half the loads and stores of the tile, and
  // half the work items' fixed costs, for the same products in the same
  // order); the last update before TRSM(i, j) stays a single GEMM, so the
  // critical path does not wait for a double update.  id_gemm[(i, j, k)]
  // holds the task that applies update k (a GEMM2 under both of its k).
  auto pair_first = [](int32_t j, int32_t k) { return (k % 2 == 0) && (k + 1 <= j - 2); };
  auto pair_second = [](int32_t j, int32_t k) { return (k % 2 == 1) && (k <= j - 2); };
  auto gemm_parts = [&](int32_t i, int32_t j) {
    return Builder::cdiv(b.tile_size(i), b.s.gemm_m) * Builder::cdiv(b.tile_size(j), b.s.gemm_n);
  };
  for (int32_t k = 0; k < T; ++k) {
    // a single-tile system's POTRF is the whole factorization: in a batch of
    // many such systems the workgroups have independent work enough, so it
    // takes one work item unless the system asks for several (wgs, a tuning
    // choice: they share the tile's sub-block pool); the diagonal tiles of
    // tiled systems are split
    const int32_t wgs = b.p.systems[b.sys].wgs;
    id_potrf[k] = b.add(TK_POTRF, k, k, k,
                        T > 1 ? potrf_parts(b.tile_size(k))
                              : (wgs > 1 && b.tile_size(k) > 128 ? std::min(wgs, potrf_parts(b.tile_size(k))) : 1));
    if (inv_trsm && k + 1 < T) id_inv[k] = b.add(TK_TRTRI, k, k, k, Builder::cdiv(b.tile_size(k), b.s.trsm_rows));
    for (int32_t i = k + 1; i < T; ++i)
      id_trsm[ix2(i, k)] =
          b.add(TK_TRSM, i, k, k, Builder::cdiv(b.tile_size(i), inv_trsm ? b.s.gemm_m : b.s.trsm_rows));
    for (int32_t i = k + 1; i < T; ++i) {
      int32_t sb = Builder::cdiv(b.tile_size(i), b.s.syrk_b);
      id_syrk[ix2(i, k)] = b.add(TK_SYRK, i, i, k, sb * (sb + 1) / 2);
      for (int32_t j = k + 1; j < i; ++j) {
        if (pair_first(j, k)) continue;  // created with its second update, after TRSM(., k+1)
        const bool second = pair_second(j, k);
        const int32_t id = second ? b.add(TK_GEMM2, i, j, k - 1, gemm_parts(i, j))
                                  : b.add(TK_GEMM, i, j, k, gemm_parts(i, j));
        id_gemm[ix3(i, j, k)] = id;
        if (second) id_gemm[ix3(i, j, k - 1)] = id;
      }
    }
  }
  for (int32_t k = 0; k < T; ++k) {
    if (id_inv[k] >= 0) {
      succ[id_potrf[k]].push_back(id_inv[k]);
      for (int32_t i = k + 1; i < T; ++i) succ[id_inv[k]].push_back(id_trsm[ix2(i, k)]);
    } else {
      for (int32_t i = k + 1; i < T; ++i) succ[id_potrf[k]].push_back(id_trsm[ix2(i, k)]);
    }
    for (int32_t i = k + 1; i < T; ++i) {
      auto& st = succ[id_trsm[ix2(i, k)]];
      st.push_back(id_syrk[ix2(i, k)]);
      for (int32_t j = k + 1; j < i; ++j) st.push_back(id_gemm[ix3(i, j, k)]);
      for (int32_t m = i + 1; m < T; ++m) st.push_back(id_gemm[ix3(m, i, k)]);
      succ[id_syrk[ix2(i, k)]].push_back(k + 1 < i ? id_syrk[ix2(i, k + 1)] : id_potrf[i]);
      // each update task passes the tile on to the next one, the last to TRSM(i, j)
      for (int32_t j = k + 1; j < i; ++j) {
        if (pair_first(j, k)) continue;
        succ[id_gemm[ix3(i, j, k)]].push_back(k + 1 < j ? id_gemm[ix3(i, j, k + 1)] : id_trsm[ix2(i, j)]);
      }
    }
  }
  if (trtri)
    for (int32_t k = 0; k < T; ++k) {
      const int64_t mpad = (b.tile_size(k) + 15) / 16 * 16;
      // add() appends to succ, so take the id before indexing succ
      const int32_t id = b.add(TK_TRTRI, k, k, k, Builder::cdiv(mpad, b.s.trsm_rows));
      succ[id_potrf[k]].push_back(id);
    }
  if (ids) {
    ids->potrf = id_potrf;
    ids->trsm = id_trsm;
    ids->trtri = id_inv;
  }
}

// How the solve's diagonal steps run: substitution; explicit inverses that
// another launch computed (the mixed-precision solve, which pads ragged
// tiles); explicit inverses from this plan's own TRTRI tasks (the FP64 solve,
// for the tiles whose order is a multiple of 16; a ragged last tile keeps
// the substitution).
enum class Diag { kSubst, kInvGiven, kInvHere };

void build_solve(Builder& b, const FactorIds* after = nullptr, Diag diag = Diag::kSubst) {
  auto& succ = b.succ;
  const int32_t T = b.T;
  std::vector<int32_t> id_ft(T), id_bt(T), id_tri(T, -1), id_fg((size_t)T * T, -1), id_bg((size_t)T * T, -1);
  auto ix2 = [T](int32_t i, int32_t k) { return (size_t)i * T + k; };
  auto inv = [&](int32_t k) {
    return diag == Diag::kInvGiven || (diag == Diag::kInvHere && b.tile_size(k) % 16 == 0);
  };
  auto dparts = [&](int32_t k) { return inv(k) ? Builder::cdiv(b.tile_size(k), b.s.gemv_rows) : 1; };
  // the factorization's own inverses (inverse-TRSM factorizations) serve the solve as well
  auto given = [&](int32_t k) { return after && !after->trtri.empty() && after->trtri[k] >= 0; };
  for (int32_t k = 0; k < T; ++k) {
    if (diag == Diag::kInvHere && inv(k) && !given(k))
      id_tri[k] = b.add(TK_TRTRI, k, k, k, Builder::cdiv(b.tile_size(k), b.s.trsm_rows));
    id_ft[k] = b.add(TK_FTRSV, k, k, k, dparts(k));
    for (int32_t i = k + 1; i < T; ++i)
      id_fg[ix2(i, k)] = b.add(TK_FGEMV, i, k, k, Builder::cdiv(b.tile_size(i), b.s.gemv_rows));
  }
  for (int32_t k = T - 1; k >= 0; --k) {
    id_bt[k] = b.add(TK_BTRSV, k, k, k, dparts(k));
    for (int32_t i = 0; i < k; ++i)
      id_bg[ix2(i, k)] = b.add(TK_BGEMV, i, k, k, Builder::cdiv(b.tile_size(i), b.s.gemv_rows));
  }
  for (int32_t k = 0; k < T; ++k)
    if (id_tri[k] >= 0) succ[id_tri[k]].push_back(id_ft[k]);
  if (after) {
    // the solve of a system reads the final tiles of its factor
    for (int32_t k = 0; k < T; ++k) {
      if (given(k) && diag == Diag::kInvHere)
        succ[after->trtri[k]].push_back(id_ft[k]);
      else
        succ[after->potrf[k]].push_back(id_tri[k] >= 0 ? id_tri[k] : id_ft[k]);
      for (int32_t i = k + 1; i < T; ++i) succ[after->trsm[ix2(i, k)]].push_back(id_fg[ix2(i, k)]);
    }
  }
  for (int32_t k = 0; k < T; ++k) {
    for (int32_t i = k + 1; i < T; ++i) {
      succ[id_ft[k]].push_back(id_fg[ix2(i, k)]);
      succ[id_fg[ix2(i, k)]].push_back(k + 1 < i ? id_fg[ix2(i, k + 1)] : id_ft[i]);
    }
  }
  succ[id_ft[T - 1]].push_back(id_bt[T - 1]);
  for (int32_t k = T - 1; k >= 0; --k) {
    for (int32_t i = 0; i < k; ++i) {
      succ[id_bt[k]].push_back(id_bg[ix2(i, k)]);
      succ[id_bg[ix2(i, k)]].push_back(k - 1 > i ? id_bg[ix2(i, k - 1)] : id_bt[i]);
    }
  }
}

// Adjoint of the factorization: the reverse of the factor DAG, steps k
// from T-1 down to 0, in lower-parameter form (P: derivative with respect to
// the lower triangle of A; Q = P + P^T, whose tile Q_ij is P_ij, P_ji^T or
// P_ii + P_ii^T).  Reversing TRSM(i, k), SYRK(i, k) and GEMM(i, j, k) of the
// forward DAG gives, per step k,
//   GREV(i, k, j)  Lbar_ik -= Q_ij L_jk     i > k, j = T-1 down to k+1: a
//                  chain per (i, k) in a fixed order; after the task that
//                  produced Q_ij: TREV(i, j) (j < i), PREV(i) (j = i) or
//                  TREV(j, i) (j > i)
//   TREV(i, k)     P_ik = Lbar_ik L_kk^{-1}  after GREV(i, k, k+1) and TRTRI(k)
//                  (the product with the explicit inverse)
//   DPART(i, k)    S_ik = tril(P_ik^T L_ik)  after TREV(i, k)
//   DRED(k)        Lbar_kk -= sum_i S_ik (i ascending), by 16-row strips,
//                  after every DPART(i, k)   (k < T-1)
//   PREV(k)        the diagonal tile's adjoint, after DRED(k)
// The partial products S_ik give the diagonal tile's update one task per
// term instead of a chain of T - k - 1 dependent ones on the critical path,
// and their sum is spread over workgroups by row strips.
//
// A diagonal tile whose order is a multiple of 16 takes its adjoint in
// closed form instead of PREV(k): DRED(k) (then also for k = T-1) leaves
// Lbar_kk^T in the Q_kk tile, and
//   TRTRI(k)       L_kk^{-T}, no predecessors (L is an input); TREV(i, k) uses it too
//   PADJM(k)       M = Phi(L_kk^T Lbar_kk)         after DRED(k)
//   PADJY(k)       Y^T = (M L_kk^{-1})^T           after PADJM(k), TRTRI(k)
//   PADJS(k)       Q_kk = S, Lbar_kk = tril(S)/2   after PADJY(k)
// each over TCHOL_PRB x TCHOL_PRB blocks of the tile's lower (Y^T: upper)
// triangle, so that the chain of the diagonal tile runs on many workgroups.
bool closed_form_tile(int64_t m) { return m % 16 == 0; }

// GREV(i, k, j) and GREV(i, k, j - 1) form one task (TK_GREV2 at j - 1)
// when j is the upper link of a pair: the links j = T-1 .. k+2 are paired
// from the top, k+1 stays alone (and so does k+2 when their count is odd).
bool grev_paired(int32_t j, int32_t k, int32_t T) { return j - 1 >= k + 2 && (T - 1 - j) % 2 == 0; }

void build_backward(Builder& b) {
  auto& succ = b.succ;
  const int32_t T = b.T;
  std::vector<int32_t> id_prev(T), id_dred(T, -1), id_trev((size_t)T * T, -1), id_dpart((size_t)T * T, -1);
  std::vector<int32_t> id_grev((size_t)T * T * T, -1);
  std::vector<int32_t> id_inv(T, -1), id_pm(T, -1), id_py(T, -1);
  auto ix2 = [T](int32_t i, int32_t k) { return (size_t)i * T + k; };
  auto ix3 = [T](int32_t i, int32_t j, int32_t k) { return ((size_t)k * T + i) * T + j; };
  for (int32_t k = T - 1; k >= 0; --k) {
    const int64_t m = b.tile_size(k);
    // tasks are numbered so that every edge runs forward: L_kk^{-T} first,
    // as TREV(i, k) reads it
    if (closed_form_tile(m)) id_inv[k] = b.add(TK_TRTRI, k, k, k, Builder::cdiv(m, b.s.trsm_rows));
    // the chain into Lbar_ik: its last link (j = k + 1, which waits for the
    // most recent Q tile) alone, the links above it in pairs from the top
    // (one task of K = 2 nb: half the loads and stores of Lbar_ik)
    // the kinds on the critical path of a step (the last GREV link, TREV,
    // DPART) work on TCHOL_PRB-order blocks, so that many workgroups share
    // them; the paired links on 128 x 128 sub-tiles
    for (int32_t i = k + 1; i < T; ++i)
      for (int32_t j = T - 1; j > k; --j) {
        if (grev_paired(j, k, T)) {
          const int32_t parts =
              Builder::cdiv(b.tile_size(i), b.s.gemm_m) * Builder::cdiv(b.tile_size(k), b.s.gemm_n);
          id_grev[ix3(i, j, k)] = id_grev[ix3(i, j - 1, k)] = b.add(TK_GREV2, i, j - 1, k, parts);
          --j;
        } else {
          const int32_t parts =
              Builder::cdiv(b.tile_size(i), TCHOL_PRB) * Builder::cdiv(b.tile_size(k), TCHOL_PRB);
          id_grev[ix3(i, j, k)] = b.add(TK_GREV, i, j, k, parts);
        }
      }
    // TREV by row blocks through L_kk^{-T} (TRTRI(k); tile k is never the ragged last one)
    for (int32_t i = k + 1; i < T; ++i)
      id_trev[ix2(i, k)] = b.add(TK_TREV, i, k, k, Builder::cdiv(b.tile_size(i), TCHOL_PRB));
    const int32_t sb = Builder::cdiv(b.tile_size(k), TCHOL_PRB);
    for (int32_t i = k + 1; i < T; ++i) id_dpart[ix2(i, k)] = b.add(TK_DPART, i, k, k, sb * (sb + 1) / 2);
    if (closed_form_tile(m)) {
      const int32_t nbk = Builder::cdiv(m, TCHOL_PRB), blocks = nbk * (nbk + 1) / 2;
      id_dred[k] = b.add(TK_DRED, k, k, k, Builder::cdiv(m, 16));
      id_pm[k] = b.add(TK_PADJM, k, k, k, blocks);
      id_py[k] = b.add(TK_PADJY, k, k, k, blocks);
      id_prev[k] = b.add(TK_PADJS, k, k, k, blocks);  // the task that produces Q_kk
    } else {
      if (k + 1 < T) id_dred[k] = b.add(TK_DRED, k, k, k, Builder::cdiv(m, 16));
      id_prev[k] = b.add(TK_PREV, k, k, k, 1);
    }
  }
  auto producer = [&](int32_t i, int32_t j) {
    return j < i ? id_trev[ix2(i, j)] : (j == i ? id_prev[i] : id_trev[ix2(j, i)]);
  };
  for (int32_t k = T - 1; k >= 0; --k) {
    for (int32_t i = k + 1; i < T; ++i) {
      for (int32_t j = T - 1; j > k; --j) {
        const int32_t g = id_grev[ix3(i, j, k)];
        succ[producer(i, j)].push_back(g);
        if (j > k + 1 && id_grev[ix3(i, j - 1, k)] == g) continue;  // the pair's other link
        succ[g].push_back(j > k + 1 ? id_grev[ix3(i, j - 1, k)] : id_trev[ix2(i, k)]);
      }
      succ[id_trev[ix2(i, k)]].push_back(id_dpart[ix2(i, k)]);
      succ[id_dpart[ix2(i, k)]].push_back(id_dred[k]);
    }
    if (id_inv[k] >= 0)
      for (int32_t i = k + 1; i < T; ++i) succ[id_inv[k]].push_back(id_trev[ix2(i, k)]);
    if (id_pm[k] >= 0) {
      succ[id_dred[k]].push_back(id_pm[k]);
      succ[id_pm[k]].push_back(id_py[k]);
      succ[id_inv[k]].push_back(id_py[k]);
      succ[id_py[k]].push_back(id_prev[k]);
    } else if (id_dred[k] >= 0) {
      succ[id_dred[k]].push_back(id_prev[k]);
    }
  }
}

// tie-break key: (step, kind, i, j); the backward sweep of the solve comes
// after the forward one and runs k downwards.
std::tuple<int32_t, int32_t, int32_t, int32_t, int32_t> tie_key(const Plan& p, int32_t t) {
  const int32_t T = p.systems[p.sys[t]].T;
  int32_t kind = p.kind[t], step = p.tk[t];
  if (kind == TK_BTRSV || kind == TK_BGEMV) step = T + (T - 1 - p.tk[t]);
  if (p.op == TCHOL_OP_BATCHED && kind >= TK_FTRSV && kind <= TK_BGEMV) step += T;  // a system's solve after its factor
  const bool adjoint = p.op == TCHOL_OP_BACKWARD;
  if (adjoint) step = T - 1 - p.tk[t];  // the adjoint runs its steps downwards
  int32_t kord = kind;
  if (kind == TK_GEMM2) {  // a double update belongs to the step of its second update
    step = p.tk[t] + 1;
    kord = TK_GEMM;
  }
  // the inverses that the factorization's TRSMs apply: right after POTRF(k)
  const bool factor_inv = kind == TK_TRTRI && (p.op == OP_FACTOR_INVT || (p.op == TCHOL_OP_BATCHED && p.inv &&
                                                                          p.tk[t] + 1 < T));
  if (kind == TK_TRTRI && p.op != OP_FACTOR_INV && !factor_inv) {  // the FP64 solve's (the adjoint's) inverses:
    if (p.op == TCHOL_OP_BATCHED) step += T;                        // first in their step
    kord = -1;
  }
  if (kind == TK_BTRSV) kord = 0;  // within a backward step: BTRSV before BGEMV
  if (kind == TK_BGEMV) kord = 1;
  if (kind == TK_FTRSV) kord = 0;
  if (kind == TK_FGEMV) kord = 1;
  // within an adjoint step: the updates, the solves, the partial products, their sum, the tile
  if (kind == TK_GREV || kind == TK_GREV2) kord = 0;
  if (kind == TK_TREV) kord = 1;
  if (kind == TK_DPART) kord = 2;
  if (kind == TK_DRED) kord = 3;
  if (kind == TK_PREV || kind == TK_PADJM) kord = 4;
  if (kind == TK_PADJY) kord = 5;
  if (kind == TK_PADJS) kord = 6;
  // the chain of GREV(i, k, j) into Lbar_ik runs j downwards
  const int32_t tj = (kind == TK_GREV || kind == TK_GREV2) ? T - 1 - p.tj[t] : p.tj[t];
  // kinds in steps of two, so that a factorization's TRTRI(k) sits between
  // POTRF(k) and the TRSMs of step k
  return std::make_tuple(p.sys[t], step, factor_inv ? 2 * TK_POTRF + 1 : 2 * kord, p.ti[t], tj);
}

uint32_t xorshift32(uint32_t& x) {
  x ^= x << 13;
  x ^= x >> 17;
  x ^= x << 5;
  return x;
}

}  // namespace

const Split& default_split() {
  static const Split s;
  return s;
}

const Split& split_for(int32_t op) {
  static const Split mixed = [] {
    Split s;
    s.gemm_m = 256;
    return s;
  }();
  return op == OP_FACTOR_INV ? mixed : default_split();
}

namespace {

// HEFT's list scheduling (section 3.1) on P identical workers: whenever a
// worker is free, it takes the next work item of the ready task of highest
// upward rank (ties as in the rank order); an item lasts its task's weight
// divided by the task's parts.  The work items, in the order the simulation
// starts them, are the ticket list: a worker that claims a ticket then tends
// to find it ready, instead of waiting on a high-rank task whose
// predecessors are still running.  Start times respect the dependences, so
// the list is topological.  The task order records each task's first item.
constexpr int kListWorkers = 256;

bool list_schedule(Plan& p, int64_t ni) {
  const int64_t nt = p.ntask();
  std::vector<double> dur(nt);
  for (int64_t t = 0; t < nt; ++t) {
    double w = (double)weight(p.kind[t], p.op);
    if (p.op == TCHOL_OP_BATCHED) {
      const double u = (double)(p.systems[p.sys[t]].nb / 16);
      w *= u * u * u;
    }
    dur[t] = w / (double)std::max(1, p.parts[t]);
  }
  auto lower = [&](int32_t a, int32_t c) {  // priority_queue: true when a ranks below c
    if (p.rank[a] != p.rank[c]) return p.rank[a] < p.rank[c];
    return tie_key(p, c) < tie_key(p, a);
  };
  std::priority_queue<int32_t, std::vector<int32_t>, decltype(lower)> ready(lower);
  using Ev = std::pair<double, int32_t>;  // (time, task) of an item's end
  std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> ends;
  std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
  for (int w = 0; w < kListWorkers; ++w) free_at.push(0.0);
  std::vector<int32_t> indeg = p.dep0, next_part(nt, 0), left(p.parts.begin(), p.parts.end());
  for (int64_t t = 0; t < nt; ++t)
    if (indeg[t] == 0) ready.push((int32_t)t);
  auto finish = [&](int32_t t) {
    if (--left[t] == 0)
      for (int32_t e = p.succ_off[t]; e < p.succ_off[t + 1]; ++e)
        if (--indeg[p.succ[e]] == 0) ready.push(p.succ[e]);
  };
  std::vector<char> listed(nt, 0);
  p.order.clear();
  while ((int64_t)p.item_task.size() < ni) {
    const double tw = free_at.top();
    while (!ends.empty() && ends.top().first <= tw) {
      finish(ends.top().second);
      ends.pop();
    }
    if (ready.empty()) {  // idle until the next item ends
      if (ends.empty()) return false;  // unreachable for an acyclic graph
      free_at.pop();
      free_at.push(ends.top().first);
      continue;
    }
    const int32_t t = ready.top();
    const int32_t q = next_part[t]++;
    if (next_part[t] == p.parts[t]) ready.pop();
    free_at.pop();
    free_at.push(tw + dur[t]);
    ends.push(Ev(tw + dur[t], t));
    p.item_task.push_back(t);
    p.item_part.push_back(q);
    if (!listed[t]) {
      listed[t] = 1;
      p.order.push_back(t);
    }
  }
  return (int64_t)p.order.size() == nt;
}

// dependency counters, CSR successors, upward ranks, claim order and work items
bool finalize(Plan& p, std::vector<std::vector<int32_t>>& succ, int32_t policy, uint32_t seed) {
  const int64_t nt = p.ntask();
  p.dep0.assign(nt, 0);
  p.succ_off.assign(nt + 1, 0);
  for (int64_t t = 0; t < nt; ++t) {
    if ((int64_t)p.succ_off[t] + (int64_t)succ[t].size() > (int64_t)INT32_MAX) return false;
    p.succ_off[t + 1] = p.succ_off[t] + (int32_t)succ[t].size();
    for (int32_t s : succ[t]) p.dep0[s]++;
  }
  p.succ.reserve(p.succ_off[nt]);
  for (int64_t t = 0; t < nt; ++t) p.succ.insert(p.succ.end(), succ[t].begin(), succ[t].end());
  // upward ranks: tasks were created in a topological order, so a reverse
  // sweep suffices.  Systems of different tile sizes are weighed in a common
  // unit, (16)^3/3 flops, so that their ranks compare.
  p.rank.assign(nt, 0);
  for (int64_t t = nt - 1; t >= 0; --t) {
    int64_t best = 0;
    for (int32_t e = p.succ_off[t]; e < p.succ_off[t + 1]; ++e) best = std::max(best, p.rank[p.succ[e]]);
    int64_t w = weight(p.kind[t], p.op);
    if (p.op == TCHOL_OP_BATCHED) {
      const int64_t u = p.systems[p.sys[t]].nb / 16;
      w *= u * u * u;
    }
    p.rank[t] = w + best;
  }
  // claim order
  p.order.resize(nt);
  std::iota(p.order.begin(), p.order.end(), 0);
  if (policy == TCHOL_POLICY_RANK) {
    std::stable_sort(p.order.begin(), p.order.end(), [&](int32_t a, int32_t c) {
      if (p.rank[a] != p.rank[c]) return p.rank[a] > p.rank[c];
      return tie_key(p, a) < tie_key(p, c);
    });
  } else if (policy == TCHOL_POLICY_FIFO) {
    std::stable_sort(p.order.begin(), p.order.end(),
                     [&](int32_t a, int32_t c) { return tie_key(p, a) < tie_key(p, c); });
  } else if (policy == TCHOL_POLICY_RANDOM) {
    // Kahn's algorithm, choosing uniformly among the ready tasks
    std::vector<int32_t> indeg = p.dep0, ready;
    for (int64_t t = 0; t < nt; ++t)
      if (indeg[t] == 0) ready.push_back((int32_t)t);
    uint32_t x = seed ? seed : 0x9e3779b9u;
    p.order.clear();
    while (!ready.empty()) {
      size_t pick = xorshift32(x) % ready.size();
      int32_t t = ready[pick];
      ready[pick] = ready.back();
      ready.pop_back();
      p.order.push_back(t);
      for (int32_t e = p.succ_off[t]; e < p.succ_off[t + 1]; ++e)
        if (--indeg[p.succ[e]] == 0) ready.push_back(p.succ[e]);
    }
  }
  // every policy's order must be topological: the persistent kernel's
  // freedom from deadlock rests on it (a plan that broke it is refused)
  {
    std::vector<int32_t> pos(nt);
    for (int64_t q = 0; q < nt; ++q) pos[p.order[q]] = (int32_t)q;
    for (int64_t t = 0; t < nt; ++t)
      for (int32_t e = p.succ_off[t]; e < p.succ_off[t + 1]; ++e)
        if (pos[p.succ[e]] < pos[t]) return false;
  }
  int64_t ni = 0;
  for (int64_t t = 0; t < nt; ++t) ni += p.parts[t];
  if (ni > (int64_t)INT32_MAX / 2) return false;
  p.item_task.reserve(ni);
  p.item_part.reserve(ni);
  if (policy == TCHOL_POLICY_LIST) return list_schedule(p, ni);
  for (int32_t t : p.order)
    for (int32_t q = 0; q < p.parts[t]; ++q) {
      p.item_task.push_back(t);
      p.item_part.push_back(q);
    }
  return true;
}

}  // namespace

std::shared_ptr<Plan> build_plan(int32_t op, int64_t n, int64_t nb, int32_t policy, uint32_t seed,
                                 const Split& split) {
  auto plan = std::make_shared<Plan>();
  Plan& p = *plan;
  p.op = op;
  p.n = n;
  p.nb = nb;
  p.policy = policy;
  p.seed = seed;
  int64_t T64 = n == 0 ? 0 : (n + nb - 1) / nb;
  // the factorization's DAG has about T^3/6 tasks, the adjoint's T^3/3
  if (T64 > 1200 || (op == TCHOL_OP_BACKWARD && T64 > 160)) return nullptr;
  p.T = (int32_t)T64;
  System sy;
  sy.n = n;
  sy.nb = nb;
  sy.ld = n;
  sy.T = p.T;
  p.systems.push_back(sy);
  if (p.T == 0) {
    p.succ_off.assign(1, 0);
    return plan;
  }
  std::vector<std::vector<int32_t>> succ;
  Builder b(p, split, succ, 0);
  if (op == TCHOL_OP_FACTOR)
    build_factor(b);
  else if (op == OP_FACTOR_INVT)
    build_factor(b, nullptr, false, true);
  else if (op == OP_FACTOR_INV)
    build_factor(b, nullptr, true);
  else if (op == TCHOL_OP_SOLVE)
    build_solve(b, nullptr, Diag::kInvHere);
  else if (op == OP_SOLVE_INV)
    build_solve(b, nullptr, Diag::kInvGiven);
  else if (op == OP_SOLVE_SUBST)
    build_solve(b);
  else if (op == TCHOL_OP_BACKWARD)
    build_backward(b);
  else
    return nullptr;
  p.inv = op == TCHOL_OP_SOLVE || op == OP_FACTOR_INVT;
  if (!finalize(p, succ, policy, seed)) return nullptr;
  return plan;
}

std::shared_ptr<Plan> build_batched_plan(const std::vector<System>& systems, int32_t policy, uint32_t seed,
                                         const Split& split, bool inv) {
  auto plan = std::make_shared<Plan>();
  Plan& p = *plan;
  p.op = TCHOL_OP_BATCHED;
  p.inv = inv && systems.size() == 1;
  p.policy = policy;
  p.seed = seed;
  p.systems = systems;
  int64_t est = 0;
  for (auto& sy : p.systems) {
    const int64_t T64 = sy.n == 0 ? 0 : (sy.n + sy.nb - 1) / sy.nb;
    if (T64 > 1200) return nullptr;
    sy.T = (int32_t)T64;
    est += T64 * T64 * T64 / 6 + 3 * T64 * T64 + 4;
  }
  if (est > (int64_t)INT32_MAX / 4) return nullptr;
  std::vector<std::vector<int32_t>> succ;
  for (int32_t s = 0; s < (int32_t)p.systems.size(); ++s) {
    if (p.systems[s].T == 0) continue;
    Builder b(p, split, succ, s);
    FactorIds ids;
    build_factor(b, &ids, false, p.inv);
    build_solve(b, &ids, p.inv ? Diag::kInvHere : Diag::kSubst);
  }
  if (p.ntask() == 0) {
    p.succ_off.assign(1, 0);
    return plan;
  }
  if (!finalize(p, succ, policy, seed)) return nullptr;
  return plan;
}

std::shared_ptr<const Plan> get_plan(int32_t op, int64_t n, int64_t nb, int32_t policy, uint32_t seed) {
  static std::mutex mu;
  static std::map<std::tuple<int32_t, int64_t, int64_t, int32_t, uint32_t>, std::shared_ptr<const Plan>> cache;
  auto key = std::make_tuple(op, n, nb, policy, policy == TCHOL_POLICY_RANDOM ? seed : 0u);
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  std::shared_ptr<const Plan> p = build_plan(op, n, nb, policy, seed, split_for(op));
  if (!p) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  if (cache.size() > 64) cache.clear();
  cache[key] = p;
  return p;
}

std::shared_ptr<const Plan> get_batched_plan(const std::vector<System>& systems, int32_t policy, uint32_t seed,
                                             bool inv) {
  static std::mutex mu;
  static std::map<std::vector<int64_t>, std::shared_ptr<const Plan>> cache;
  std::vector<int64_t> key;
  key.reserve(3 * systems.size() + 3);
  key.push_back(inv ? 1 : 0);
  key.push_back(policy);
  key.push_back(policy == TCHOL_POLICY_RANDOM ? seed : 0);
  for (const System& sy : systems) {
    key.push_back(sy.n);
    key.push_back(sy.nb);
    key.push_back(sy.wgs);
  }
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  std::shared_ptr<const Plan> p = build_batched_plan(systems, policy, seed, default_split(), inv);
  if (!p) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  if (cache.size() >= 8) cache.clear();
  cache[key] = p;
  return p;
}

}  // namespace tchol
