// Host planner: builds the tile task DAG of the right-looking tile Cholesky
// (and of the tiled triangular solves), its dependency counters, successor
// lists, upward ranks and the ticket order in which the persistent kernel's
// workers claim work items.
//
// The paper's runtime discovers the same DAG implicitly from the data each
// task reads and writes (section 2, data-flow model), makes a task ready
// when its last predecessor completes (section 2.2, "activate") and, in its
// HEFT strategy, recalls the original priority rule: decreasing upward rank,
// the length of the longest path to the exit (section 3.1).  On one GPU all
// workers are identical, so the placement phase disappears and only the
// priority order remains; it is computed here once per (operation, n, nb).
#pragma once
#include <cstdint>
#include <memory>
#include <vector>

#include "tchol_kinds.h"   // task kinds, numbered alike on host and device

namespace tchol {

// One system of a plan: its matrix and right-hand sides, as offsets (in
// elements) from the launch's base pointers, and its order and tile size.
struct System {
  int64_t a_off = 0, b_off = 0;  // A_s at A + a_off (column-major, ld), B_s at B + b_off (ld n)
  int64_t n = 0, nb = 0, ld = 0;
  int32_t T = 0;                 // tiles per side
  int64_t d_off = 0;             // mixed precision: offset (doubles) of its FP64 diagonal tiles
  int32_t wgs = 0;               // work items of a one-tile system's POTRF above 128 (its
                                 // sub-block pool); 0: the default (one)
  int64_t ld2 = 0;               // FP32 batched systems on the compact instance: the
                                 // leading dimension of the FP32 matrix (d_off its offset)
};

struct Plan {
  int32_t op = 0;          // TCHOL_OP_FACTOR / TCHOL_OP_SOLVE / TCHOL_OP_BATCHED
  int64_t n = 0, nb = 0;   // matrix order, tile size (single-system plans)
  int32_t T = 0;           // tiles per side (single-system plans)
  int32_t policy = 0;      // TCHOL_POLICY_*
  uint32_t seed = 0;       // for TCHOL_POLICY_RANDOM
  std::vector<System> systems;             // one for factor and solve plans
  bool inv = false;        // the FP64 solve in it applies explicit inverses of the diagonal
                           // tiles, computed by its TRTRI tasks (single-system plans)
  // per task
  std::vector<int32_t> kind, ti, tj, tk;   // kind and tile coordinates (i, j, k)
  std::vector<int32_t> sys;                // the system the task belongs to
  std::vector<int32_t> parts;              // work items the task is split into
  std::vector<int32_t> dep0;               // initial dependency counter (in-degree)
  std::vector<int32_t> succ_off;           // CSR successor lists, size ntask + 1
  std::vector<int32_t> succ;
  std::vector<int64_t> rank;               // upward rank, in units of nb^3/3 flops (of (nb/16)^3
                                           // 16^3/3 flops in batched plans, whose systems differ in nb)
  std::vector<int32_t> order;              // tasks in claim order
  std::vector<int32_t> item_task, item_part;  // work items in ticket order
  int64_t ntask() const { return (int64_t)kind.size(); }
  int64_t nitem() const { return (int64_t)item_task.size(); }
  int64_t nedge() const { return (int64_t)succ.size(); }
};

// Plan operations used only inside the library (beyond the public TCHOL_OP_*):
// the mixed-precision factorization, whose DAG adds TRTRI(k) after POTRF(k),
// and its solve, whose diagonal steps are split into row strips (they apply
// explicit inverses).
constexpr int32_t OP_FACTOR_INV = 16;
constexpr int32_t OP_SOLVE_INV = 17;
// The FP64 solve by substitution against the diagonal tiles (tchol_opts.subst).
constexpr int32_t OP_SOLVE_SUBST = 18;
// The FP64 factorization whose TRSM tasks apply the diagonal tiles' explicit
// inverses (TRTRI(k) between POTRF(k) and TRSM(., k); tchol_opts.inv_trsm):
// the factorization of the merged factor + solve launch, alone.
constexpr int32_t OP_FACTOR_INVT = 19;

// Work-item granularity (rows x cols of one work item of each task kind).
struct Split {
  int32_t gemm_m = 128, gemm_n = 128;   // GEMM output sub-tile (also the adjoint's products)
  int32_t syrk_b = 128;                 // SYRK output sub-tile (square; the lower ones of the tile)
  int32_t trsm_rows = 32;               // TRSM row strip
  int32_t gemv_rows = 32;               // solve update row strip
};

// Builds (or fetches from a process-wide cache) the plan.  Returns nullptr
// for arguments the planner cannot represent (task counts beyond int32).
std::shared_ptr<const Plan> get_plan(int32_t op, int64_t n, int64_t nb, int32_t policy, uint32_t seed);

// Uncached build, used by get_plan and by the plan-introspection entry point.
std::shared_ptr<Plan> build_plan(int32_t op, int64_t n, int64_t nb, int32_t policy, uint32_t seed,
                                 const Split& split);

// Factorization followed by the solve, for every system, as one DAG: each
// system's factor tasks, then its solve tasks, joined by the data-flow
// edges POTRF(k) -> FTRSV(k) and TRSM(i, k) -> FGEMV(i, k).  With inv (one
// system: the merged factor + solve launch) the diagonal tiles' explicit
// inverses serve the TRSMs and the solve: POTRF(k) -> TRTRI(k) -> TRSM(., k)
// and FTRSV(k) (the last tile's TRTRI only for the solve, when its order is
// a multiple of 16).  Uncached.  Returns nullptr if the task count exceeds
// what the kernel indexes.
std::shared_ptr<Plan> build_batched_plan(const std::vector<System>& systems, int32_t policy, uint32_t seed,
                                         const Split& split, bool inv = false);

// The batched plan for these systems' orders and tile sizes, from a small
// process-wide cache keyed by them (offsets and leading dimensions are not
// part of the plan's task structure; the caller supplies them per launch).
std::shared_ptr<const Plan> get_batched_plan(const std::vector<System>& systems, int32_t policy, uint32_t seed,
                                             bool inv = false);

const Split& default_split();
// The split a single-system plan of this operation is built with: the
// mixed-precision factorization (OP_FACTOR_INV) takes 256 x 128 GEMM
// sub-tiles, whose FP32 products need twice the rows per work item to
// amortise its fixed costs; every other operation the default.
const Split& split_for(int32_t op);

}  // namespace tchol
