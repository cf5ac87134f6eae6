// Host-only check of the planner and the C ABI's argument validation, built
// with AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed): the
// device entry points are replaced by stubs that report an error, so only
// validation, planning and host bookkeeping run.
//
// Build and run: tests/test_sanitize.py (g++ -fsanitize=address,undefined).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include <hip/hip_runtime.h>

#include "tchol.h"
#include "plan.hpp"

extern "C" {
// stubs of the device-side entry points: never reached by the calls below
#define STUB(name, ...) hipError_t name(__VA_ARGS__) { std::fprintf(stderr, "stub %s reached\n", #name); std::abort(); }
struct KArgs;
STUB(tchol_dev_launch, const KArgs*, int32_t, const int32_t*, int64_t, int, int, hipStream_t, hipEvent_t, hipEvent_t)
STUB(tchol_dev_max_grid, int, int*)
STUB(tchol_dev_compact_grid, int, int*)
STUB(tchol_dev_backward_prep, const double*, int64_t, double*, double*, int64_t, int64_t, hipStream_t)
STUB(tchol_refine_convert, const double*, int64_t, float*, int64_t, int64_t, hipStream_t)
STUB(tchol_refine_residual, const double*, int64_t, int64_t, const double*, const double*, double*, int64_t, int, int,
     double*, hipStream_t)
STUB(tchol_refine_colmax, const double*, int64_t, int64_t, int, double*, hipStream_t)
STUB(tchol_refine_axpy, double*, const double*, int64_t, hipStream_t)
STUB(tchol_b32_prepare, const int64_t*, int32_t, const float*, const float*, double*, double*, int, hipStream_t)
STUB(tchol_b32_finish, const int64_t*, int32_t, float*, float*, const double*, const double*, int, hipStream_t)
STUB(tchol_refine_diag, const double*, int64_t, int64_t, int64_t, double*, hipStream_t)
}

static int failures = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

// every work item's task comes after all of its predecessors' items
static void check_plan(const tchol::Plan& p) {
  const int64_t nt = p.ntask();
  std::vector<int64_t> last(nt, -1), first(nt, -1);
  for (int64_t i = 0; i < p.nitem(); ++i) {
    const int t = p.item_task[i];
    CHECK(t >= 0 && t < nt);
    if (first[t] < 0) first[t] = i;
    last[t] = i;
  }
  std::vector<int32_t> indeg(nt, 0);
  for (int64_t t = 0; t < nt; ++t) {
    CHECK(first[t] >= 0);
    for (int32_t e = p.succ_off[t]; e < p.succ_off[t + 1]; ++e) {
      const int s = p.succ[e];
      CHECK(s >= 0 && s < nt);
      ++indeg[s];
      CHECK(last[t] < first[s]);
    }
  }
  for (int64_t t = 0; t < nt; ++t) CHECK(indeg[t] == p.dep0[t]);
}

int main() {
  const int64_t ns[] = {0, 1, 17, 100, 513, 1000, 2048};
  const int64_t nbs[] = {16, 64, 128, 512};
  const int32_t ops[] = {TCHOL_OP_FACTOR, TCHOL_OP_SOLVE, TCHOL_OP_BACKWARD, tchol::OP_FACTOR_INV,
                         tchol::OP_SOLVE_INV};
  for (int32_t op : ops)
    for (int64_t n : ns)
      for (int64_t nb : nbs)
        for (int32_t pol = 0; pol <= 3; ++pol) {
          auto p = tchol::build_plan(op, n, nb, pol, 7, tchol::split_for(op));
          CHECK(p != nullptr);
          if (p) check_plan(*p);
        }
  // a ragged batch, every policy
  std::vector<tchol::System> sys;
  for (int s = 0; s < 40; ++s) {
    tchol::System y;
    y.n = (s * 37) % 700;
    y.nb = 16 * (1 + (s * 5) % 32);
    y.ld = y.n + 1;
    sys.push_back(y);
  }
  for (int32_t pol = 0; pol <= 3; ++pol) {
    auto p = tchol::build_batched_plan(sys, pol, 3, tchol::default_split());
    CHECK(p != nullptr);
    if (p) check_plan(*p);
  }
  // argument validation of the C ABI (every call returns before any HIP call)
  double* fake = reinterpret_cast<double*>(0x10000);
  CHECK(tchol_factor(fake, -1, 128, fake, 1 << 20, nullptr) == -2);
  CHECK(tchol_factor(fake, 100, 24, fake, 1 << 20, nullptr) == -3);
  CHECK(tchol_factor(nullptr, 100, 128, fake, 1 << 20, nullptr) == -1);
  CHECK(tchol_factor(fake, 0, 128, nullptr, 0, nullptr) == 0);
  CHECK(tchol_solve(fake, 100, 128, fake, -1, fake, 1 << 20, nullptr) == -5);
  CHECK(tchol_factor_solve(fake, 100, 128, fake, 1, nullptr, 0, nullptr, nullptr) == -6);
  CHECK(tchol_workspace_bytes(7, 10, 16, 0) == -1);
  CHECK(tchol_workspace_bytes(TCHOL_OP_FACTOR, 4096, 512, 0) > 0);
  CHECK(tchol_backward(fake, 100, 16, nullptr, fake, 1 << 20, nullptr) == -4);
  tchol_opts bad = {};
  bad.policy = 9;
  CHECK(tchol_factor_ex(fake, 100, 16, fake, 1 << 20, nullptr, &bad) == TCHOL_E_UNSUPPORTED);
  int64_t counts[4] = {0, 0, 0, 0};
  CHECK(tchol_plan_query(TCHOL_OP_FACTOR, 1000, 128, TCHOL_POLICY_LIST, 0, counts, nullptr, nullptr, nullptr, nullptr,
                         nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == 0);
  CHECK(counts[0] == 8 + 28 + 28 + 30 + 13);  // T = 8: 30 single GEMMs, 13 merged pairs
  std::vector<int32_t> kind(counts[0]), items(counts[2]);
  CHECK(tchol_plan_query(TCHOL_OP_FACTOR, 1000, 128, TCHOL_POLICY_RANDOM, 5, nullptr, kind.data(), nullptr, nullptr,
                         nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, items.data(), nullptr) == 0);
  const int32_t bn[3] = {10, 300, 0}, bnb[3] = {16, 128, 64};
  CHECK(tchol_batched_workspace_bytes(bn, bnb, 3) > 0);
  CHECK(tchol_strerror(TCHOL_E_SCRATCH) != nullptr);
  std::printf("sanitized host checks: %d failures\n", failures);
  return failures == 0 ? 0 : 1;
}
