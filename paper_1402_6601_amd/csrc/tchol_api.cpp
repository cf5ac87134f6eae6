// C ABI of libtchol: argument checks, workspace layout, plan upload and the
// launch of the persistent kernel.  See include/tchol.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/tchol.h"
#include "kargs.h"
#include "plan.hpp"

extern "C" hipError_t tchol_dev_launch(const KArgs* a, int32_t ntask, const int32_t* dep0, int64_t npool, int grid,
                                       int wide, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1);
extern "C" hipError_t tchol_dev_max_grid(int device, int* grid);
extern "C" hipError_t tchol_dev_compact_grid(int device, int* grid);
extern "C" hipError_t tchol_dev_backward_prep(const double* L, int64_t n, double* LT, double* Q, int64_t ldq,
                                              int64_t np, hipStream_t stream);
extern "C" hipError_t tchol_refine_convert(const double* A, int64_t lda, float* W, int64_t ldw, int64_t n,
                                           hipStream_t s);
extern "C" hipError_t tchol_refine_residual(const double* A, int64_t lda, int64_t n, const double* X,
                                            const double* Bin, double* Out, int64_t ldb, int nrhs, int absmode,
                                            double* P, hipStream_t s);
extern "C" hipError_t tchol_refine_colmax(const double* V, int64_t ldv, int64_t n, int ncols, double* out,
                                          hipStream_t s);
extern "C" hipError_t tchol_refine_axpy(double* X, const double* D, int64_t count, hipStream_t s);
extern "C" hipError_t tchol_b32_prepare(const int64_t* desc, int32_t batch, const float* A, const float* B, double* D,
                                        double* Bd, int nrhs, hipStream_t s);
extern "C" hipError_t tchol_b32_finish(const int64_t* desc, int32_t batch, float* A, float* B, const double* D,
                                       const double* Bd, int nrhs, hipStream_t s);
extern "C" hipError_t tchol_refine_diag(const double* A, int64_t lda, int64_t n, int64_t nb, double* D,
                                        hipStream_t s);

namespace {

using tchol::Plan;

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Byte offsets of the workspace regions.  [dep0, end) is a copy of the
// plan's constant image (counters, descriptors, successors, ticket list and
// the system table), uploaded in one transfer; hdr, dep, done, sinfo and the
// POTRF pools are (re)initialised by a small kernel on every call.
struct Layout {
  int64_t hdr = 0, dep = 0, done = 0, sinfo = 0, pool = 0, dep0 = 0, desc = 0, succ = 0, items = 0, sys = 0,
          end = 0;
  int64_t npool = 0;  // words of the POTRF pools
};

// Diagonal tiles over all systems of a plan (one POTRF pool each).
int64_t diag_tiles(const Plan& p) {
  int64_t t = 0;
  for (const auto& sy : p.systems) t += sy.n == 0 ? 0 : (sy.n + sy.nb - 1) / sy.nb;
  return t;
}

Layout layout_of(const Plan& p) {
  Layout L;
  const int64_t nt = p.ntask(), ns = (int64_t)p.systems.size();
  L.npool = POOL_WORDS * diag_tiles(p);
  L.hdr = 0;
  L.dep = align_up(HDR_WORDS * 4);
  L.done = align_up(L.dep + 4 * nt);
  L.sinfo = align_up(L.done + 4 * nt);
  L.pool = align_up(L.sinfo + 4 * ns);
  L.dep0 = align_up(L.pool + 4 * L.npool);
  L.desc = align_up(L.dep0 + 4 * nt);
  L.succ = align_up(L.desc + 4 * DESC_WORDS * nt);
  L.items = align_up(L.succ + 4 * p.nedge());
  L.sys = align_up(L.items + 8 * p.nitem());
  L.end = align_up(L.sys + 8 * SYS_WORDS * ns);
  return L;
}

// The FP64 solve's explicit inverses and intermediate vector (plans with
// inv), after the scheduler's regions: L_kk^{-T} of every diagonal tile
// (nb x nb FP64 each) and y (n x nrhs FP64).
struct InvLayout {
  int64_t dinvt = 0, dinv = 0, sx = 0, end = 0;
};

InvLayout inv_layout(const Plan& p, int64_t nrhs) {
  InvLayout V;
  V.end = layout_of(p).end;
  if (!p.inv || p.systems.empty()) return V;
  const tchol::System& sy = p.systems[0];
  const int64_t T = sy.n == 0 ? 0 : (sy.n + sy.nb - 1) / sy.nb;
  V.dinvt = align_up(V.end);
  V.dinv = align_up(V.dinvt + 8 * T * sy.nb * sy.nb);  // L_kk^{-1}, for the TRSM items
  V.sx = align_up(V.dinv + 8 * T * sy.nb * sy.nb);
  V.end = align_up(V.sx + 8 * sy.n * std::max<int64_t>(nrhs, 1));
  return V;
}

// The constant part of the workspace for one plan, in pinned host memory
// when the runtime can provide it.
struct Image {
  Layout lay;
  std::vector<char> pageable;
  char* pinned = nullptr;
  int64_t bytes = 0;
  const char* data() const { return pinned ? pinned : pageable.data(); }
  ~Image() {
    if (pinned) (void)hipHostFree(pinned);
  }
};

// sys_override: the systems' offsets and leading dimensions for this launch
// (a cached batched plan's own records are not used for them).
std::shared_ptr<Image> make_image(const Plan& p, bool pin, const std::vector<tchol::System>* sys_override = nullptr) {
  auto img = std::make_shared<Image>();
  img->lay = layout_of(p);
  const Layout& L = img->lay;
  img->bytes = L.end - L.dep0;
  char* buf = nullptr;
  if (pin && hipHostMalloc(reinterpret_cast<void**>(&buf), (size_t)img->bytes, hipHostMallocDefault) == hipSuccess &&
      buf) {
    img->pinned = buf;
  } else {
    if (pin) (void)hipGetLastError();
    img->pageable.resize((size_t)img->bytes);
    buf = img->pageable.data();
  }
  std::memset(buf, 0, (size_t)img->bytes);
  const int64_t nt = p.ntask();
  int32_t* dep0 = reinterpret_cast<int32_t*>(buf + (L.dep0 - L.dep0));
  int32_t* desc = reinterpret_cast<int32_t*>(buf + (L.desc - L.dep0));
  int32_t* succ = reinterpret_cast<int32_t*>(buf + (L.succ - L.dep0));
  int32_t* items = reinterpret_cast<int32_t*>(buf + (L.items - L.dep0));
  int64_t* sys = reinterpret_cast<int64_t*>(buf + (L.sys - L.dep0));
  for (int64_t t = 0; t < nt; ++t) {
    dep0[t] = p.dep0[t];
    int32_t* d = desc + DESC_WORDS * t;
    d[0] = p.kind[t];
    d[1] = p.ti[t];
    d[2] = p.tj[t];
    d[3] = p.tk[t];
    d[4] = p.parts[t];
    d[5] = p.succ_off[t];
    d[6] = p.succ_off[t + 1];
    d[7] = p.sys[t];
  }
  if (p.nedge()) std::memcpy(succ, p.succ.data(), 4 * (size_t)p.nedge());
  for (int64_t i = 0; i < p.nitem(); ++i) {
    items[2 * i] = p.item_task[i];
    items[2 * i + 1] = p.item_part[i];
  }
  int64_t pool_off = 0;
  for (size_t s = 0; s < p.systems.size(); ++s) {
    const tchol::System& sy = sys_override ? (*sys_override)[s] : p.systems[s];
    int64_t* r = sys + SYS_WORDS * s;
    r[0] = sy.a_off;
    r[1] = sy.b_off;
    r[2] = sy.n;
    r[3] = sy.nb;
    r[4] = sy.ld;
    r[5] = sy.d_off;
    r[6] = pool_off;
    r[7] = sy.ld2;
    pool_off += p.systems[s].n == 0 ? 0 : (p.systems[s].n + p.systems[s].nb - 1) / p.systems[s].nb;
  }
  return img;
}

// Cached per (plan, leading dimension); ld = 0 keeps the plan's own (the
// mixed-precision working copy has a padded one).  Single-system plans are
// themselves cached.
std::shared_ptr<const Image> image_of(const std::shared_ptr<const Plan>& p, int64_t ld = 0) {
  using Key = std::pair<const Plan*, int64_t>;
  static std::mutex mu;
  static std::map<Key, std::pair<std::weak_ptr<const Plan>, std::shared_ptr<const Image>>> cache;
  const Key key(p.get(), ld);
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end() && !it->second.first.expired()) return it->second.second;
  }
  std::shared_ptr<const Image> img;
  if (ld > 0) {
    std::vector<tchol::System> sys = p->systems;
    for (auto& sy : sys) sy.ld = ld;
    img = make_image(*p, true, &sys);
  } else {
    img = make_image(*p, true);
  }
  std::lock_guard<std::mutex> g(mu);
  if (cache.size() > 64) cache.clear();
  cache[key] = std::make_pair(std::weak_ptr<const Plan>(p), img);
  return img;
}

// The image of a batched launch: the plan with the systems' offsets and
// leading dimensions of this call.  The last few are kept (pinned, so the
// upload is one asynchronous copy), matched by plan and by every system's
// record, so a caller that repeats a batch on the same buffers pays for the
// image once.
std::shared_ptr<const Image> batched_image_of(const std::shared_ptr<const Plan>& p,
                                              const std::vector<tchol::System>& sys) {
  struct Entry {
    std::weak_ptr<const Plan> plan;
    const Plan* key;
    std::vector<tchol::System> sys;
    std::shared_ptr<const Image> img;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;  // most recently used last
  auto same = [&](const std::vector<tchol::System>& a) {
    if (a.size() != sys.size()) return false;
    for (size_t i = 0; i < a.size(); ++i) {
      const tchol::System &x = a[i], &y = sys[i];
      if (x.a_off != y.a_off || x.b_off != y.b_off || x.n != y.n || x.nb != y.nb || x.ld != y.ld ||
          x.d_off != y.d_off || x.ld2 != y.ld2)
        return false;
    }
    return true;
  };
  {
    std::lock_guard<std::mutex> g(mu);
    for (size_t i = 0; i < cache.size(); ++i) {
      if (cache[i].key == p.get() && !cache[i].plan.expired() && same(cache[i].sys)) {
        Entry e = cache[i];
        cache.erase(cache.begin() + (std::ptrdiff_t)i);
        cache.push_back(e);
        return e.img;
      }
    }
  }
  std::shared_ptr<const Image> img = make_image(*p, true, &sys);
  std::lock_guard<std::mutex> g(mu);
  if (cache.size() >= 8) cache.erase(cache.begin());
  cache.push_back(Entry{std::weak_ptr<const Plan>(p), p.get(), sys, img});
  return img;
}

struct DeviceInfo {
  int grid = 0;
  int grid_compact = 0;  // the compact instance (batched one-tile systems)
  int64_t clock_khz = 0;
};

hipError_t device_info(DeviceInfo* out) {
  static std::mutex mu;
  static std::map<int, DeviceInfo> cache;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) {
    *out = it->second;
    return hipSuccess;
  }
  DeviceInfo di;
  e = tchol_dev_max_grid(dev, &di.grid);
  if (e != hipSuccess) return e;
  e = tchol_dev_compact_grid(dev, &di.grid_compact);
  if (e != hipSuccess) return e;
  int khz = 0;
  e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return e;
  di.clock_khz = khz > 0 ? khz : 100000;
  cache[dev] = di;
  *out = di;
  return hipSuccess;
}

bool policy_ok(int32_t p) { return p >= TCHOL_POLICY_LIST && p <= TCHOL_POLICY_RANDOM; }

bool nb_ok(int64_t nb) { return nb >= TCHOL_NB_MIN && nb <= TCHOL_NB_MAX && nb % 16 == 0; }

const tchol_opts kDefaultOpts = {TCHOL_POLICY_LIST, 0u, 0, nullptr, nullptr, 0, 0, nullptr, 0};

// Uploads the plan image, launches reset + persistent kernel on the stream,
// reads the header back and synchronises.  sinfo_out (batched): per-system
// failing columns.  mixed: 0 FP64; 1 / 2 the mixed-precision factor / solve
// (A is then the FP32 working copy and D its FP64 diagonal tiles); 6 the
// compact FP64 instance for batched systems of one tile each, 7 the same
// reading and writing FP32 matrices at A32.  Returns the library code.
int32_t execute(const Plan& plan, const Image& img, double* A, double* B, int64_t nrhs, bool wide, bool batched,
                void* ws, int64_t ws_bytes, void* stream_v, const tchol_opts& o, int32_t ws_arg,
                int32_t* sinfo_out, double* D = nullptr, int mixed = 0, double* Qp = nullptr,
                double* LTp = nullptr, int64_t ldq = 0, double* Dinv = nullptr, double* DinvT = nullptr,
                double* Sx = nullptr, uint16_t* H = nullptr, int64_t hrows = 0, float* A32 = nullptr) {
  const Layout& L = img.lay;
  if (ws_bytes < L.end) return -(ws_arg + 1);
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return -ws_arg;
  // the trace buffer must hold 4 words per work item of this launch (the
  // options follow the stream, which follows ws and ws_bytes)
  if (o.trace && o.trace_words / 4 < plan.nitem()) return -(ws_arg + 3);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
  DeviceInfo di;
  if (device_info(&di) != hipSuccess) return TCHOL_E_HIP;
  char* w = static_cast<char*>(ws);
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.A = A;
  a.B = B;
  a.n = plan.n;
  a.nb = plan.nb;
  a.ld = plan.n;
  a.ldb = plan.n;
  a.nrhs = nrhs;
  a.T = plan.T;
  a.nitem = (int32_t)plan.nitem();
  const tchol::Split& sp = tchol::split_for(plan.op);
  a.gemm_m = sp.gemm_m;
  a.gemm_n = sp.gemm_n;
  a.syrk_b = sp.syrk_b;
  a.trsm_rows = sp.trsm_rows;
  a.gemv_rows = sp.gemv_rows;
  a.hdr = reinterpret_cast<int32_t*>(w + L.hdr);
  a.dep = reinterpret_cast<int32_t*>(w + L.dep);
  a.done = reinterpret_cast<int32_t*>(w + L.done);
  a.desc = reinterpret_cast<const int32_t*>(w + L.desc);
  a.succ = reinterpret_cast<const int32_t*>(w + L.succ);
  a.items = reinterpret_cast<const int32_t*>(w + L.items);
  a.sys = reinterpret_cast<const int64_t*>(w + L.sys);
  a.sinfo = reinterpret_cast<int32_t*>(w + L.sinfo);
  a.pool = reinterpret_cast<int32_t*>(w + L.pool);
  a.batched = batched ? 1 : 0;
  a.nsys = (int32_t)plan.systems.size();
  a.D = D;
  a.mixed = mixed;
  a.Q = Qp;
  a.LT = LTp;
  a.ldq = ldq;
  a.Dinv = Dinv;
  a.DinvT = DinvT;
  a.S = Sx;
  a.inv = plan.inv ? 1 : 0;
  a.H = H;
  a.hrows = hrows;
  a.A32 = A32;
  const int64_t limit_us = o.wait_limit_us > 0 ? o.wait_limit_us : 30000000;
  a.wait_limit = limit_us * di.clock_khz / 1000;
  a.trace = o.trace;

  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int32_t rc = 0;
  int32_t hdr[HDR_WORDS];
  hipError_t e = hipMemcpyAsync(w + L.dep0, img.data(), (size_t)img.bytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && o.kernel_ms) {
    e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
  }
  const int grid =
      (int)std::min<int64_t>(mixed >= 6 ? di.grid_compact : di.grid, std::max<int64_t>(1, plan.nitem()));
  if (e == hipSuccess)
    e = tchol_dev_launch(&a, (int32_t)plan.ntask(), reinterpret_cast<const int32_t*>(w + L.dep0), L.npool, grid,
                         wide ? 1 : 0, stream, ev0, ev1);
  if (e == hipSuccess) e = hipMemcpyAsync(hdr, a.hdr, sizeof(hdr), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && sinfo_out && a.nsys > 0)
    e = hipMemcpyAsync(sinfo_out, a.sinfo, 4 * (size_t)a.nsys, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e == hipSuccess && o.kernel_ms) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, ev0, ev1);
    *o.kernel_ms = ms;
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (e != hipSuccess) return TCHOL_E_HIP;
  if (hdr[HDR_ERROR] == DEV_ERR_TIMEOUT)
    rc = TCHOL_E_TIMEOUT;
  else if (hdr[HDR_ERROR] != 0)
    rc = TCHOL_E_INTERNAL;
  else if (hdr[HDR_INFO] > 0)
    rc = hdr[HDR_INFO];
  else if (hdr[HDR_DONE] != a.nitem)
    rc = TCHOL_E_INTERNAL;
  return rc;
}

int32_t run(int32_t op, double* A, double* B, int64_t n, int64_t nb, int64_t nrhs, void* ws, int64_t ws_bytes,
            void* stream_v, const tchol_opts* opts, int32_t ws_arg) {
  const tchol_opts& o = opts ? *opts : kDefaultOpts;
  if (!policy_ok(o.policy)) return TCHOL_E_UNSUPPORTED;
  const int32_t pop = op == TCHOL_OP_SOLVE && o.subst        ? tchol::OP_SOLVE_SUBST
                     : op == TCHOL_OP_FACTOR && o.inv_trsm ? tchol::OP_FACTOR_INVT
                                                           : op;
  auto plan = tchol::get_plan(pop, n, nb, o.policy, o.seed);
  if (!plan) return TCHOL_E_UNSUPPORTED;
  if (o.trace && o.trace_words / 4 < plan->nitem()) return -(ws_arg + 3);
  auto img = image_of(plan);
  // 16-byte panel transfers need an even leading dimension and an aligned matrix
  const bool wide = (n % 2 == 0) && (reinterpret_cast<uintptr_t>(A) % 16 == 0);
  const InvLayout V = inv_layout(*plan, nrhs);
  if (ws_bytes < V.end) return -(ws_arg + 1);
  char* w = static_cast<char*>(ws);
  double* DinvT = plan->inv ? reinterpret_cast<double*>(w + V.dinvt) : nullptr;
  double* Dinv = plan->inv ? reinterpret_cast<double*>(w + V.dinv) : nullptr;
  double* Sx = plan->inv ? reinterpret_cast<double*>(w + V.sx) : nullptr;
  return execute(*plan, *img, A, B, nrhs, wide, false, ws, ws_bytes, stream_v, o, ws_arg, nullptr, nullptr, 0,
                 nullptr, nullptr, 0, Dinv, DinvT, Sx);
}

void fill_query(const Plan& pl, int64_t* counts, int32_t* kind, int32_t* ti, int32_t* tj, int32_t* tk, int32_t* sys,
                int32_t* parts, int32_t* dep0, int64_t* rank, int32_t* succ_off, int32_t* succ, int32_t* item_task,
                int32_t* item_part) {
  const Plan* p = &pl;
  const int64_t nt = p->ntask();
  if (counts) {
    // longest path counted in tasks; creation order is topological
    std::vector<int32_t> depth(nt, 1);
    int32_t cp = 0;
    for (int64_t t = nt - 1; t >= 0; --t) {
      int32_t best = 0;
      for (int32_t e = p->succ_off[t]; e < p->succ_off[t + 1]; ++e) best = std::max(best, depth[p->succ[e]]);
      depth[t] = 1 + best;
      cp = std::max(cp, depth[t]);
    }
    counts[0] = nt;
    counts[1] = p->nedge();
    counts[2] = p->nitem();
    counts[3] = cp;
  }
  for (int64_t t = 0; t < nt; ++t) {
    if (kind) kind[t] = p->kind[t];
    if (ti) ti[t] = p->ti[t];
    if (tj) tj[t] = p->tj[t];
    if (tk) tk[t] = p->tk[t];
    if (sys) sys[t] = p->sys[t];
    if (parts) parts[t] = p->parts[t];
    if (dep0) dep0[t] = p->dep0[t];
    if (rank) rank[t] = p->rank[t];
  }
  if (succ_off) std::copy(p->succ_off.begin(), p->succ_off.end(), succ_off);
  if (succ) std::copy(p->succ.begin(), p->succ.end(), succ);
  if (item_task) std::copy(p->item_task.begin(), p->item_task.end(), item_task);
  if (item_part) std::copy(p->item_part.begin(), p->item_part.end(), item_part);
}

// Validates the batched arguments and collects the systems; returns 0 or -i.
int32_t batched_systems(const int64_t* a_off, const int32_t* lda, const int64_t* b_off, const int32_t* n,
                        const int32_t* nb, int32_t batch, std::vector<tchol::System>* out) {
  if (batch < 0) return -9;
  if (batch > 0 && !n) return -6;
  if (batch > 0 && !nb) return -7;
  out->clear();
  out->reserve(batch);
  for (int32_t s = 0; s < batch; ++s) {
    if (n[s] < 0) return -6;
    if (!nb_ok(nb[s])) return -7;
    tchol::System sy;
    sy.n = n[s];
    sy.nb = nb[s];
    if (out && a_off && lda && b_off) {
      if (a_off[s] < 0) return -2;
      if (lda[s] < std::max<int32_t>(1, n[s])) return -3;
      if (b_off[s] < 0) return -5;
      sy.a_off = a_off[s];
      sy.ld = lda[s];
      sy.b_off = b_off[s];
    }
    out->push_back(sy);
  }
  return 0;
}


// Adjoint: workspace regions (byte offsets).  LT (the transposed factor) and
// Q (twice the symmetric adjoint) are np x np with np = n rounded up to 16
// and ldq = np, zero past the order; the partial-product slots hold
// T (T - 1) / 2 tiles of nb x nb; the diagonal tiles' inverses L_kk^{-T}
// and the closed-form adjoint's two scratch tiles per diagonal tile follow.
struct BackLayout {
  int64_t np = 0, ldq = 0, lt = 0, q = 0, slots = 0, inv = 0, scr = 0, sched = 0, end = 0;
};

BackLayout back_layout(int64_t n, int64_t nb, const Plan& p) {
  BackLayout B;
  const int64_t T = (n + nb - 1) / nb;
  B.np = (n + 15) / 16 * 16;
  B.ldq = B.np;
  B.lt = 0;
  B.q = align_up(B.lt + 8 * B.ldq * B.np);
  B.slots = align_up(B.q + 8 * B.ldq * B.np);
  // the closed-form tile adjoints: L_kk^{-T}, then two scratch tiles, per diagonal tile
  B.inv = align_up(B.slots + 8 * (T * (T - 1) / 2) * nb * nb);
  B.scr = align_up(B.inv + 8 * T * nb * nb);
  B.sched = align_up(B.scr + 8 * 2 * T * nb * nb);
  B.end = B.sched + layout_of(p).end;
  return B;
}

// Batched FP32: workspace regions (byte offsets): the per-system descriptor
// table, the FP64 diagonal tiles (d_off per system) and the compact FP64
// right-hand sides.
struct B32Layout {
  int64_t desc = 0, d = 0, bd = 0, sched = 0, end = 0;
};

// Fills d_off and the compact right-hand-side offsets (b_off) of the systems.
B32Layout b32_layout(std::vector<tchol::System>* sys, int64_t nrhs, const Plan& p) {
  int64_t dtot = 0, btot = 0;
  for (auto& sy : *sys) {
    const int64_t T = sy.n == 0 ? 0 : (sy.n + sy.nb - 1) / sy.nb;
    sy.d_off = dtot;
    dtot += T * sy.nb * sy.nb;
    sy.b_off = btot;
    btot += sy.n * nrhs;
  }
  B32Layout L;
  L.desc = 0;
  L.d = align_up(L.desc + 8 * 8 * (int64_t)sys->size());
  L.bd = align_up(L.d + 8 * dtot);
  L.sched = align_up(L.bd + 8 * btot);
  L.end = L.sched + layout_of(p).end;
  return L;
}

// Mixed-precision solve: workspace regions (byte offsets).  The FP32 working
// copy has ld = n + 3 rounded up to a multiple of 4 (its matrix-core loads
// move four rows per 16-byte lane, so three rows past the order are read;
// they hold zeros).
// With BF16 updates the workspace also holds the panels' BF16 terms (H):
// three terms, per column block T nb rows of nb K-contiguous values.
struct MixedLayout {
  int64_t ldw = 0, w = 0, h = 0, hrows = 0, d = 0, dinv = 0, dinvt = 0, b0 = 0, r = 0, sx = 0, part = 0, norms = 0,
          sched = 0, end = 0;
};

MixedLayout mixed_layout(int64_t n, int64_t nb, int64_t nrhs, const Plan& fp, const Plan& sp, bool bf16 = false) {
  MixedLayout M;
  const int64_t T = (n + nb - 1) / nb;
  M.ldw = (n + 3 + 3) / 4 * 4;
  M.w = 0;
  M.h = align_up(M.w + 4 * M.ldw * n);
  M.hrows = T * nb;
  M.d = align_up(M.h + (bf16 ? 2 * 3 * T * M.hrows * nb : 0));
  M.dinv = align_up(M.d + 8 * T * nb * nb);        // L_kk^{-1} per diagonal tile (FP64)
  M.dinvt = align_up(M.dinv + 8 * T * nb * nb);    // L_kk^{-T}
  M.b0 = align_up(M.dinvt + 8 * T * nb * nb);
  M.r = align_up(M.b0 + 8 * n * nrhs);
  // the residual region first holds the row sums of |A| (n entries)
  M.sx = align_up(M.r + 8 * n * std::max<int64_t>(nrhs, 1));   // the solves' intermediate y
  M.part = align_up(M.sx + 8 * n * nrhs);                        // the residual's partial sums
  M.norms = align_up(M.part + 8 * 2 * 8 * n * std::max<int64_t>(nrhs, 1));
  M.sched = align_up(M.norms + 8 * (1 + 3 * nrhs));
  M.end = M.sched + std::max(layout_of(fp).end, layout_of(sp).end);
  return M;
}

}  // namespace

namespace tchol {

// Workspace bytes of the merged factor + solve launch (inv as below).
int64_t factor_solve_bytes(int64_t n, int64_t nb, int64_t nrhs, bool inv) {
  std::vector<tchol::System> systems(1);
  systems[0].n = n;
  systems[0].nb = nb;
  auto plan = tchol::get_batched_plan(systems, TCHOL_POLICY_RANK, 0, inv);
  if (!plan) return TCHOL_E_UNSUPPORTED;
  // every policy yields the same task, edge and item counts, hence the same layout
  return inv_layout(*plan, nrhs).end;
}

// The merged factor + solve launch on validated arguments (n > 0).  pinned:
// keep the plan's constant image in pinned host memory (allocated once per
// plan); otherwise in pageable memory, so that the call allocates no device
// or pinned memory once the plan is cached.  inv: the solve applies the
// diagonal tiles' explicit inverses (workspace for them included); else it
// substitutes against the tiles.
int32_t factor_solve_run(double* A, int64_t n, int64_t nb, double* B, int64_t nrhs, void* ws, int64_t ws_bytes,
                         void* stream, const tchol_opts* opts, bool pinned, bool inv) {
  const tchol_opts& o = opts ? *opts : kDefaultOpts;
  if (!policy_ok(o.policy)) return TCHOL_E_UNSUPPORTED;
  // one system of the merged factor + solve DAG: A at offset 0 with ld n, B at 0
  std::vector<tchol::System> systems(1);
  systems[0].n = n;
  systems[0].nb = nb;
  systems[0].ld = n;
  auto plan = tchol::get_batched_plan(systems, o.policy, o.seed, inv);
  if (!plan) return TCHOL_E_UNSUPPORTED;
  const InvLayout V = inv_layout(*plan, nrhs);
  if (ws_bytes < V.end) return -7;
  if (o.trace && o.trace_words / 4 < plan->nitem()) return -9;
  std::shared_ptr<const Image> img;
  {
    // the image depends only on the plan here (fixed offsets), so it is cached
    using Key = std::pair<const Plan*, bool>;
    static std::mutex mu;
    static std::map<Key, std::pair<std::weak_ptr<const Plan>, std::shared_ptr<const Image>>> cache;
    std::lock_guard<std::mutex> g(mu);
    const Key key(plan.get(), pinned);
    auto it = cache.find(key);
    if (it != cache.end() && !it->second.first.expired()) {
      img = it->second.second;
    } else {
      img = make_image(*plan, pinned, &systems);
      if (cache.size() > 16) cache.clear();
      cache[key] = std::make_pair(std::weak_ptr<const Plan>(plan), img);
    }
  }
  const bool wide = (n % 2 == 0) && (reinterpret_cast<uintptr_t>(A) % 16 == 0);
  int32_t info = 0;
  char* w = static_cast<char*>(ws);
  double* DinvT = plan->inv ? reinterpret_cast<double*>(w + V.dinvt) : nullptr;
  double* Dinv = plan->inv ? reinterpret_cast<double*>(w + V.dinv) : nullptr;
  double* Sx = plan->inv ? reinterpret_cast<double*>(w + V.sx) : nullptr;
  const int32_t rc = execute(*plan, *img, A, B, nrhs, wide, true, ws, ws_bytes, stream, o, 6, &info, nullptr, 0,
                             nullptr, nullptr, 0, Dinv, DinvT, Sx);
  if (rc != 0) return rc;
  return info;
}

}  // namespace tchol

extern "C" {

int64_t tchol_workspace_bytes(int32_t op, int64_t n, int64_t nb, int64_t nrhs) {
  if (op != TCHOL_OP_FACTOR && op != TCHOL_OP_SOLVE && op != TCHOL_OP_BACKWARD) return -1;
  if (n < 0) return -2;
  if (!nb_ok(nb)) return -3;
  if (op == TCHOL_OP_SOLVE && nrhs < 0) return -4;
  // the factorization's workspace covers opts.inv_trsm (its DAG and inverses)
  auto plan = tchol::get_plan(op == TCHOL_OP_FACTOR ? tchol::OP_FACTOR_INVT : op, n, nb, TCHOL_POLICY_RANK, 0);
  if (!plan) return TCHOL_E_UNSUPPORTED;
  if (op == TCHOL_OP_BACKWARD) return back_layout(n, nb, *plan).end;
  // every policy yields the same task, edge and item counts, hence the same layout
  int64_t end = inv_layout(*plan, nrhs).end;
  if (op == TCHOL_OP_FACTOR) {
    auto plain = tchol::get_plan(TCHOL_OP_FACTOR, n, nb, TCHOL_POLICY_RANK, 0);
    if (!plain) return TCHOL_E_UNSUPPORTED;
    end = std::max(end, inv_layout(*plain, nrhs).end);
  }
  return end;
}

int32_t tchol_factor_ex(double* A, int64_t n, int64_t nb, void* ws, int64_t ws_bytes, void* stream,
                        const tchol_opts* opts) {
  if (n < 0) return -2;
  if (!nb_ok(nb)) return -3;
  if (n == 0) return 0;
  if (!A) return -1;
  if (!ws) return -4;
  if (ws_bytes <= 0) return -5;
  return run(TCHOL_OP_FACTOR, A, nullptr, n, nb, 0, ws, ws_bytes, stream, opts, 4);
}

int32_t tchol_factor(double* A, int64_t n, int64_t nb, void* ws, int64_t ws_bytes, void* stream) {
  return tchol_factor_ex(A, n, nb, ws, ws_bytes, stream, nullptr);
}

int32_t tchol_solve_ex(const double* L, int64_t n, int64_t nb, double* B, int64_t nrhs, void* ws, int64_t ws_bytes,
                       void* stream, const tchol_opts* opts) {
  if (n < 0) return -2;
  if (!nb_ok(nb)) return -3;
  if (nrhs < 0) return -5;
  if (n == 0 || nrhs == 0) return 0;
  if (!L) return -1;
  if (!B) return -4;
  if (!ws) return -6;
  if (ws_bytes <= 0) return -7;
  return run(TCHOL_OP_SOLVE, const_cast<double*>(L), B, n, nb, nrhs, ws, ws_bytes, stream, opts, 6);
}

int32_t tchol_solve(const double* L, int64_t n, int64_t nb, double* B, int64_t nrhs, void* ws, int64_t ws_bytes,
                    void* stream) {
  return tchol_solve_ex(L, n, nb, B, nrhs, ws, ws_bytes, stream, nullptr);
}

int32_t tchol_backward_ex(const double* L, int64_t n, int64_t nb, double* Lbar, void* ws, int64_t ws_bytes,
                          void* stream_v, const tchol_opts* opts) {
  if (n < 0) return -2;
  if (!nb_ok(nb)) return -3;
  if (n == 0) return 0;
  if (!L) return -1;
  if (!Lbar) return -4;
  if (!ws) return -5;
  if (ws_bytes <= 0) return -6;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return -5;
  const tchol_opts& o = opts ? *opts : kDefaultOpts;
  if (!policy_ok(o.policy)) return TCHOL_E_UNSUPPORTED;
  auto plan = tchol::get_plan(TCHOL_OP_BACKWARD, n, nb, o.policy, o.seed);
  if (!plan) return TCHOL_E_UNSUPPORTED;
  const BackLayout B = back_layout(n, nb, *plan);
  if (ws_bytes < B.end) return -6;
  auto img = image_of(plan);
  char* w = static_cast<char*>(ws);
  double* LT = reinterpret_cast<double*>(w + B.lt);
  double* Q = reinterpret_cast<double*>(w + B.q);
  double* slots = reinterpret_cast<double*>(w + B.slots);
  if (tchol_dev_backward_prep(L, n, LT, Q, B.ldq, B.np, reinterpret_cast<hipStream_t>(stream_v)) != hipSuccess)
    return TCHOL_E_HIP;
  return execute(*plan, *img, const_cast<double*>(L), Lbar, 0, true, false, w + B.sched, ws_bytes - B.sched,
                 stream_v, o, 5, nullptr, slots, 3, Q, LT, B.ldq, reinterpret_cast<double*>(w + B.scr),
                 reinterpret_cast<double*>(w + B.inv));
}

int32_t tchol_backward(const double* L, int64_t n, int64_t nb, double* Lbar, void* ws, int64_t ws_bytes,
                       void* stream) {
  return tchol_backward_ex(L, n, nb, Lbar, ws, ws_bytes, stream, nullptr);
}

int64_t tchol_factor_solve_workspace_bytes(int64_t n, int64_t nb, int64_t nrhs) {
  if (n < 0 || n > INT32_MAX) return -1;
  if (!nb_ok(nb)) return -2;
  if (nrhs < 0) return -3;
  return tchol::factor_solve_bytes(n, nb, nrhs, true);
}

int32_t tchol_factor_solve(double* A, int64_t n, int64_t nb, double* B, int64_t nrhs, void* ws, int64_t ws_bytes,
                           void* stream, const tchol_opts* opts) {
  if (n < 0 || n > INT32_MAX) return -2;
  if (!nb_ok(nb)) return -3;
  if (nrhs < 0 || nrhs > INT32_MAX) return -5;
  if (n == 0) return 0;
  if (!A) return -1;
  if (nrhs > 0 && !B) return -4;
  if (!ws) return -6;
  if (ws_bytes <= 0) return -7;
  return tchol::factor_solve_run(A, n, nb, B, nrhs, ws, ws_bytes, stream, opts, true, !(opts && opts->subst));
}

int64_t tchol_batched_workspace_bytes(const int32_t* n, const int32_t* nb, int32_t batch) {
  std::vector<tchol::System> systems;
  if (batch < 0) return -3;
  if (batch > 0 && !n) return -1;
  if (batch > 0 && !nb) return -2;
  const int32_t rc = batched_systems(nullptr, nullptr, nullptr, n, nb, batch, &systems);
  if (rc == -6) return -1;
  if (rc == -7) return -2;
  if (rc != 0) return rc;
  auto plan = tchol::get_batched_plan(systems, TCHOL_POLICY_RANK, 0);
  if (!plan) return TCHOL_E_UNSUPPORTED;
  // every policy yields the same task, edge and item counts, hence the same
  // layout; up to 7 more work items (8 bytes each) for every one-tile system
  // above 128 that opts.wgs may split
  int64_t extra = 0;
  for (const auto& sy : systems)
    if (sy.n > 128 && sy.nb >= sy.n) extra += 7 * 8;
  return layout_of(*plan).end + align_up(extra);
}

int32_t tchol_factor_solve_batched(double* A, const int64_t* a_off, const int32_t* lda, double* B,
                                   const int64_t* b_off, const int32_t* n, const int32_t* nb, int32_t nrhs,
                                   int32_t batch, int32_t* info, void* ws, int64_t ws_bytes, void* stream,
                                   const tchol_opts* opts) {
  if (nrhs < 0) return -8;
  if (batch < 0) return -9;
  if (batch == 0) return 0;
  if (!a_off) return -2;
  if (!lda) return -3;
  if (!b_off) return -5;
  if (!info) return -10;
  std::vector<tchol::System> systems;
  const int32_t rc = batched_systems(a_off, lda, b_off, n, nb, batch, &systems);
  if (rc != 0) return rc;
  bool any = false, wide = true;
  for (auto& sy : systems) {
    if (sy.n == 0) continue;
    any = true;
    // 16-byte transfers move rows in pairs: even ld, aligned columns, and a
    // row after the last one when the order is odd
    if (sy.ld % 2 != 0 || (reinterpret_cast<uintptr_t>(A + sy.a_off) % 16) != 0 || (sy.n % 2 != 0 && sy.ld <= sy.n))
      wide = false;
  }
  for (int32_t s = 0; s < batch; ++s) info[s] = 0;
  if (!any) return 0;
  if (!A) return -1;
  if (nrhs > 0 && !B) return -4;
  if (!ws) return -11;
  if (ws_bytes <= 0) return -12;
  const tchol_opts& o = opts ? *opts : kDefaultOpts;
  if (!policy_ok(o.policy)) return TCHOL_E_UNSUPPORTED;
  if (o.wgs) {
    for (int32_t s = 0; s < batch; ++s) {
      if (o.wgs[s] < 0 || o.wgs[s] > 8) return -14;
      systems[s].wgs = o.wgs[s];
    }
  }
  if (nrhs == 0) {
    // nothing to solve: the plan still holds the solve tasks, which then have no columns
  }
  auto plan = tchol::get_batched_plan(systems, o.policy, o.seed);
  if (!plan) return TCHOL_E_UNSUPPORTED;
  auto img = batched_image_of(plan, systems);
  // systems of one tile each, factored by one workgroup (no pooled POTRF):
  // the compact instance, two workgroups per compute unit
  bool compact = wide;
  for (int64_t t = 0; compact && t < plan->ntask(); ++t) {
    const int32_t k = plan->kind[t];
    if (!((k == TK_POTRF && plan->parts[t] == 1) || k == TK_FTRSV || k == TK_BTRSV)) compact = false;
  }
  return execute(*plan, *img, A, B, nrhs, wide, true, ws, ws_bytes, stream, o, 11, info, nullptr, compact ? 6 : 0);
}

int64_t tchol_mixed_workspace_bytes_ex(int64_t n, int64_t nb, int64_t nrhs, int32_t lowp) {
  if (n < 0) return -1;
  if (!nb_ok(nb)) return -2;
  if (nrhs < 0) return -3;
  if (lowp != TCHOL_LOWP_FP32 && lowp != TCHOL_LOWP_BF16) return -4;
  auto fp = tchol::get_plan(tchol::OP_FACTOR_INV, n, nb, TCHOL_POLICY_RANK, 0);
  auto sp = tchol::get_plan(tchol::OP_SOLVE_INV, n, nb, TCHOL_POLICY_RANK, 0);
  if (!fp || !sp) return TCHOL_E_UNSUPPORTED;
  return mixed_layout(n, nb, nrhs, *fp, *sp, lowp == TCHOL_LOWP_BF16).end;
}

int64_t tchol_mixed_workspace_bytes(int64_t n, int64_t nb, int64_t nrhs) {
  return tchol_mixed_workspace_bytes_ex(n, nb, nrhs, TCHOL_LOWP_FP32);
}

int32_t tchol_solve_mixed(const double* A, int64_t n, int64_t nb, double* B, int64_t nrhs, int32_t lowp, double tol,
                          int32_t maxit, double* berr_out, int32_t* iters_out, void* ws, int64_t ws_bytes,
                          void* stream_v, const tchol_opts* opts) {
  if (n < 0) return -2;
  if (!nb_ok(nb)) return -3;
  if (nrhs < 0) return -5;
  if (lowp != TCHOL_LOWP_FP32 && lowp != TCHOL_LOWP_BF16) return -6;
  if (!(tol > 0.0)) return -7;
  if (maxit < 0) return -8;
  if (iters_out) *iters_out = 0;
  if (n == 0 || nrhs == 0) {
    for (int64_t j = 0; j < nrhs; ++j)
      if (berr_out) berr_out[j] = 0.0;
    return 0;
  }
  if (!A) return -1;
  if (!B) return -4;
  if (!ws) return -11;
  if (ws_bytes <= 0) return -12;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return -11;
  const tchol_opts& o = opts ? *opts : kDefaultOpts;
  if (!policy_ok(o.policy)) return TCHOL_E_UNSUPPORTED;
  auto fplan = tchol::get_plan(tchol::OP_FACTOR_INV, n, nb, o.policy, o.seed);
  auto splan = tchol::get_plan(tchol::OP_SOLVE_INV, n, nb, o.policy, o.seed);
  if (!fplan || !splan) return TCHOL_E_UNSUPPORTED;
  const bool bf16 = lowp == TCHOL_LOWP_BF16;
  const MixedLayout M = mixed_layout(n, nb, nrhs, *fplan, *splan, bf16);
  if (ws_bytes < M.end) return -12;
  auto fimg = image_of(fplan, M.ldw);
  auto simg = image_of(splan, M.ldw);
  char* w = static_cast<char*>(ws);
  float* W = reinterpret_cast<float*>(w + M.w);
  double* D = reinterpret_cast<double*>(w + M.d);
  double* Dinv = reinterpret_cast<double*>(w + M.dinv);
  double* DinvT = reinterpret_cast<double*>(w + M.dinvt);
  double* Sx = reinterpret_cast<double*>(w + M.sx);
  double* Part = reinterpret_cast<double*>(w + M.part);
  double* B0 = reinterpret_cast<double*>(w + M.b0);
  double* R = reinterpret_cast<double*>(w + M.r);
  double* norms = reinterpret_cast<double*>(w + M.norms);  // {||A||, ||b_j||, ||x_j||, ||r_j||}
  void* sched = w + M.sched;
  const int64_t sched_bytes = ws_bytes - M.sched;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream_v);
  const int nr = (int)nrhs;

  // the working copy, then its factorization (FP32 updates, FP64 diagonal tiles)
  if (tchol_refine_convert(A, n, W, M.ldw, n, s) != hipSuccess) return TCHOL_E_HIP;
  if (tchol_refine_diag(A, n, n, nb, D, s) != hipSuccess) return TCHOL_E_HIP;
  const tchol_opts& fo = o;  // kernel_ms and trace describe the factorization launch
  int32_t rc = execute(*fplan, *fimg, reinterpret_cast<double*>(W), nullptr, 0, true, false, sched, sched_bytes,
                       stream_v, fo, 11, nullptr, D, bf16 ? 5 : 1, nullptr, nullptr, 0, Dinv, DinvT, nullptr,
                       bf16 ? reinterpret_cast<uint16_t*>(w + M.h) : nullptr, M.hrows);
  if (rc != 0) return rc;
  tchol_opts so = o;
  so.trace = nullptr;
  so.kernel_ms = nullptr;

  // ||A||_inf (row sums of |A|, A symmetric) and ||b_j||_inf, kept with b
  const size_t bbytes = 8 * (size_t)n * (size_t)nrhs;
  if (hipMemcpyAsync(B0, B, bbytes, hipMemcpyDeviceToDevice, s) != hipSuccess) return TCHOL_E_HIP;
  if (tchol_refine_residual(A, n, n, B0, B0, R, n, 1, 1, Part, s) != hipSuccess) return TCHOL_E_HIP;
  if (tchol_refine_colmax(R, n, n, 1, norms, s) != hipSuccess) return TCHOL_E_HIP;
  if (tchol_refine_colmax(B0, n, n, nr, norms + 1, s) != hipSuccess) return TCHOL_E_HIP;

  // x_0
  rc = execute(*splan, *simg, reinterpret_cast<double*>(W), B, nrhs, true, false, sched, sched_bytes, stream_v, so,
               11, nullptr, D, 2, nullptr, nullptr, 0, Dinv, DinvT, Sx);
  if (rc != 0) return rc;
  std::vector<double> hn(1 + 3 * (size_t)nrhs);
  for (int32_t it = 0;; ++it) {
    if (tchol_refine_residual(A, n, n, B, B0, R, n, nr, 0, Part, s) != hipSuccess) return TCHOL_E_HIP;
    if (tchol_refine_colmax(B, n, n, nr, norms + 1 + nrhs, s) != hipSuccess) return TCHOL_E_HIP;
    if (tchol_refine_colmax(R, n, n, nr, norms + 1 + 2 * nrhs, s) != hipSuccess) return TCHOL_E_HIP;
    if (hipMemcpyAsync(hn.data(), norms, 8 * hn.size(), hipMemcpyDeviceToHost, s) != hipSuccess) return TCHOL_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return TCHOL_E_HIP;
    double worst = 0.0;
    bool finite = true;
    for (int64_t j = 0; j < nrhs; ++j) {
      const double den = hn[0] * hn[1 + nrhs + j] + hn[1 + j];
      const double rn = hn[1 + 2 * nrhs + j];
      const double eta = den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
      if (!(eta == eta) || eta == INFINITY) finite = false;
      if (berr_out) berr_out[j] = eta;
      worst = std::max(worst, eta);
    }
    if (iters_out) *iters_out = it;
    if (finite && worst <= tol) return 0;
    if (it >= maxit || !finite) return TCHOL_E_NOCONV;
    // correction: R := L~^{-T} L~^{-1} R, then X += R
    rc = execute(*splan, *simg, reinterpret_cast<double*>(W), R, nrhs, true, false, sched, sched_bytes, stream_v, so,
                 11, nullptr, D, 2, nullptr, nullptr, 0, Dinv, DinvT, Sx);
    if (rc != 0) return rc;
    if (tchol_refine_axpy(B, R, n * nrhs, s) != hipSuccess) return TCHOL_E_HIP;
  }
}

int64_t tchol_batched_f32_workspace_bytes(const int32_t* n, const int32_t* nb, int32_t batch, int32_t nrhs) {
  std::vector<tchol::System> systems;
  if (batch < 0) return -3;
  if (batch > 0 && !n) return -1;
  if (batch > 0 && !nb) return -2;
  if (nrhs < 0) return -4;
  const int32_t rc = batched_systems(nullptr, nullptr, nullptr, n, nb, batch, &systems);
  if (rc == -6) return -1;
  if (rc == -7) return -2;
  if (rc != 0) return rc;
  auto plan = tchol::get_batched_plan(systems, TCHOL_POLICY_RANK, 0);
  if (!plan) return TCHOL_E_UNSUPPORTED;
  return b32_layout(&systems, nrhs, *plan).end;
}

int32_t tchol_factor_solve_batched_f32(float* A, const int64_t* a_off, const int32_t* lda, float* B,
                                       const int64_t* b_off, const int32_t* n, const int32_t* nb, int32_t nrhs,
                                       int32_t batch, int32_t* info, void* ws, int64_t ws_bytes, void* stream_v,
                                       const tchol_opts* opts) {
  if (nrhs < 0) return -8;
  if (batch < 0) return -9;
  if (batch == 0) return 0;
  if (!a_off) return -2;
  if (!lda) return -3;
  if (!b_off) return -5;
  if (!info) return -10;
  std::vector<tchol::System> systems;
  const int32_t rc0 = batched_systems(a_off, lda, b_off, n, nb, batch, &systems);
  if (rc0 != 0) return rc0;
  bool any = false;
  for (auto& sy : systems) {
    if (sy.n == 0) continue;
    any = true;
    // the FP32 tile products move four rows per 16-byte lane: ld a multiple
    // of 4, three readable rows after the order, 16-byte aligned systems
    if (sy.ld % 4 != 0 || sy.ld < sy.n + 3) return -3;
    if (sy.a_off % 4 != 0) return -2;
  }
  for (int32_t s = 0; s < batch; ++s) info[s] = 0;
  if (!any) return 0;
  if (!A || reinterpret_cast<uintptr_t>(A) % 16 != 0) return -1;
  if (nrhs > 0 && !B) return -4;
  if (!ws) return -11;
  if (ws_bytes <= 0) return -12;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return -11;
  const tchol_opts& o = opts ? *opts : kDefaultOpts;
  if (!policy_ok(o.policy)) return TCHOL_E_UNSUPPORTED;
  auto plan = tchol::get_batched_plan(systems, o.policy, o.seed);
  if (!plan) return TCHOL_E_UNSUPPORTED;
  std::vector<int64_t> desc(8 * (size_t)batch, 0);
  for (int32_t s = 0; s < batch; ++s) {
    desc[8 * s + 0] = a_off[s];
    desc[8 * s + 1] = lda[s];
    desc[8 * s + 2] = n[s];
    desc[8 * s + 3] = nb[s];
    desc[8 * s + 5] = b_off[s];
  }
  const B32Layout L = b32_layout(&systems, nrhs, *plan);  // d_off, compact b_off
  if (ws_bytes < L.end) return -12;
  for (int32_t s = 0; s < batch; ++s) {
    desc[8 * s + 4] = systems[s].d_off;
    desc[8 * s + 6] = systems[s].b_off;
  }
  // Systems of one tile each (no pooled POTRF): the compact instance for
  // FP32 storage factors each system reading its FP32 matrix, keeps L in
  // FP64 in the system's tile of D (leading dimension nb, even and 16-byte
  // aligned) for its products and solves, and writes L rounded to FP32 back;
  // only the right-hand sides are staged.
  bool compact = true;
  for (int64_t t = 0; compact && t < plan->ntask(); ++t) {
    const int32_t k = plan->kind[t];
    if (!((k == TK_POTRF && plan->parts[t] == 1) || k == TK_FTRSV || k == TK_BTRSV)) compact = false;
  }
  std::vector<tchol::System> dsys;
  if (compact) {
    dsys = systems;
    for (size_t i = 0; i < dsys.size(); ++i) {
      auto& sy = dsys[i];
      sy.ld2 = sy.ld;
      sy.d_off = sy.a_off;
      sy.a_off = systems[i].d_off;
      sy.ld = sy.nb;
      desc[8 * i + 7] = 1;
    }
  }
  auto img = batched_image_of(plan, compact ? dsys : systems);
  char* w = static_cast<char*>(ws);
  int64_t* ddesc = reinterpret_cast<int64_t*>(w + L.desc);
  double* D = reinterpret_cast<double*>(w + L.d);
  double* Bd = reinterpret_cast<double*>(w + L.bd);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream_v);
  if (hipMemcpyAsync(ddesc, desc.data(), 8 * desc.size(), hipMemcpyHostToDevice, s) != hipSuccess) return TCHOL_E_HIP;
  if (tchol_b32_prepare(ddesc, batch, A, B, D, Bd, nrhs, s) != hipSuccess) return TCHOL_E_HIP;
  const int32_t rc =
      compact ? execute(*plan, *img, D, Bd, nrhs, true, true, w + L.sched, ws_bytes - L.sched, stream_v, o, 11, info,
                        nullptr, 7, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, 0, A)
              : execute(*plan, *img, reinterpret_cast<double*>(A), Bd, nrhs, true, true, w + L.sched,
                        ws_bytes - L.sched, stream_v, o, 11, info, D, 4, nullptr, nullptr, 0, D, D, Bd);
  if (rc != 0) return rc;
  if (tchol_b32_finish(ddesc, batch, A, B, D, Bd, nrhs, s) != hipSuccess) return TCHOL_E_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return TCHOL_E_HIP;
  return 0;
}

const char* tchol_strerror(int32_t code) {
  if (code == 0) return "success";
  if (code > 0) return "matrix is not positive definite (leading minor of order `code`)";
  if (code == TCHOL_E_HIP) return "a HIP runtime call failed";
  if (code == TCHOL_E_TIMEOUT) return "a dependency wait inside the kernel exceeded its bound";
  if (code == TCHOL_E_UNSUPPORTED) return "unsupported size or option";
  if (code == TCHOL_E_INTERNAL) return "work items left unfinished at kernel exit";
  if (code == TCHOL_E_NOCONV) return "iterative refinement did not reach its tolerance";
  if (code == TCHOL_E_SCRATCH)
    return "the problem needs more scheduler scratch than the fixed array of tchol_factor_solve_noalloc holds";
  if (code < 0 && code > -100) return "invalid argument (number -code)";
  return "unknown error";
}

const char* tchol_version(void) { return "tchol 0.1 (gfx950)"; }

int32_t tchol_plan_query(int32_t op, int64_t n, int64_t nb, int32_t policy, uint32_t seed, int64_t* counts,
                         int32_t* kind, int32_t* ti, int32_t* tj, int32_t* tk, int32_t* parts, int32_t* dep0,
                         int64_t* rank, int32_t* succ_off, int32_t* succ, int32_t* item_task, int32_t* item_part) {
  if (op != TCHOL_OP_FACTOR && op != TCHOL_OP_SOLVE && op != TCHOL_OP_BACKWARD && op != TCHOL_OP_MIXED_FACTOR &&
      op != TCHOL_OP_FACTOR_SOLVE)
    return -1;
  if (n < 0 || n > INT32_MAX) return -2;
  if (!nb_ok(nb)) return -3;
  if (!policy_ok(policy)) return -4;
  std::shared_ptr<const Plan> p;
  if (op == TCHOL_OP_FACTOR_SOLVE) {
    std::vector<tchol::System> systems(1);
    systems[0].n = n;
    systems[0].nb = nb;
    p = tchol::get_batched_plan(systems, policy, seed, true);
  } else {
    p = tchol::get_plan(op == TCHOL_OP_MIXED_FACTOR ? tchol::OP_FACTOR_INV : op, n, nb, policy, seed);
  }
  if (!p) return TCHOL_E_UNSUPPORTED;
  fill_query(*p, counts, kind, ti, tj, tk, nullptr, parts, dep0, rank, succ_off, succ, item_task, item_part);
  return 0;
}

int32_t tchol_batched_plan_query(const int32_t* n, const int32_t* nb, int32_t batch, int32_t policy, uint32_t seed,
                                 const int32_t* wgs, int64_t* counts, int32_t* kind, int32_t* ti, int32_t* tj,
                                 int32_t* tk, int32_t* sys,
                                 int32_t* parts, int32_t* dep0, int64_t* rank, int32_t* succ_off, int32_t* succ,
                                 int32_t* item_task, int32_t* item_part) {
  if (batch < 0) return -3;
  if (batch > 0 && !n) return -1;
  if (batch > 0 && !nb) return -2;
  if (!policy_ok(policy)) return -4;
  std::vector<tchol::System> systems;
  const int32_t rc = batched_systems(nullptr, nullptr, nullptr, n, nb, batch, &systems);
  if (rc == -6) return -1;
  if (rc == -7) return -2;
  if (rc != 0) return rc;
  if (wgs) {
    for (int32_t s = 0; s < batch; ++s) {
      if (wgs[s] < 0 || wgs[s] > 8) return -6;
      systems[s].wgs = wgs[s];
    }
  }
  auto p = tchol::build_batched_plan(systems, policy, seed, tchol::default_split());
  if (!p) return TCHOL_E_UNSUPPORTED;
  fill_query(*p, counts, kind, ti, tj, tk, sys, parts, dep0, rank, succ_off, succ, item_task, item_part);
  return 0;
}

}  // extern "C"
