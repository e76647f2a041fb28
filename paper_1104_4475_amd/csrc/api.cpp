// C ABI of the tiled QR library (declared in include/tiledqr.h).
#include "tiledqr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "device.hpp"
#include "plan.hpp"

using tqr::DevSub;
using tqr::ExecArgs;
using tqr::ExecPlan;
using tqr::Plan;

namespace {

thread_local int g_last_hip = 0;

bool hip_ok(hipError_t e) {
  if (e != hipSuccess) {
    g_last_hip = static_cast<int>(e);
    return false;
  }
  return true;
}

#define HIP_TRY(expr)                   \
  do {                                  \
    if (!hip_ok(expr)) return TQR_EHIP; \
  } while (0)

bool nb_supported(int nb) { return nb == 32 || nb == 64 || nb == 128 || nb == 256; }
// Tile sizes that are valid for the method but have no kernels here: an
// FP64 tile of 512 is 2 MB, and the update kernels keep a column slab of a
// whole tile in registers (half the register file of a workgroup at 256).
bool nb_unsupported(int nb) { return nb == 512; }

// Device copy of an executor plan with its flags.
struct DevPlan {
  DevSub* sub = nullptr;
  int32_t* deps = nullptr;
  int32_t* flags = nullptr;
  int32_t* prog = nullptr;   // per-block progress of streamed predecessors
  int32_t* order = nullptr;
  int32_t nsub = 0;
  std::vector<int32_t> level_ptr;
  int32_t epoch = 0;

  void release() {
    if (sub) (void)hipFree(sub);
    if (deps) (void)hipFree(deps);
    if (flags) (void)hipFree(flags);
    if (prog) (void)hipFree(prog);
    if (order) (void)hipFree(order);
    sub = nullptr;
    deps = nullptr;
    flags = nullptr;
    prog = nullptr;
    order = nullptr;
  }
};

int upload(const ExecPlan& ex, DevPlan& d) {
  // The executor waits only on earlier subtasks; anything else could block.
  for (size_t t = 0; t < ex.sub.size(); ++t) {
    if (ex.sub[t].dep_begin < 0 || ex.sub[t].dep_end > static_cast<int32_t>(ex.deps.size()) ||
        ex.sub[t].dep_begin > ex.sub[t].dep_end)
      return TQR_EINVAL;
    // Entries waited for inside a subtask (stages 1 and 2) only occur on
    // panel block subtasks, which are the only ones that wait there.
    const int kd = ex.sub[t].kind;
    const bool panel_blk = (kd == tqr::K_GEQRT || kd == tqr::K_TSQRT || kd == tqr::K_TTQRT) && ex.sub[t].slab >= 0;
    for (int32_t e = ex.sub[t].dep_begin; e < ex.sub[t].dep_end; ++e) {
      const int32_t d = ex.deps[e];
      if (d < 0 || tqr::dep_index(d) >= static_cast<int32_t>(t) || tqr::dep_stage(d) == 3) return TQR_EINVAL;
      if (tqr::dep_stage(d) != 0 && !panel_blk) return TQR_EINVAL;
    }
    if (ex.sub[t].sdep >= static_cast<int32_t>(t)) return TQR_EINVAL;
    if (ex.sub[t].pdep >= 0) {
      if (ex.sub[t].pdep + ex.pblk > static_cast<int32_t>(ex.deps.size())) return TQR_EINVAL;
      for (int b = 0; b < ex.pblk; ++b) {
        const int32_t d = ex.deps[ex.sub[t].pdep + b];
        if (d < 0 || tqr::dep_index(d) >= static_cast<int32_t>(t) || tqr::dep_stage(d) != 0) return TQR_EINVAL;
      }
    }
  }
  d.nsub = static_cast<int32_t>(ex.sub.size());
  d.level_ptr = ex.level_ptr;
  const size_t ns = std::max<size_t>(1, ex.sub.size());
  const size_t nd = std::max<size_t>(1, ex.deps.size());
  if (!hip_ok(hipMalloc(&d.sub, ns * sizeof(DevSub))) || !hip_ok(hipMalloc(&d.deps, nd * sizeof(int32_t))) ||
      !hip_ok(hipMalloc(&d.flags, ns * sizeof(int32_t))) || !hip_ok(hipMalloc(&d.prog, ns * sizeof(int32_t))) ||
      !hip_ok(hipMalloc(&d.order, ns * sizeof(int32_t)))) {
    d.release();
    return TQR_ENOMEM;
  }
  static_assert(sizeof(DevSub) == sizeof(tqr::SubTask), "task record layout");
  if (!ex.sub.empty()) HIP_TRY(hipMemcpy(d.sub, ex.sub.data(), ex.sub.size() * sizeof(DevSub), hipMemcpyHostToDevice));
  if (!ex.deps.empty())
    HIP_TRY(hipMemcpy(d.deps, ex.deps.data(), ex.deps.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (!ex.level_order.empty())
    HIP_TRY(hipMemcpy(d.order, ex.level_order.data(), ex.level_order.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(d.flags, 0, ns * sizeof(int32_t)));
  HIP_TRY(hipMemset(d.prog, 0, ns * sizeof(int32_t)));
  return TQR_OK;
}

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  return cus;
}

int64_t wall_ticks_per_second() {
  static int64_t rate = 0;
  if (!rate) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      rate = static_cast<int64_t>(khz) * 1000;
    else
      rate = 100000000;
  }
  return rate;
}

bool use_level_path() {
  const char* e = std::getenv("TQR_EXEC");
  return e && std::strcmp(e, "level") == 0;
}

// Dispatch order of the executor: the start order of a list schedule
// simulated on the executor's workgroups, which starts the ready subtask of
// largest bottom level (longest remaining path through the DAG) whenever a
// workgroup is free; or (TQR_ORDER) the plain bottom-level order ("bl"), or
// the ASAP or ALAP start time.  At 10240^2 the simulated order is 6% faster
// than the bottom-level order: a subtask's ticket is taken about when it can
// run, so fewer workgroups sit waiting on subtasks that are far from ready.
int exec_order() {
  const char* e = std::getenv("TQR_ORDER");
  if (e && std::strcmp(e, "asap") == 0) return 0;
  if (e && std::strcmp(e, "alap") == 0) return 1;
  if (e && std::strcmp(e, "bl") == 0) return 2;
  return 3;
}

// Dispatch order of a batch's problems: the plain bottom-level order
// (TQR_ORDER overrides).  The simulated list schedule assumes that one
// problem has every workgroup; across 512 tall-skinny problems the
// bottom-level order is 3.7% faster (19.5 ms against 20.3 ms).  The order
// does not change any task's arithmetic.
int batch_order() { return std::getenv("TQR_ORDER") ? exec_order() : 2; }

// Per-kind task weights (GEQRT, UNMQR, TSQRT, TSMQR, TTQRT, TTMQR) for the
// priorities: measured durations on MI355X of one task (all column slabs of
// an update) in microseconds, per tile size and update precision.  Other
// tile sizes use the Table 1 flop weights.  TQR_WEIGHTS (six comma-separated
// numbers) overrides them for diagnostics.
void exec_weights(int nb, int upd, double w[6]) {
  static const double table1[6] = {4, 6, 6, 12, 2, 6};
  static const double nb256[3][6] = {{600, 364, 735, 480, 533, 412},
                                     {600, 144, 560, 212, 466, 156},
                                     {560, 110, 500, 144, 456, 122}};
  static const double nb128[6] = {199, 164, 260, 300, 213, 228};
  const double* src = table1;
  if (nb == 256 && upd >= 0 && upd < 3) src = nb256[upd];
  if (nb == 128) src = nb128;
  for (int k = 0; k < 6; ++k) w[k] = src[k];
  if (const char* e = std::getenv("TQR_WEIGHTS")) {
    double v[6];
    if (std::sscanf(e, "%lf,%lf,%lf,%lf,%lf,%lf", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == 6)
      for (int k = 0; k < 6; ++k) w[k] = v[k];
  }
}

}  // namespace

struct tqr_factors {
  tqr_opts o{};
  int p = 0, q = 0, nb = 0;
  Plan plan;
  DevPlan exec;
  std::map<int, DevPlan> apply;  // key: trans * 1024 + nslab
  double* tiles = nullptr;
  double* Tg = nullptr;
  double* Tp = nullptr;
  unsigned char* imgg = nullptr;  // low-precision reflector images (nb >= 128, upd != FP64)
  unsigned char* imgp = nullptr;
  int32_t* ctl = nullptr;  // [0] ticket, [1] executor err, [2] solve err, [3..3+8q) solve flags
  ExecPlan exec_host;      // host copy of the factorization plan (joint plans are built from it)
  DevPlan fused;           // factorization + Q^T B (16 columns) in one executor plan
  double* Bt16 = nullptr;  // packed right-hand sides of the joint plan (p row tiles of nb x 16)
  mutable int32_t solve_epoch = 0;  // advanced by every triangular solve launch
  mutable double* rinv = nullptr;   // inverses of the q diagonal tiles of R
  mutable bool rinv_ok = false;     // rinv matches the current factors
  mutable double* wn = nullptr;     // coupling tiles of the R solve
  mutable double* wnt = nullptr;    // coupling tiles of the R^T solve
  mutable double* rt = nullptr;     // tiles of R^T (q x q grid, lower part)
  mutable double* rinvt = nullptr;  // transposes of the diagonal-tile inverses
  mutable bool rt_ok = false;       // rt, rinvt match the current factors
  hipStream_t stream = nullptr;
  int grid = 1;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  int64_t* trace = nullptr;  // device, 4 per executor subtask

  ~tqr_factors() {
    if (trace) (void)hipFree(trace);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    exec.release();
    fused.release();
    if (Bt16) (void)hipFree(Bt16);
    if (rinv) (void)hipFree(rinv);
    if (rt) (void)hipFree(rt);
    if (wn) (void)hipFree(wn);
    if (wnt) (void)hipFree(wnt);
    if (rinvt) (void)hipFree(rinvt);
    for (auto& kv : apply) kv.second.release();
    if (tiles) (void)hipFree(tiles);
    if (Tg) (void)hipFree(Tg);
    if (Tp) (void)hipFree(Tp);
    if (imgg) (void)hipFree(imgg);
    if (imgp) (void)hipFree(imgp);
    if (ctl) (void)hipFree(ctl);
  }
};

// Double-complex factorization (nb = 32): tiles, tau of the GEQRT and TS/TT
// sets, the executor's subtask table and its ticket / error words.
struct tqr_zfactors {
  tqr_opts o{};
  int p = 0, q = 0, grid = 1;
  Plan plan;
  DevPlan exec;
  std::map<int, DevPlan> apply;  // Q application plans by trans * 1024 + slabs
  double* tiles = nullptr;
  double* taug = nullptr;
  double* taup = nullptr;
  int32_t* ctl = nullptr;
  hipStream_t stream = nullptr;

  ~tqr_zfactors() {
    exec.release();
    for (auto& kv : apply) kv.second.release();
    for (void* ptr : {static_cast<void*>(tiles), static_cast<void*>(taug), static_cast<void*>(taup),
                      static_cast<void*>(ctl)})
      if (ptr) (void)hipFree(ptr);
  }
};

struct tqr_batch {
  int32_t nprob = 0;
  int32_t upd = 0;
  std::vector<tqr_factors*> F;  // owned; entries handed out by tiledqr_factor_batched become null
  std::vector<int64_t> lda;
  DevPlan exec;
  tqr::ProbDesc* prob = nullptr;
  int32_t* prob_of = nullptr;
  int64_t* tile_start = nullptr;
  int64_t* lda_dev = nullptr;
  double** aptr_dev = nullptr;
  double** aptr_host = nullptr;  // pinned staging of the A pointers
  int32_t* ctl = nullptr;        // ticket, err, epoch
  int64_t** trace_slot = nullptr;  // device word: the trace buffer, or null
  int64_t* trace = nullptr;      // 4 int64 per subtask while tracing
  int64_t ntiles = 0;
  int grid = 1;
  hipStream_t cap = nullptr;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool ran = false;

  ~tqr_batch() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    exec.release();
    if (trace_slot) (void)hipFree(trace_slot);
    if (trace) (void)hipFree(trace);
    if (prob) (void)hipFree(prob);
    if (prob_of) (void)hipFree(prob_of);
    if (tile_start) (void)hipFree(tile_start);
    if (lda_dev) (void)hipFree(lda_dev);
    if (aptr_dev) (void)hipFree(aptr_dev);
    if (aptr_host) (void)hipHostFree(aptr_host);
    if (ctl) (void)hipFree(ctl);
    for (tqr_factors* f : F) delete f;
  }
};

namespace {

ExecArgs base_args(const tqr_factors* F, const DevPlan& d) {
  ExecArgs a{};
  a.tiles = F->tiles;
  a.Tg = F->Tg;
  a.Tp = F->Tp;
  a.imgg = F->imgg;
  a.imgp = F->imgp;
  a.B = nullptr;
  a.sub = d.sub;
  a.deps = d.deps;
  a.flags = d.flags;
  a.prog = d.prog;
  a.ticket = F->ctl;
  a.err = F->ctl + 1;
  a.nsub = d.nsub;
  a.p = F->p;
  a.q = F->q;
  a.nb = F->nb;
  a.ncolB = 0;
  a.transB = 1;
  a.upd = F->o.upd;
  a.spin_ticks = 4 * wall_ticks_per_second();
  a.trace = (&d == &F->exec) ? F->trace : nullptr;
  // Diagnostics: TQR_TRACE_APPLY=1 records Q-application subtasks into the
  // same trace buffer (rows 0 .. nsub - 1 of that plan).
  if (!a.trace && F->trace && d.nsub <= F->exec.nsub) {
    const char* ta = std::getenv("TQR_TRACE_APPLY");
    if (ta && ta[0] == '1') a.trace = F->trace;
  }
  const char* dbg = std::getenv("TQR_DEBUG");
  a.debug = dbg ? std::atoi(dbg) : 0;
  return a;
}

// Inverses of the diagonal tiles of R for the triangular solves, computed
// once per factorization (nullptr with TQR_TRSM_SUBST=1: substitution inside
// the diagonal tiles).
const double* diag_inverses(const tqr_factors* F, hipStream_t s, hipError_t* e) {
  *e = hipSuccess;
  const char* sub = std::getenv("TQR_TRSM_SUBST");
  if (sub && sub[0] == '1') return nullptr;
  if (F->rinv_ok) return F->rinv;
  const size_t bytes = static_cast<size_t>(F->q) * F->nb * F->nb * sizeof(double);
  if (!F->rinv) {
    *e = hipMalloc(&F->rinv, bytes);
    if (*e != hipSuccess) {
      F->rinv = nullptr;
      return nullptr;
    }
  }
  if (!F->wn) {
    *e = hipMalloc(&F->wn, 2 * bytes);  // coupling at distances 1 and 2
    if (*e != hipSuccess) {
      F->wn = nullptr;
      return nullptr;
    }
  }
  *e = tqr::launch_trinv(F->tiles, F->p, F->q, F->nb, F->rinv, s);
  if (*e == hipSuccess) *e = tqr::launch_coupling(F->tiles, nullptr, F->rinv, F->p, F->q, F->nb, 0, F->wn, s);
  F->rinv_ok = *e == hipSuccess;
  return F->rinv;
}

// X <- R^{-1} X (n x nrhs, in place) with the handle's tiled R.
hipError_t solve_r(const tqr_factors* F, double* X, int64_t ldx, int64_t nrhs, hipStream_t s) {
  hipError_t e;
  const double* ri = diag_inverses(F, s, &e);
  if (e != hipSuccess) return e;
  return tqr::launch_trsm_upper(F->tiles, ri, ri ? F->wn : nullptr, F->p, F->q, F->nb, X, ldx, nrhs, F->ctl + 3,
                                &F->solve_epoch, F->ctl + 2, 4 * wall_ticks_per_second(), s);
}

// X <- R^{-T} X (n x nrhs, in place), from the transposed tiles of R and
// of the diagonal inverses (made once per factorization) so that every
// load of the solve is coalesced.
hipError_t solve_rt(const tqr_factors* F, double* X, int64_t ldx, int64_t nrhs, hipStream_t s) {
  hipError_t e;
  const double* ri = diag_inverses(F, s, &e);
  if (e != hipSuccess) return e;
  if (ri && !F->rt_ok) {
    const size_t tile = static_cast<size_t>(F->nb) * F->nb;
    if (!F->rt) {
      e = hipMalloc(&F->rt, static_cast<size_t>(F->q) * F->q * tile * sizeof(double));
      if (e != hipSuccess) {
        F->rt = nullptr;
        return e;
      }
    }
    if (!F->rinvt) {
      e = hipMalloc(&F->rinvt, static_cast<size_t>(F->q) * tile * sizeof(double));
      if (e != hipSuccess) {
        F->rinvt = nullptr;
        return e;
      }
    }
    if (!F->wnt) {
      e = hipMalloc(&F->wnt, 2 * static_cast<size_t>(F->q) * tile * sizeof(double));  // distances 1 and 2
      if (e != hipSuccess) {
        F->wnt = nullptr;
        return e;
      }
    }
    e = tqr::launch_transpose_r(F->tiles, ri, F->p, F->q, F->nb, F->rt, F->rinvt, s);
    if (e == hipSuccess) e = tqr::launch_coupling(F->tiles, F->rt, F->rinvt, F->p, F->q, F->nb, 1, F->wnt, s);
    if (e != hipSuccess) return e;
    F->rt_ok = true;
  }
  return tqr::launch_trsm_upper_t(F->tiles, ri ? F->rt : nullptr, ri ? F->rinvt : nullptr, ri ? F->wnt : nullptr, F->p,
                                  F->q, F->nb, X, ldx, nrhs, F->ctl + 3, &F->solve_epoch, F->ctl + 2,
                                  4 * wall_ticks_per_second(), s);
}

int run_plan(tqr_factors* F, DevPlan& d, ExecArgs a, hipStream_t s) {
  if (&d == &F->exec || &d == &F->fused) F->rinv_ok = F->rt_ok = false;  // the factors change
  if (d.nsub == 0) return TQR_OK;
  a.epoch = ++d.epoch;
  if (use_level_path()) {
    HIP_TRY(tqr::launch_reset(a.ticket, a.err, s));
    const int nl = static_cast<int>(d.level_ptr.size()) - 1;
    for (int l = 0; l < nl; ++l) {
      const int b = d.level_ptr[l], c = d.level_ptr[l + 1] - b;
      if (c > 0) HIP_TRY(tqr::launch_level(a, d.order, b, c, s));
    }
    return TQR_OK;
  }
  HIP_TRY(tqr::launch_reset(a.ticket, a.err, s));
  int grid = std::max(1, std::min(d.nsub, F->grid));
  if (const char* g = std::getenv("TQR_GRID")) {
    const int want = std::atoi(g);
    if (want > 0) grid = std::min(grid, want);
  }
  HIP_TRY(tqr::launch_persistent(a, grid, s));
  return TQR_OK;
}

int check_opts(const tqr_opts* o, int64_t lda) {
  if (!o) return TQR_EINVAL;
  if (o->nb <= 0 || o->m <= 0 || o->n <= 0) return TQR_EINVAL;
  if (nb_unsupported(o->nb)) return TQR_EUNSUPPORTED;
  if (!nb_supported(o->nb)) return TQR_EINVAL;
  if (o->ib != 0 && o->ib != tqr::IB) return TQR_EINVAL;
  if (o->m % o->nb || o->n % o->nb || o->m < o->n) return TQR_EINVAL;
  if (lda < o->m) return TQR_EINVAL;
  if (o->upd < TQR_UPD_F64 || o->upd > TQR_UPD_BF16) return TQR_EINVAL;
  if (o->kernels < TQR_KERN_DEFAULT || o->kernels > TQR_KERN_TS) return TQR_EINVAL;
  const int64_t p = o->m / o->nb, q = o->n / o->nb;
  if (p > (1 << 20)) return TQR_EINVAL;
  if (!tqr::valid_shape(static_cast<int>(p), static_cast<int>(q), o->tree, o->bs)) return TQR_EINVAL;
  return TQR_OK;
}

int create(const tqr_opts* o, tqr_factors** out, ExecPlan* keep = nullptr, int order = -1) {
  std::unique_ptr<tqr_factors> F(new (std::nothrow) tqr_factors());
  if (!F) return TQR_ENOMEM;
  F->o = *o;
  F->o.ib = tqr::IB;
  F->nb = o->nb;
  F->p = static_cast<int>(o->m / o->nb);
  F->q = static_cast<int>(o->n / o->nb);
  if (!tqr::make_plan(F->p, F->q, o->tree, o->bs, o->kernels, F->plan)) return TQR_EINVAL;
  double w[6];
  exec_weights(o->nb, o->upd, w);
  ExecPlan ex;
  const int nslab = std::max(1, F->nb / tqr::update_slab(F->nb, o->upd));
  // Panel tasks as one subtask per inner block (nb >= 128; TQR_PANEL_SPLIT=0
  // keeps whole panel tasks).
  const char* ps = std::getenv("TQR_PANEL_SPLIT");
  const int pblk = (F->nb >= 128 && !(ps && ps[0] == '0')) ? F->nb / tqr::IB : 1;
  // Wide low-precision updates stream their reflectors and C1 tiles block by
  // block (TQR_STREAM=0 waits for whole predecessors instead).
  const char* sv = std::getenv("TQR_STREAM");
  const bool stream = tqr::update_slab(F->nb, o->upd) == tqr::WIDE_SLAB && !(sv && sv[0] == '0');
  // Panel block subtasks release their successors after their look-ahead
  // update (TQR_EARLY=0: only when they finish).
  const char* ev = std::getenv("TQR_EARLY");
  const bool early = pblk > 1 && !(ev && ev[0] == '0');
  const int workers = device_cus() * tqr::persistent_occupancy(o->nb, o->upd);
  tqr::make_exec_plan(F->plan, nslab, order < 0 ? exec_order() : order, w, ex, pblk, stream, early, workers);
  int st = upload(ex, F->exec);
  if (st != TQR_OK) return st;
  if (keep) *keep = ex;
  F->exec_host = std::move(ex);
  const size_t ntile = static_cast<size_t>(F->p) * F->q;
  const size_t nbb = static_cast<size_t>(F->nb);
  if (!hip_ok(hipMalloc(&F->tiles, ntile * nbb * nbb * sizeof(double))) ||
      !hip_ok(hipMalloc(&F->Tg, ntile * tqr::IB * nbb * sizeof(double))) ||
      !hip_ok(hipMalloc(&F->Tp, ntile * tqr::IB * nbb * sizeof(double))) ||
      !hip_ok(hipMalloc(&F->ctl, (3 + 8 * F->q) * sizeof(int32_t))))
    return TQR_ENOMEM;
  HIP_TRY(hipMemset(F->Tg, 0, ntile * tqr::IB * nbb * sizeof(double)));
  HIP_TRY(hipMemset(F->Tp, 0, ntile * tqr::IB * nbb * sizeof(double)));
  if (tqr::update_slab(F->nb, o->upd) == tqr::WIDE_SLAB) {
    const size_t ib = ntile * static_cast<size_t>(F->nb / tqr::IB) * tqr::image_bytes(F->nb, o->upd);
    if (!hip_ok(hipMalloc(&F->imgg, ib)) || !hip_ok(hipMalloc(&F->imgp, ib))) return TQR_ENOMEM;
  }
  HIP_TRY(hipMemset(F->ctl, 0, (3 + 8 * F->q) * sizeof(int32_t)));
  F->grid = device_cus() * tqr::persistent_occupancy(F->nb, F->o.upd);
  *out = F.release();
  return TQR_OK;
}

int factor_into(tqr_factors* F, const double* A, int64_t lda, hipStream_t s) {
  F->stream = s;
  HIP_TRY(tqr::launch_pack(A, lda, F->tiles, F->p, F->q, F->nb, s));
  if (!F->ev0) {
    HIP_TRY(hipEventCreate(&F->ev0));
    HIP_TRY(hipEventCreate(&F->ev1));
  }
  HIP_TRY(hipEventRecord(F->ev0, s));
  const int st = run_plan(F, F->exec, base_args(F, F->exec), s);
  if (st != TQR_OK) return st;
  HIP_TRY(hipEventRecord(F->ev1, s));
  F->timed = true;
  return TQR_OK;
}

DevPlan* apply_plan(tqr_factors* F, int trans, int nslab, int* st) {
  const int key = trans * 1024 + nslab;
  auto it = F->apply.find(key);
  if (it != F->apply.end()) return &it->second;
  ExecPlan ex;
  tqr::make_apply_plan(F->plan, trans, nslab, ex);
  DevPlan d;
  *st = upload(ex, d);
  if (*st != TQR_OK) return nullptr;
  return &(F->apply[key] = d);
}

// Apply Q^T / Q to the packed row tiles Bt (ncolB columns).
int apply_tiles(const tqr_factors* Fc, int trans, double* Bt, int ncolB, hipStream_t s) {
  tqr_factors* F = const_cast<tqr_factors*>(Fc);
  const int nslab = (ncolB + tqr::SLAB - 1) / tqr::SLAB;
  int st = TQR_OK;
  DevPlan* d = apply_plan(F, trans, nslab, &st);
  if (!d) return st;
  ExecArgs a = base_args(F, *d);
  a.B = Bt;
  a.ncolB = ncolB;
  a.transB = trans;
  return run_plan(F, *d, a, s);
}

// Least-squares refinement on the augmented system (Bjorck, 1967):
//   [I A; A^T 0] [r; x] = [b; 0],
// with residuals f = b - r - A x and g = -A^T r in FP64 and corrections from
// the QR factors: h = R^{-T} g, d = Q^T f, dx = R^{-1}(d_1 - h),
// dr = Q [h; d_2].  Stops when the backward error of x, the smaller of
// ||b - A x|| / (||A||_F ||x|| + ||b||) and ||A^T (b - A x)|| / (||A||_F
// ||b - A x||), is at most tol in every column, after max_iter iterations,
// or when it has not halved in three iterations (TQR_ENOTCONV).  X holds the
// initial solution on entry.  Bt: packed scratch of p row tiles x ncolB.
int refine_augmented(const tqr_factors* F, const double* A0, int64_t lda, const double* B, int64_t ldb,
                     int64_t nrhs, double* X, int64_t ldx, double tol, int max_iter, double* Bt, int ncolB,
                     tqr_refine_info* info, hipStream_t s) {
  const int64_t m = F->o.m, n = F->o.n;
  double *Rv = nullptr, *Rr = nullptr, *Z = nullptr, *H = nullptr, *D = nullptr, *nrm = nullptr, *ca = nullptr,
         *Xb = nullptr;
  auto done = [&](int code) {
    for (double* ptr : {Rv, Rr, Z, H, D, nrm, ca, Xb})
      if (ptr) (void)hipFreeAsync(ptr, s);
    return code;
  };
  const size_t mb = static_cast<size_t>(m) * nrhs * sizeof(double), nbytes = static_cast<size_t>(n) * nrhs * sizeof(double);
  if (!hip_ok(hipMallocAsync(reinterpret_cast<void**>(&Rv), mb, s)) ||
      !hip_ok(hipMallocAsync(reinterpret_cast<void**>(&Rr), mb, s)) ||
      !hip_ok(hipMallocAsync(reinterpret_cast<void**>(&Z), mb, s)) ||
      !hip_ok(hipMallocAsync(reinterpret_cast<void**>(&H), nbytes, s)) ||
      !hip_ok(hipMallocAsync(reinterpret_cast<void**>(&D), nbytes, s)) ||
      !hip_ok(hipMallocAsync(reinterpret_cast<void**>(&Xb), nbytes, s)) ||
      !hip_ok(hipMallocAsync(reinterpret_cast<void**>(&nrm), 4 * nrhs * sizeof(double), s)) ||
      !hip_ok(hipMallocAsync(reinterpret_cast<void**>(&ca), n * sizeof(double), s)))
    return done(TQR_ENOMEM);
  // ||A||_F and ||b|| once.
  std::vector<double> colA(static_cast<size_t>(n)), hb(nrhs);
  if (!hip_ok(hipMemsetAsync(ca, 0, n * sizeof(double), s)) ||
      !hip_ok(hipMemsetAsync(nrm, 0, 4 * nrhs * sizeof(double), s)) ||
      !hip_ok(tqr::launch_colnorms2(A0, lda, m, n, ca, s)) ||
      !hip_ok(tqr::launch_colnorms2(B, ldb, m, nrhs, nrm + 3 * nrhs, s)) ||
      !hip_ok(hipMemcpyAsync(colA.data(), ca, n * sizeof(double), hipMemcpyDeviceToHost, s)) ||
      !hip_ok(hipMemcpyAsync(hb.data(), nrm + 3 * nrhs, nrhs * sizeof(double), hipMemcpyDeviceToHost, s)) ||
      !hip_ok(hipStreamSynchronize(s)))
    return done(TQR_EHIP);
  double fa = 0.0;
  for (double v : colA) fa += v;
  fa = std::sqrt(fa);
  // r = b - A x
  if (!hip_ok(tqr::launch_residual(A0, lda, m, n, X, ldx, B, ldb, nrhs, Rr, m, s))) return done(TQR_EHIP);
  std::vector<double> h(3 * nrhs);
  std::vector<double> hist;
  double eta = INFINITY, best = INFINITY;
  int it = 0;
  bool conv = false;
  for (;; ++it) {
    // Rv = b - A x; backward error of x.
    if (!hip_ok(tqr::launch_residual(A0, lda, m, n, X, ldx, B, ldb, nrhs, Rv, m, s)) ||
        !hip_ok(tqr::launch_gemv_t(A0, lda, m, n, Rv, m, nrhs, D, n, 1.0, s)) ||
        !hip_ok(hipMemsetAsync(nrm, 0, 3 * nrhs * sizeof(double), s)) ||
        !hip_ok(tqr::launch_colnorms2(Rv, m, m, nrhs, nrm, s)) ||
        !hip_ok(tqr::launch_colnorms2(D, n, n, nrhs, nrm + nrhs, s)) ||
        !hip_ok(tqr::launch_colnorms2(X, ldx, n, nrhs, nrm + 2 * nrhs, s)))
      return done(TQR_EHIP);
    int32_t serr = 0;
    if (!hip_ok(hipMemcpyAsync(h.data(), nrm, 3 * nrhs * sizeof(double), hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipMemcpyAsync(&serr, F->ctl + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipStreamSynchronize(s)))
      return done(TQR_EHIP);
    if (serr) return done(TQR_EEXEC);
    eta = 0.0;
    for (int64_t c = 0; c < nrhs; ++c) {
      const double nr = std::sqrt(h[c]), natr = std::sqrt(h[nrhs + c]), nx = std::sqrt(h[2 * nrhs + c]);
      const double den_sq = fa * nx + std::sqrt(hb[c]);
      const double e_sq = den_sq > 0 ? nr / den_sq : 0.0;
      const double e_ls = (nr > 0 && fa > 0) ? natr / (fa * nr) : 0.0;
      eta = std::max(eta, std::min(e_sq, e_ls));
    }
    hist.push_back(eta);
    if (eta <= tol) {
      conv = true;
      break;
    }
    if (eta < best) {  // keep the best iterate for a non-converged return
      best = eta;
      if (!hip_ok(tqr::launch_copy_cols(X, ldx, Xb, n, n, nrhs, s))) return done(TQR_EHIP);
    }
    if (it >= max_iter) break;
    if (hist.size() > 3 && hist.back() > 0.5 * hist[hist.size() - 4]) break;
    // f = b - A x - r (in Rv), h = R^{-T} (-A^T r)
    if (!hip_ok(tqr::launch_axpy_cols(Rv, m, Rr, m, m, nrhs, s, -1.0)) ||
        !hip_ok(tqr::launch_gemv_t(A0, lda, m, n, Rr, m, nrhs, H, n, -1.0, s)) ||
        !hip_ok(solve_rt(F, H, n, nrhs, s)))
      return done(TQR_EHIP);
    // d = Q^T f (packed), Z = d
    if (!hip_ok(tqr::launch_pack_b(Rv, m, nrhs, Bt, F->p, F->nb, ncolB, s))) return done(TQR_EHIP);
    int st = apply_tiles(F, 1, Bt, ncolB, s);
    if (st != TQR_OK) return done(st);
    if (!hip_ok(tqr::launch_unpack_b(Bt, Z, m, nrhs, static_cast<int>(m), F->nb, ncolB, s))) return done(TQR_EHIP);
    // dx = R^{-1} (d_1 - h); x += dx
    if (!hip_ok(tqr::launch_copy_cols(Z, m, D, n, n, nrhs, s)) ||
        !hip_ok(tqr::launch_axpy_cols(D, n, H, n, n, nrhs, s, -1.0)) || !hip_ok(solve_r(F, D, n, nrhs, s)) ||
        !hip_ok(tqr::launch_axpy_cols(X, ldx, D, n, n, nrhs, s)))
      return done(TQR_EHIP);
    // dr = Q [h; d_2]; r += dr
    if (!hip_ok(tqr::launch_copy_cols(H, n, Z, m, n, nrhs, s)) ||
        !hip_ok(tqr::launch_pack_b(Z, m, nrhs, Bt, F->p, F->nb, ncolB, s)))
      return done(TQR_EHIP);
    st = apply_tiles(F, 0, Bt, ncolB, s);
    if (st != TQR_OK) return done(st);
    if (!hip_ok(tqr::launch_unpack_b(Bt, Z, m, nrhs, static_cast<int>(m), F->nb, ncolB, s)) ||
        !hip_ok(tqr::launch_axpy_cols(Rr, m, Z, m, m, nrhs, s)))
      return done(TQR_EHIP);
  }
  if (!conv && eta > best) {  // return the best iterate seen
    if (!hip_ok(tqr::launch_copy_cols(Xb, n, X, ldx, n, nrhs, s))) return done(TQR_EHIP);
    eta = best;
  }
  if (info) {
    info->iters = it;
    info->converged = conv ? 1 : 0;
    info->backward_err = eta;
    info->semi_normal = 0;
    info->augmented = it;
  }
  return done(conv ? TQR_OK : TQR_ENOTCONV);
}

int lstsq_impl(const tqr_factors* F, const double* A0, int64_t lda, const double* B, int64_t ldb,
               const double* QtB, int64_t ldq, int64_t nrhs, double* X, int64_t ldx, const tqr_refine* r,
               tqr_refine_info* info, void* stream);

}  // namespace

extern "C" {

const char* tiledqr_strerror(int status) {
  switch (status) {
    case TQR_OK: return "success";
    case TQR_EINVAL: return "invalid argument";
    case TQR_ENOMEM: return "out of memory";
    case TQR_EHIP: return "HIP runtime error";
    case TQR_ENOTCONV: return "refinement did not converge";
    case TQR_EUNSUPPORTED: return "unsupported configuration";
    case TQR_EEXEC: return "device executor stopped (dependency wait time limit)";
    default: return "unknown status";
  }
}

int tiledqr_last_hip_error(void) { return g_last_hip; }

int tiledqr_factor(const tqr_opts* opts, const double* A, int64_t lda, tqr_factors** F, void* stream) {
  if (!F || !A) return TQR_EINVAL;
  int st = check_opts(opts, lda);
  if (st != TQR_OK) return st;
  tqr_factors* h = nullptr;
  st = create(opts, &h);
  if (st != TQR_OK) return st;
  st = factor_into(h, A, lda, static_cast<hipStream_t>(stream));
  if (st != TQR_OK) {
    delete h;
    return st;
  }
  *F = h;
  return TQR_OK;
}

int tiledqr_refactor(tqr_factors* F, const double* A, int64_t lda, void* stream) {
  if (!F || !A || lda < F->o.m) return TQR_EINVAL;
  return factor_into(F, A, lda, static_cast<hipStream_t>(stream));
}

int tiledqr_sync(tqr_factors* F) {
  if (!F) return TQR_EINVAL;
  HIP_TRY(hipStreamSynchronize(F->stream));
  int32_t err = 0;
  int32_t errs[2] = {0, 0};
  HIP_TRY(hipMemcpy(errs, F->ctl + 1, 2 * sizeof(int32_t), hipMemcpyDeviceToHost));
  return (errs[0] || errs[1]) ? TQR_EEXEC : TQR_OK;
}

int tiledqr_exec_time(tqr_factors* F, float* ms) {
  if (!F || !ms || !F->timed) return TQR_EINVAL;
  HIP_TRY(hipEventSynchronize(F->ev1));
  HIP_TRY(hipEventElapsedTime(ms, F->ev0, F->ev1));
  return TQR_OK;
}

int tiledqr_set_trace(tqr_factors* F, int enable) {
  if (!F) return TQR_EINVAL;
  if (enable && !F->trace) {
    const size_t bytes = 4 * sizeof(int64_t) * std::max<int32_t>(1, F->exec.nsub);
    if (!hip_ok(hipMalloc(&F->trace, bytes))) return TQR_ENOMEM;
    HIP_TRY(hipMemset(F->trace, 0, bytes));
  } else if (!enable && F->trace) {
    HIP_TRY(hipStreamSynchronize(F->stream));
    HIP_TRY(hipFree(F->trace));
    F->trace = nullptr;
  }
  return TQR_OK;
}

int tiledqr_get_trace(tqr_factors* F, int64_t* out, int64_t* n, double* ticks_per_second) {
  if (!F || !n) return TQR_EINVAL;
  *n = F->exec.nsub;
  if (ticks_per_second) *ticks_per_second = static_cast<double>(wall_ticks_per_second());
  if (!out) return TQR_OK;
  if (!F->trace) return TQR_EINVAL;
  HIP_TRY(hipStreamSynchronize(F->stream));
  std::vector<int64_t> t(4 * static_cast<size_t>(F->exec.nsub));
  std::vector<DevSub> sub(F->exec.nsub);
  HIP_TRY(hipMemcpy(t.data(), F->trace, t.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(sub.data(), F->exec.sub, sub.size() * sizeof(DevSub), hipMemcpyDeviceToHost));
  for (int32_t s = 0; s < F->exec.nsub; ++s) {
    int64_t* o = out + 10 * static_cast<int64_t>(s);
    o[0] = sub[s].kind;
    o[1] = sub[s].i;
    o[2] = sub[s].piv;
    o[3] = sub[s].k;
    o[4] = sub[s].j;
    o[5] = sub[s].slab;
    o[6] = t[4 * s];
    o[7] = t[4 * s + 1];
    o[8] = t[4 * s + 2];
    o[9] = t[4 * s + 3];
  }
  return TQR_OK;
}

int tiledqr_exec_plan(const tqr_factors* F, int32_t* sub, int64_t* nsub, int32_t* deps, int64_t* ndeps) {
  if (!F || !nsub || !ndeps) return TQR_EINVAL;
  const tqr::ExecPlan& ex = F->exec_host;
  *nsub = static_cast<int64_t>(ex.sub.size());
  *ndeps = static_cast<int64_t>(ex.deps.size());
  if (sub)
    for (size_t t = 0; t < ex.sub.size(); ++t) {
      const tqr::SubTask& st = ex.sub[t];
      int32_t* o = sub + 10 * t;
      o[0] = st.kind;
      o[1] = st.i;
      o[2] = st.piv;
      o[3] = st.k;
      o[4] = st.j;
      o[5] = st.slab;
      o[6] = st.dep_begin;
      o[7] = st.dep_end;
      o[8] = st.sdep;
      o[9] = st.pdep;
    }
  if (deps) std::copy(ex.deps.begin(), ex.deps.end(), deps);
  return TQR_OK;
}

int tiledqr_solve_r(const tqr_factors* F, char trans, double* X, int64_t ldx, int64_t nrhs, void* stream) {
  if (!F || (!X && nrhs > 0) || ldx < F->o.n || nrhs < 0 || nrhs > (1 << 20)) return TQR_EINVAL;
  const bool t = trans == 'T' || trans == 't';
  if (!t && trans != 'N' && trans != 'n') return TQR_EINVAL;
  if (nrhs == 0) return TQR_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(t ? solve_rt(F, X, ldx, nrhs, s) : solve_r(F, X, ldx, nrhs, s));
  return TQR_OK;
}

int tiledqr_destroy(tqr_factors* F) {
  if (!F) return TQR_OK;
  (void)hipStreamSynchronize(F->stream);
  delete F;
  return TQR_OK;
}

int tiledqr_get_r(const tqr_factors* F, double* R, int64_t ldr, void* stream) {
  if (!F || !R || ldr < F->o.n) return TQR_EINVAL;
  HIP_TRY(tqr::launch_unpack(F->tiles, R, ldr, F->p, F->q, F->nb, static_cast<int>(F->o.n),
                             static_cast<int>(F->o.n), 1, static_cast<hipStream_t>(stream)));
  return TQR_OK;
}

int tiledqr_get_packed(const tqr_factors* F, double* out, int64_t ld, void* stream) {
  if (!F || !out || ld < F->o.m) return TQR_EINVAL;
  HIP_TRY(tqr::launch_unpack(F->tiles, out, ld, F->p, F->q, F->nb, static_cast<int>(F->o.m),
                             static_cast<int>(F->o.n), 0, static_cast<hipStream_t>(stream)));
  return TQR_OK;
}

int tiledqr_get_tau(const tqr_factors* F, double* tau, void* stream) {
  if (!F || !tau) return TQR_EINVAL;
  HIP_TRY(tqr::launch_tau(F->Tg, F->Tp, tau, F->p, F->q, F->nb, static_cast<hipStream_t>(stream)));
  return TQR_OK;
}

int tiledqr_apply_q(const tqr_factors* F, char trans, double* B, int64_t ldb, int64_t nrhs, void* stream) {
  if (!F || (!B && nrhs > 0) || ldb < F->o.m || nrhs < 0) return TQR_EINVAL;
  if (trans != 'T' && trans != 'N' && trans != 't' && trans != 'n') return TQR_EINVAL;
  if (nrhs == 0) return TQR_OK;
  if (nrhs > (1 << 20)) return TQR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ncolB = static_cast<int>((nrhs + 15) / 16 * 16);
  double* Bt = nullptr;
  if (!hip_ok(hipMallocAsync(reinterpret_cast<void**>(&Bt),
                             static_cast<size_t>(F->p) * F->nb * ncolB * sizeof(double), s)))
    return TQR_ENOMEM;
  int st = TQR_OK;
  if (!hip_ok(tqr::launch_pack_b(B, ldb, nrhs, Bt, F->p, F->nb, ncolB, s))) st = TQR_EHIP;
  if (st == TQR_OK) st = apply_tiles(F, (trans == 'T' || trans == 't') ? 1 : 0, Bt, ncolB, s);
  if (st == TQR_OK && !hip_ok(tqr::launch_unpack_b(Bt, B, ldb, nrhs, static_cast<int>(F->o.m), F->nb, ncolB, s)))
    st = TQR_EHIP;
  (void)hipFreeAsync(Bt, s);
  return st;
}

int tiledqr_elim_list(int32_t p, int32_t q, int32_t tree, int32_t bs, int32_t* out, int64_t* nelim) {
  if (!nelim) return TQR_EINVAL;
  std::vector<tqr::Elim> el;
  if (!tqr::make_elims(p, q, tree, bs, el)) return TQR_EINVAL;
  *nelim = static_cast<int64_t>(el.size());
  if (out)
    for (size_t e = 0; e < el.size(); ++e) {
      out[3 * e] = el[e].i;
      out[3 * e + 1] = el[e].piv;
      out[3 * e + 2] = el[e].k;
    }
  return TQR_OK;
}

int tiledqr_schedule(int32_t p, int32_t q, int32_t tree, int32_t bs, int32_t kernels, int32_t* tasks,
                     int64_t* ntasks, int64_t* cp) {
  if (!ntasks) return TQR_EINVAL;
  if (kernels < TQR_KERN_DEFAULT || kernels > TQR_KERN_TS) return TQR_EINVAL;
  Plan pl;
  if (!tqr::make_plan(p, q, tree, bs, kernels, pl)) return TQR_EINVAL;
  *ntasks = static_cast<int64_t>(pl.tasks.size());
  if (cp) *cp = pl.cp;
  if (tasks)
    for (size_t t = 0; t < pl.tasks.size(); ++t) {
      const tqr::Task& k = pl.tasks[t];
      int32_t* o = tasks + 7 * t;
      o[0] = k.kind;
      o[1] = k.i;
      o[2] = k.piv;
      o[3] = k.k;
      o[4] = k.j;
      o[5] = static_cast<int32_t>(pl.start[t]);
      o[6] = static_cast<int32_t>(pl.finish[t]);
    }
  return TQR_OK;
}

int tiledqr_task_preds(int32_t p, int32_t q, int32_t tree, int32_t bs, int32_t kernels, int64_t* ptr, int32_t* idx) {
  if (!ptr) return TQR_EINVAL;
  if (kernels < TQR_KERN_DEFAULT || kernels > TQR_KERN_TS) return TQR_EINVAL;
  Plan pl;
  if (!tqr::make_plan(p, q, tree, bs, kernels, pl)) return TQR_EINVAL;
  std::copy(pl.pred_ptr.begin(), pl.pred_ptr.end(), ptr);
  if (idx) std::copy(pl.pred_idx.begin(), pl.pred_idx.end(), idx);
  return TQR_OK;
}

int tiledqr_lstsq(const tqr_factors* F, const double* A0, int64_t lda, const double* B, int64_t ldb, int64_t nrhs,
                  double* X, int64_t ldx, const tqr_refine* r, tqr_refine_info* info, void* stream) {
  return lstsq_impl(F, A0, lda, B, ldb, nullptr, 0, nrhs, X, ldx, r, info, stream);
}

int tiledqr_lstsq_qtb(const tqr_factors* F, const double* A0, int64_t lda, const double* B, int64_t ldb,
                      const double* QtB, int64_t ldq, int64_t nrhs, double* X, int64_t ldx, const tqr_refine* r,
                      tqr_refine_info* info, void* stream) {
  if (!F || !QtB || ldq < F->o.n) return TQR_EINVAL;
  return lstsq_impl(F, A0, lda, B, ldb, QtB, ldq, nrhs, X, ldx, r, info, stream);
}

int tiledqr_zrefactor(tqr_zfactors* F, const double* A, int64_t lda, void* stream);

int tiledqr_zfactor(const tqr_opts* o, const double* A, int64_t lda, tqr_zfactors** out, void* stream) {
  if (!out) return TQR_EINVAL;
  *out = nullptr;
  const int st0 = check_opts(o, lda);
  if (st0 != TQR_OK) return st0;
  if (o->nb != 32) return TQR_EUNSUPPORTED;
  if (o->upd != TQR_UPD_F64 || !A) return TQR_EINVAL;
  std::unique_ptr<tqr_zfactors> F(new (std::nothrow) tqr_zfactors());
  if (!F) return TQR_ENOMEM;
  F->o = *o;
  F->o.ib = tqr::IB;
  F->p = static_cast<int>(o->m / 32);
  F->q = static_cast<int>(o->n / 32);
  if (!tqr::make_plan(F->p, F->q, o->tree, o->bs, o->kernels, F->plan)) return TQR_EINVAL;
  double w[6];
  exec_weights(32, TQR_UPD_F64, w);
  F->grid = device_cus() * tqr::zqr_occupancy();
  ExecPlan ex;
  tqr::make_exec_plan(F->plan, 1, exec_order(), w, ex, 1, false, false, F->grid);
  int st = upload(ex, F->exec);
  if (st != TQR_OK) return st;
  const size_t ntile = static_cast<size_t>(F->p) * F->q;
  if (!hip_ok(hipMalloc(&F->tiles, ntile * 32 * 32 * 16)) || !hip_ok(hipMalloc(&F->taug, ntile * 32 * 16)) ||
      !hip_ok(hipMalloc(&F->taup, ntile * 32 * 16)) || !hip_ok(hipMalloc(&F->ctl, 2 * sizeof(int32_t))))
    return TQR_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemsetAsync(F->taug, 0, ntile * 32 * 16, s));
  HIP_TRY(hipMemsetAsync(F->taup, 0, ntile * 32 * 16, s));
  F->stream = s;
  st = tiledqr_zrefactor(F.get(), A, lda, stream);
  if (st != TQR_OK) return st;
  *out = F.release();
  return TQR_OK;
}

int tiledqr_zrefactor(tqr_zfactors* F, const double* A, int64_t lda, void* stream) {
  if (!F || !A || lda < F->o.m) return TQR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  F->stream = s;
  HIP_TRY(tqr::launch_zpack(const_cast<double*>(A), lda, F->tiles, F->p, F->q, false, s));
  if (F->exec.nsub > 0) {
    const int epoch = ++F->exec.epoch;
    HIP_TRY(tqr::launch_zqr(F->tiles, F->taug, F->taup, F->exec.sub, F->exec.deps, F->exec.flags, F->ctl,
                            F->exec.nsub, epoch, F->p, 4 * wall_ticks_per_second(),
                            std::max(1, std::min(F->exec.nsub, F->grid)), s));
  }
  return TQR_OK;
}

int tiledqr_zapply_q(tqr_zfactors* F, char trans, double* B, int64_t ldb, int64_t nrhs, void* stream) {
  if (!F || !B || nrhs < 1 || ldb < F->o.m || (trans != 'C' && trans != 'N')) return TQR_EINVAL;
  if (nrhs > 4096) return TQR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int tr = trans == 'C' ? 1 : 0;
  const int ncolB = static_cast<int>((nrhs + 31) / 32 * 32), nslab = ncolB / 32;
  const int key = tr * 1024 + nslab;
  auto it = F->apply.find(key);
  if (it == F->apply.end()) {
    ExecPlan ex;
    tqr::make_apply_plan(F->plan, tr, nslab, ex);
    DevPlan d;
    const int st = upload(ex, d);
    if (st != TQR_OK) return st;
    it = F->apply.emplace(key, d).first;
  }
  DevPlan& d = it->second;
  double* Bt = nullptr;
  const size_t bytes = static_cast<size_t>(F->p) * 32 * ncolB * 16;
  if (!hip_ok(hipMallocAsync(reinterpret_cast<void**>(&Bt), bytes, s))) return TQR_ENOMEM;
  F->stream = s;
  hipError_t e = tqr::launch_zpack_b(B, ldb, nrhs, Bt, F->p, ncolB, false, s);
  if (e == hipSuccess && d.nsub > 0)
    e = tqr::launch_zqr(F->tiles, F->taug, F->taup, d.sub, d.deps, d.flags, F->ctl, d.nsub, ++d.epoch, F->p,
                        4 * wall_ticks_per_second(), std::max(1, std::min(d.nsub, F->grid)), s, Bt, ncolB, tr);
  if (e == hipSuccess) e = tqr::launch_zpack_b(B, ldb, nrhs, Bt, F->p, ncolB, true, s);
  (void)hipFreeAsync(Bt, s);
  return hip_ok(e) ? TQR_OK : TQR_EHIP;
}

int tiledqr_zsolve_r(const tqr_zfactors* F, double* X, int64_t ldx, int64_t nrhs, void* stream) {
  if (!F || !X || ldx < F->o.n || nrhs < 1 || F->o.n > 4096) return TQR_EINVAL;
  HIP_TRY(tqr::launch_zsolve_r(F->tiles, F->p, static_cast<int>(F->o.n), X, ldx, nrhs,
                               static_cast<hipStream_t>(stream)));
  return TQR_OK;
}

int tiledqr_zlstsq(tqr_zfactors* F, const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
                   void* stream) {
  if (!F || !B || !X || nrhs < 1 || ldb < F->o.m || ldx < F->o.n || F->o.n > 4096) return TQR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t m = F->o.m, n = F->o.n;
  double* W = nullptr;
  if (!hip_ok(hipMallocAsync(reinterpret_cast<void**>(&W), static_cast<size_t>(m) * nrhs * 16, s))) return TQR_ENOMEM;
  auto done = [&](int code) {
    (void)hipFreeAsync(W, s);
    return code;
  };
  if (!hip_ok(hipMemcpy2DAsync(W, m * 16, B, ldb * 16, m * 16, nrhs, hipMemcpyDeviceToDevice, s)))
    return done(TQR_EHIP);
  const int st = tiledqr_zapply_q(F, 'C', W, m, nrhs, stream);
  if (st != TQR_OK) return done(st);
  if (!hip_ok(hipMemcpy2DAsync(X, ldx * 16, W, m * 16, n * 16, nrhs, hipMemcpyDeviceToDevice, s)) ||
      !hip_ok(tqr::launch_zsolve_r(F->tiles, F->p, static_cast<int>(n), X, ldx, nrhs, s)))
    return done(TQR_EHIP);
  return done(TQR_OK);
}

int tiledqr_zget_packed(const tqr_zfactors* F, double* out, int64_t ld, void* stream) {
  if (!F || !out || ld < F->o.m) return TQR_EINVAL;
  HIP_TRY(tqr::launch_zpack(out, ld, F->tiles, F->p, F->q, true, static_cast<hipStream_t>(stream)));
  return TQR_OK;
}

int tiledqr_zget_tau(const tqr_zfactors* F, double* taug, double* taup, void* stream) {
  if (!F || !taug || !taup) return TQR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bytes = static_cast<size_t>(F->p) * F->q * 32 * 16;
  HIP_TRY(hipMemcpyAsync(taug, F->taug, bytes, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(taup, F->taup, bytes, hipMemcpyDeviceToDevice, s));
  return TQR_OK;
}

int tiledqr_zsync(tqr_zfactors* F) {
  if (!F) return TQR_EINVAL;
  HIP_TRY(hipStreamSynchronize(F->stream));
  int32_t err = 0;
  HIP_TRY(hipMemcpy(&err, F->ctl + 1, sizeof(int32_t), hipMemcpyDeviceToHost));
  return err ? TQR_EEXEC : TQR_OK;
}

int tiledqr_zdestroy(tqr_zfactors* F) {
  if (!F) return TQR_OK;
  (void)hipStreamSynchronize(F->stream);
  delete F;
  return TQR_OK;
}

int tiledqr_refactor_qtb(tqr_factors* F, const double* A, int64_t lda, double* B, int64_t ldb, int64_t nrhs,
                         void* stream) {
  if (!F || !A || lda < F->o.m || !B || ldb < F->o.m || nrhs < 1 || nrhs > 16) return TQR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!F->fused.sub) {
    double w[6];
    exec_weights(F->nb, F->o.upd, w);
    const int nslab = std::max(1, F->nb / tqr::update_slab(F->nb, F->o.upd));
    ExecPlan ex;
    tqr::make_factor_apply_plan(F->plan, F->exec_host, nslab, 1, 0.1 * w[1], ex);
    const int st = upload(ex, F->fused);
    if (st != TQR_OK) return st;
    if (!hip_ok(hipMalloc(&F->Bt16, static_cast<size_t>(F->p) * F->nb * 16 * sizeof(double)))) return TQR_ENOMEM;
  }
  F->stream = s;
  HIP_TRY(tqr::launch_pack(A, lda, F->tiles, F->p, F->q, F->nb, s));
  HIP_TRY(tqr::launch_pack_b(B, ldb, nrhs, F->Bt16, F->p, F->nb, 16, s));
  if (!F->ev0) {
    HIP_TRY(hipEventCreate(&F->ev0));
    HIP_TRY(hipEventCreate(&F->ev1));
  }
  ExecArgs a = base_args(F, F->fused);
  a.B = F->Bt16;
  a.ncolB = 16;
  a.transB = 1;
  a.fused = 1;
  HIP_TRY(hipEventRecord(F->ev0, s));
  const int st = run_plan(F, F->fused, a, s);
  if (st != TQR_OK) return st;
  HIP_TRY(hipEventRecord(F->ev1, s));
  F->timed = true;
  HIP_TRY(tqr::launch_unpack_b(F->Bt16, B, ldb, nrhs, static_cast<int>(F->o.m), F->nb, 16, s));
  return TQR_OK;
}

}  // extern "C"

namespace {

int lstsq_impl(const tqr_factors* F, const double* A0, int64_t lda, const double* B, int64_t ldb,
               const double* QtB, int64_t ldq, int64_t nrhs, double* X, int64_t ldx, const tqr_refine* r,
               tqr_refine_info* info, void* stream) {
  if (!F || !B || !X || nrhs < 1 || ldb < F->o.m || ldx < F->o.n) return TQR_EINVAL;
  const bool refine = r && r->tol > 0.0;
  if (refine && (!A0 || lda < F->o.m)) return TQR_EINVAL;
  if (nrhs > 4096) return TQR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t m = F->o.m, n = F->o.n;
  const int ncolB = static_cast<int>((nrhs + 15) / 16 * 16);
  const size_t bt_elems = static_cast<size_t>(F->p) * F->nb * ncolB;
  double *Bt = nullptr, *Rv = nullptr, *D = nullptr, *nrm = nullptr, *Xp = nullptr, *Xb = nullptr;
  int st = TQR_OK;
  auto fail = [&](int code) {
    for (double* ptr : {Bt, Rv, D, nrm, Xp, Xb})
      if (ptr) (void)hipFreeAsync(ptr, s);
    return code;
  };
  if (!hip_ok(hipMallocAsync(reinterpret_cast<void**>(&Bt), bt_elems * sizeof(double), s))) return fail(TQR_ENOMEM);
  // X = R^{-1} (Q^T B)(1:n)
  if (QtB) {
    if (!hip_ok(tqr::launch_copy_cols(QtB, ldq, X, ldx, n, nrhs, s))) return fail(TQR_EHIP);
  } else {
    if (!hip_ok(tqr::launch_pack_b(B, ldb, nrhs, Bt, F->p, F->nb, ncolB, s))) return fail(TQR_EHIP);
    st = apply_tiles(F, 1, Bt, ncolB, s);
    if (st != TQR_OK) return fail(st);
    if (!hip_ok(tqr::launch_unpack_b(Bt, X, ldx, nrhs, static_cast<int>(n), F->nb, ncolB, s))) return fail(TQR_EHIP);
  }
  if (!hip_ok(solve_r(F, X, ldx, nrhs, s))) return fail(TQR_EHIP);
  if (!refine) {
    if (info) {
      info->iters = 0;
      info->converged = 1;
      info->backward_err = -1.0;
      info->semi_normal = 0;
      info->augmented = 0;
    }
    return fail(TQR_OK);
  }
  const int max_iter = r->max_iter > 0 ? r->max_iter : 30;
  const bool tall = m != n;
  // Tall systems: semi-normal corrections (methods 0 and 3), with the
  // augmented system taking over for method 0; methods 1 and 2: the
  // augmented system.
  if (r->method == 2 || (tall && r->method != 0 && r->method != 3)) {
    st = refine_augmented(F, A0, lda, B, ldb, nrhs, X, ldx, r->tol, max_iter, Bt, ncolB, info, s);
    return fail(st);
  }
  const size_t rv_elems = static_cast<size_t>(m) * nrhs;
  const size_t nx_bytes = static_cast<size_t>(n) * nrhs * sizeof(double);
  if (!hip_ok(hipMallocAsync(reinterpret_cast<void**>(&Rv), rv_elems * sizeof(double), s)) ||
      !hip_ok(hipMallocAsync(reinterpret_cast<void**>(&D), nx_bytes, s)) ||
      !hip_ok(hipMallocAsync(reinterpret_cast<void**>(&Xp), nx_bytes, s)) ||
      !hip_ok(hipMallocAsync(reinterpret_cast<void**>(&Xb), nx_bytes, s)) ||
      !hip_ok(hipMallocAsync(reinterpret_cast<void**>(&nrm), (4 * nrhs + 1) * sizeof(double), s)))
    return fail(TQR_ENOMEM);
  // Corrections: semi-normal (method 3, and method 0 while each one cuts
  // the backward error at least fourfold) or, after that, classical with Q
  // (square) or the augmented system (tall).
  bool semi = r->method == 0 || r->method == 3;
  // nrm: ||r||^2, ||x||^2, ||b||^2 (once), ||A^T r||^2 (tall) per column,
  // then ||A||_F^2 (from the first residual, which reads all of A).
  if (!hip_ok(hipMemsetAsync(nrm, 0, (4 * nrhs + 1) * sizeof(double), s)) ||
      !hip_ok(tqr::launch_colnorms2(B, ldb, m, nrhs, nrm + 2 * nrhs, s)))
    return fail(TQR_EHIP);
  std::vector<double> h(4 * nrhs + 1);
  double fa = 0.0;
  double best = INFINITY, eta = INFINITY;
  std::vector<double> hist;
  int it = 0, nsemi = 0;
  bool conv = false;
  for (;; ++it) {
    // residual and norms (tall: also A^T r into D, used by the correction)
    if (!hip_ok(tqr::launch_residual(A0, lda, m, n, X, ldx, B, ldb, nrhs, Rv, m, s, it == 0 ? nrm + 4 * nrhs : nullptr)))
      return fail(TQR_EHIP);
    if (!hip_ok(hipMemsetAsync(nrm, 0, 2 * nrhs * sizeof(double), s))) return fail(TQR_EHIP);
    if (!hip_ok(tqr::launch_colnorms2(Rv, m, m, nrhs, nrm, s)) ||
        !hip_ok(tqr::launch_colnorms2(X, ldx, n, nrhs, nrm + nrhs, s)))
      return fail(TQR_EHIP);
    if (tall && (!hip_ok(tqr::launch_gemv_t(A0, lda, m, n, Rv, m, nrhs, D, n, 1.0, s)) ||
                 !hip_ok(hipMemsetAsync(nrm + 3 * nrhs, 0, nrhs * sizeof(double), s)) ||
                 !hip_ok(tqr::launch_colnorms2(D, n, n, nrhs, nrm + 3 * nrhs, s))))
      return fail(TQR_EHIP);
    int32_t serr = 0;
    if (!hip_ok(hipMemcpyAsync(h.data(), nrm, (4 * nrhs + 1) * sizeof(double), hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipMemcpyAsync(&serr, F->ctl + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipStreamSynchronize(s)))
      return fail(TQR_EHIP);
    if (serr) return fail(TQR_EEXEC);
    if (it == 0) fa = std::sqrt(h[4 * nrhs]);
    eta = 0.0;
    for (int64_t c = 0; c < nrhs; ++c) {
      const double nr = std::sqrt(h[c]);
      const double den = fa * std::sqrt(h[nrhs + c]) + std::sqrt(h[2 * nrhs + c]);
      double e = den > 0 ? nr / den : 0.0;
      // tall: the smaller of that and ||A^T r|| / (||A|| ||r||), as in the
      // augmented refinement
      if (tall && nr > 0 && fa > 0) e = std::min(e, std::sqrt(h[3 * nrhs + c]) / (fa * nr));
      eta = std::max(eta, e);
    }
    hist.push_back(eta);
    if (eta <= r->tol) {
      conv = true;
      break;
    }
    if (semi && r->method == 0 && hist.size() >= 2 && eta > 0.25 * hist[hist.size() - 2]) {
      semi = false;
      const bool undo = eta > hist[hist.size() - 2];
      if (undo) {
        // The last semi-normal step did not help: back to its starting
        // point, then classical corrections.
        hist.pop_back();
        eta = hist.back();
        --nsemi;
        if (!hip_ok(tqr::launch_copy_cols(Xp, n, X, ldx, n, nrhs, s))) return fail(TQR_EHIP);
      }
      if (tall) {
        // The augmented system from here, with the iterations left (it
        // keeps the best of its own iterates, the first of which is this
        // one, the best so far).
        st = refine_augmented(F, A0, lda, B, ldb, nrhs, X, ldx, r->tol, std::max(1, max_iter - it), Bt, ncolB,
                              info, s);
        if (info) {
          info->iters += it;
          info->semi_normal = nsemi;
        }
        return fail(st);
      }
      if (undo) continue;
    }
    if (eta < best) {  // keep the best iterate for a non-converged return
      best = eta;
      if (!hip_ok(tqr::launch_copy_cols(X, ldx, Xb, n, n, nrhs, s))) return fail(TQR_EHIP);
    }
    if (it >= max_iter) break;
    if (hist.size() > 3 && hist.back() > 0.5 * hist[hist.size() - 4]) break;
    if (semi) {
      // Semi-normal correction D = R^{-1} R^{-T} A^T Rv (A = QR gives
      // R^{-T} A^T = Q^T); X += D.
      if (r->method == 0 && !hip_ok(tqr::launch_copy_cols(X, ldx, Xp, n, n, nrhs, s))) return fail(TQR_EHIP);
      if ((!tall && !hip_ok(tqr::launch_gemv_t(A0, lda, m, n, Rv, m, nrhs, D, n, 1.0, s))) ||
          !hip_ok(solve_rt(F, D, n, nrhs, s)) || !hip_ok(solve_r(F, D, n, nrhs, s)) ||
          !hip_ok(tqr::launch_axpy_cols(X, ldx, D, n, n, nrhs, s)))
        return fail(TQR_EHIP);
      ++nsemi;
      continue;
    }
    if (tall) break;  // method 3 only: no classical step for tall systems
    // correction D = R^{-1} (Q^T Rv)(1:n); X += D
    if (!hip_ok(tqr::launch_pack_b(Rv, m, nrhs, Bt, F->p, F->nb, ncolB, s))) return fail(TQR_EHIP);
    st = apply_tiles(F, 1, Bt, ncolB, s);
    if (st != TQR_OK) return fail(st);
    if (!hip_ok(tqr::launch_unpack_b(Bt, D, n, nrhs, static_cast<int>(n), F->nb, ncolB, s)) ||
        !hip_ok(solve_r(F, D, n, nrhs, s)) ||
        !hip_ok(tqr::launch_axpy_cols(X, ldx, D, n, n, nrhs, s)))
      return fail(TQR_EHIP);
  }
  if (!conv && eta > best) {  // return the best iterate seen
    if (!hip_ok(tqr::launch_copy_cols(Xb, n, X, ldx, n, nrhs, s))) return fail(TQR_EHIP);
    eta = best;
  }
  if (info) {
    info->iters = it;
    info->converged = conv ? 1 : 0;
    info->backward_err = eta;
    info->semi_normal = nsemi;
    info->augmented = 0;
  }
  return fail(conv ? TQR_OK : TQR_ENOTCONV);
}

}  // namespace

extern "C" {

int tiledqr_batch_create(int32_t nprob, const tqr_opts* opts, const int64_t* lda, tqr_batch** out) {
  if (!out || nprob < 1 || !opts || !lda) return TQR_EINVAL;
  *out = nullptr;
  for (int32_t i = 0; i < nprob; ++i) {
    const int st = check_opts(opts + i, lda[i]);
    if (st != TQR_OK) return st;
    if (opts[i].nb != 32 && opts[i].nb != 64) return TQR_EUNSUPPORTED;
    if (opts[i].upd != opts[0].upd) return TQR_EINVAL;
  }
  std::unique_ptr<tqr_batch> b(new (std::nothrow) tqr_batch());
  if (!b) return TQR_ENOMEM;
  b->nprob = nprob;
  b->upd = opts[0].upd;
  b->lda.assign(lda, lda + nprob);
  // Per-problem handles (tile storage, T factors, apply plans) and their
  // executor plans, merged into one priority order.  Within a problem a
  // predecessor has a strictly smaller key than its successors (positive
  // weights), so the merged order keeps every dependency pointing backwards.
  std::vector<ExecPlan> plans(nprob);
  std::vector<tqr::ProbDesc> desc(nprob);
  std::vector<int64_t> tile_start(nprob + 1, 0);
  size_t total = 0;
  for (int32_t i = 0; i < nprob; ++i) {
    tqr_factors* F = nullptr;
    const int st = create(opts + i, &F, &plans[i], batch_order());
    if (st != TQR_OK) return st;
    b->F.push_back(F);
    desc[i] = tqr::ProbDesc{F->tiles, F->Tg, F->Tp, F->p, F->q, F->nb, 0};
    tile_start[i + 1] = tile_start[i] + static_cast<int64_t>(F->p) * F->q;
    total += plans[i].sub.size();
  }
  if (total >= static_cast<size_t>(INT32_MAX)) return TQR_EUNSUPPORTED;
  std::vector<std::pair<int32_t, int32_t>> order;  // (problem, local index)
  order.reserve(total);
  for (int32_t i = 0; i < nprob; ++i)
    for (int32_t r = 0; r < static_cast<int32_t>(plans[i].sub.size()); ++r) order.emplace_back(i, r);
  std::stable_sort(order.begin(), order.end(), [&](const std::pair<int32_t, int32_t>& x,
                                                   const std::pair<int32_t, int32_t>& y) {
    const double kx = plans[x.first].key[x.second], ky = plans[y.first].key[y.second];
    if (kx != ky) return kx < ky;
    if (x.first != y.first) return x.first < y.first;
    return x.second < y.second;
  });
  std::vector<std::vector<int32_t>> gpos(nprob);
  for (int32_t i = 0; i < nprob; ++i) gpos[i].resize(plans[i].sub.size());
  for (size_t g = 0; g < order.size(); ++g) gpos[order[g].first][order[g].second] = static_cast<int32_t>(g);
  ExecPlan merged;
  std::vector<int32_t> prob_of(total);
  merged.sub.resize(total);
  for (size_t g = 0; g < order.size(); ++g) {
    const int32_t i = order[g].first, r = order[g].second;
    tqr::SubTask st = plans[i].sub[r];
    st.dep_begin = static_cast<int32_t>(merged.deps.size());
    for (int32_t e = plans[i].sub[r].dep_begin; e < plans[i].sub[r].dep_end; ++e)
      merged.deps.push_back(gpos[i][tqr::dep_index(plans[i].deps[e])] | tqr::dep_bits(plans[i].deps[e]));
    st.dep_end = static_cast<int32_t>(merged.deps.size());
    merged.sub[g] = st;
    prob_of[g] = i;
  }
  int st = upload(merged, b->exec);
  if (st != TQR_OK) return st;
  b->ntiles = tile_start[nprob];
  if (!hip_ok(hipMalloc(&b->prob, nprob * sizeof(tqr::ProbDesc))) ||
      !hip_ok(hipMalloc(&b->prob_of, std::max<size_t>(1, total) * sizeof(int32_t))) ||
      !hip_ok(hipMalloc(&b->tile_start, (nprob + 1) * sizeof(int64_t))) ||
      !hip_ok(hipMalloc(&b->lda_dev, nprob * sizeof(int64_t))) ||
      !hip_ok(hipMalloc(&b->aptr_dev, nprob * sizeof(double*))) ||
      !hip_ok(hipMalloc(&b->ctl, 3 * sizeof(int32_t))) ||
      !hip_ok(hipMalloc(&b->trace_slot, sizeof(int64_t*))) ||
      !hip_ok(hipHostMalloc(&b->aptr_host, nprob * sizeof(double*))))
    return TQR_ENOMEM;
  HIP_TRY(hipMemcpy(b->prob, desc.data(), nprob * sizeof(tqr::ProbDesc), hipMemcpyHostToDevice));
  if (total) HIP_TRY(hipMemcpy(b->prob_of, prob_of.data(), total * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->tile_start, tile_start.data(), (nprob + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->lda_dev, lda, nprob * sizeof(int64_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(b->ctl, 0, 3 * sizeof(int32_t)));
  HIP_TRY(hipMemset(b->trace_slot, 0, sizeof(int64_t*)));
  HIP_TRY(hipMemset(b->aptr_dev, 0, nprob * sizeof(double*)));
  b->grid = device_cus() * tqr::batched_occupancy(b->upd);
  // The whole run (pack every problem, reset the executor, execute) as one
  // captured graph; the A pointers are read from device memory, so the same
  // graph serves every run.
  HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  tqr::BatchArgs a{};
  a.prob = b->prob;
  a.prob_of = b->prob_of;
  a.sub = b->exec.sub;
  a.deps = b->exec.deps;
  a.flags = b->exec.flags;
  a.ctl = b->ctl;
  a.nsub = b->exec.nsub;
  a.upd = b->upd;
  a.spin_ticks = 4 * wall_ticks_per_second();
  a.trace = b->trace_slot;
  HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e1 = tqr::launch_pack_batched(b->aptr_dev, b->lda_dev, b->prob, b->tile_start, nprob, b->ntiles, 64,
                                           b->cap);
  hipError_t e2 = tqr::launch_batch_reset(b->ctl, b->cap);
  hipError_t e3 = (b->exec.nsub > 0) ? tqr::launch_batched(a, b->grid, b->cap) : hipSuccess;
  hipGraph_t g = nullptr;
  hipError_t e4 = hipStreamEndCapture(b->cap, &g);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    g_last_hip = static_cast<int>((e1 != hipSuccess) ? e1 : (e2 != hipSuccess) ? e2 : (e3 != hipSuccess) ? e3 : e4);
    return TQR_EHIP;
  }
  b->graph = g;
  HIP_TRY(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
  HIP_TRY(hipEventCreate(&b->ev0));
  HIP_TRY(hipEventCreate(&b->ev1));
  *out = b.release();
  return TQR_OK;
}

int tiledqr_batch_run(tqr_batch* b, const double* const* A, void* stream) {
  if (!b || !A) return TQR_EINVAL;
  for (int32_t i = 0; i < b->nprob; ++i)
    if (!A[i]) return TQR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // The pinned staging copy is reused: wait for the previous run's copy.
  if (b->ran) HIP_TRY(hipEventSynchronize(b->ev0));
  std::memcpy(b->aptr_host, A, b->nprob * sizeof(double*));
  HIP_TRY(hipMemcpyAsync(b->aptr_dev, b->aptr_host, b->nprob * sizeof(double*), hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(b->ev0, s));
  HIP_TRY(hipGraphLaunch(b->gexec, s));
  HIP_TRY(hipEventRecord(b->ev1, s));
  for (tqr_factors* F : b->F) {
    if (!F) continue;
    F->stream = s;
    F->timed = false;
    F->rinv_ok = F->rt_ok = false;  // the factors change
  }
  b->stream = s;
  b->ran = true;
  return TQR_OK;
}

int tiledqr_batch_sync(tqr_batch* b) {
  if (!b) return TQR_EINVAL;
  HIP_TRY(hipStreamSynchronize(b->stream));
  int32_t err = 0;
  HIP_TRY(hipMemcpy(&err, b->ctl + 1, sizeof(int32_t), hipMemcpyDeviceToHost));
  return err ? TQR_EEXEC : TQR_OK;
}

int tiledqr_batch_time(tqr_batch* b, float* ms) {
  if (!b || !ms || !b->ran) return TQR_EINVAL;
  HIP_TRY(hipEventSynchronize(b->ev1));
  HIP_TRY(hipEventElapsedTime(ms, b->ev0, b->ev1));
  return TQR_OK;
}

int tiledqr_batch_set_trace(tqr_batch* b, int enable) {
  if (!b) return TQR_EINVAL;
  if (b->stream) HIP_TRY(hipStreamSynchronize(b->stream));
  if (enable && !b->trace) {
    const size_t bytes = 4 * sizeof(int64_t) * std::max<int32_t>(1, b->exec.nsub);
    if (!hip_ok(hipMalloc(&b->trace, bytes))) return TQR_ENOMEM;
    HIP_TRY(hipMemset(b->trace, 0, bytes));
    HIP_TRY(hipMemcpy(b->trace_slot, &b->trace, sizeof(int64_t*), hipMemcpyHostToDevice));
  } else if (!enable && b->trace) {
    int64_t* none = nullptr;
    HIP_TRY(hipMemcpy(b->trace_slot, &none, sizeof(int64_t*), hipMemcpyHostToDevice));
    HIP_TRY(hipFree(b->trace));
    b->trace = nullptr;
  }
  return TQR_OK;
}

int tiledqr_batch_get_trace(tqr_batch* b, int64_t* out, int64_t* n, double* ticks_per_second) {
  if (!b || !n) return TQR_EINVAL;
  *n = b->exec.nsub;
  if (ticks_per_second) *ticks_per_second = static_cast<double>(wall_ticks_per_second());
  if (!out) return TQR_OK;
  if (!b->trace) return TQR_EINVAL;
  if (b->stream) HIP_TRY(hipStreamSynchronize(b->stream));
  const int32_t ns = b->exec.nsub;
  std::vector<int64_t> t(4 * static_cast<size_t>(ns));
  std::vector<DevSub> sub(ns);
  std::vector<int32_t> prob(ns);
  HIP_TRY(hipMemcpy(t.data(), b->trace, t.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(sub.data(), b->exec.sub, sub.size() * sizeof(DevSub), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(prob.data(), b->prob_of, prob.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int32_t s = 0; s < ns; ++s) {
    int64_t* o = out + 11 * static_cast<int64_t>(s);
    o[0] = sub[s].kind;
    o[1] = sub[s].i;
    o[2] = sub[s].piv;
    o[3] = sub[s].k;
    o[4] = sub[s].j;
    o[5] = sub[s].slab;
    o[6] = t[4 * s];
    o[7] = t[4 * s + 1];
    o[8] = t[4 * s + 2];
    o[9] = t[4 * s + 3];
    o[10] = prob[s];
  }
  return TQR_OK;
}

int tiledqr_batch_get(tqr_batch* b, int32_t i, tqr_factors** F) {
  if (!b || !F || i < 0 || i >= b->nprob || !b->F[i]) return TQR_EINVAL;
  *F = b->F[i];
  return TQR_OK;
}

int tiledqr_batch_destroy(tqr_batch* b) {
  if (!b) return TQR_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  delete b;
  return TQR_OK;
}

int tiledqr_factor_batched(int32_t nprob, const tqr_opts* opts, const double* const* A, const int64_t* lda,
                           tqr_factors** F, void* stream) {
  if (nprob < 0 || (nprob > 0 && (!opts || !A || !lda || !F))) return TQR_EINVAL;
  if (nprob == 0) return TQR_OK;
  for (int32_t i = 0; i < nprob; ++i)
    if (!A[i]) return TQR_EINVAL;
  tqr_batch* b = nullptr;
  int st = tiledqr_batch_create(nprob, opts, lda, &b);
  if (st != TQR_OK) {
    tiledqr_batch_destroy(b);
    return st;
  }
  st = tiledqr_batch_run(b, A, stream);
  if (st == TQR_OK) st = tiledqr_batch_sync(b);
  if (st == TQR_OK) {
    // Hand the problems' handles to the caller.
    for (int32_t i = 0; i < nprob; ++i) {
      F[i] = b->F[i];
      b->F[i] = nullptr;
    }
  }
  tiledqr_batch_destroy(b);
  return st;
}

}  // extern "C"
