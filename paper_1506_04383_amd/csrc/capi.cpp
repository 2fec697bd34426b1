// C-ABI of libmulment and the multilevel driver (Section 3 of the paper):
// coarsening loop with the size bound U = max(max c, min(b^h, |V|/f)) and the
// f := 0.7 f rule, initial layout, prolongation, and on every level the
// alpha schedule of the local improvement (at most `a` Jacobi iterations per
// alpha, early drop below eps_round, iteration at alpha_min until the
// relative change is below eps_final).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>
#include <string>
#include <vector>

#include "mulment.h"
#include "kernels.hpp"
#include "validate.hpp"

// Iterations of a batch level captured into one HIP graph and replayed
// between two host checks of the running-graph count (even: a replay keeps
// the parity of the coordinate buffers).
constexpr int32_t kBatchReplay = 4;
// iterations a single layout enqueues between two reads of its device-side
// schedule state
constexpr int32_t kIterChunk = 8;
// Barnes-Hut levels below this many vertices run the tiled stress sums as
// kCapPerCU persistent work-groups per compute unit (two below 2^16
// vertices, where the far field's share is larger; see mm_layout)
constexpr int32_t kCapMaxN = 1 << 17;
constexpr int32_t kCapPerCU = 3;
// Single-graph levels replay far field and sweep from two graphs above this
// many vertices, from one graph at or below it.
constexpr int32_t kSplitMinN = 1 << 16;

struct mm_context {
  int device = 0;
  hipStream_t stream = nullptr;  // the caller's stream
  hipStream_t work = nullptr;    // the layout drivers' own stream (capturable)
  mm::BHWork* bh = nullptr;
  double* pinned = nullptr;      // 16 doubles for small read-backs
  float* alpha_dev = nullptr;
  hipStream_t far = nullptr;     // far field of mm_layout, beside the sweep on `work`
  int32_t cus = 0;               // compute units of the device
  hipEvent_t ev[8] = {};
  // this device's copy of the fixed scratch of mm_sweep_noalloc (null if its
  // lookup failed; scratch_err then holds the HIP error)
  void* scratch = nullptr;
  hipError_t scratch_err = hipSuccess;
  // autotuner: sweep configuration per level shape (coarse?, n, sum |S|, k)
  struct TuneChoice { int32_t tbits, group, nb; };  // tbits 0: row kernel (nb 0)
  std::map<std::tuple<int, int32_t, int64_t, int32_t>, TuneChoice> tune;
};
struct mm_khop {
  mm::KhopDev kh;
  mm::TiledSet ts;     // tile-major copy, built on first tiled sweep
  bool ts_tried = false;
};
struct mm_coarse {
  mm::GraphDev g;
};

namespace {

thread_local std::string g_err;

mm_status fail(mm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}
mm_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? MM_ENOMEM : MM_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}
#define HIPCHK(expr)                                        \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return hip_fail(_e, #expr);       \
  } while (0)
#define STCHK(expr)                                         \
  do {                                                      \
    mm_status _s = (expr);                                  \
    if (_s != MM_OK) return _s;                             \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Host-side structural validation (undirected simple graph, weights >= 1).
mm_status validate_graph(int32_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                         const int32_t* c, const int32_t* w) {
  char msg[256];
  if (!mm::check_graph(n, nnz, rp, col, c, w, msg, sizeof(msg))) return fail(MM_EINVAL, "%s", msg);
  return MM_OK;
}

mm_status validate_params(const mm_params* p) {
  if (!p) return fail(MM_EINVAL, "params is NULL");
  if (p->k < 1 || p->k > 8) return fail(MM_EINVAL, "k must be in [1, 8]");
  if (std::isnan(p->theta) || std::isnan(p->q)) return fail(MM_EINVAL, "theta/q NaN");
  if (!(p->alpha0 > 0) || !(p->alpha_min > 0)) return fail(MM_EINVAL, "alpha0, alpha_min must be > 0");
  if (p->alpha0 < p->alpha_min) return fail(MM_EINVAL, "alpha schedule inverted (alpha0 < alpha_min)");
  if (!(p->alpha_decay > 0 && p->alpha_decay < 1)) return fail(MM_EINVAL, "alpha_decay must be in (0,1)");
  if (p->iters_per_round < 1 || p->max_final_iters < 0) return fail(MM_EINVAL, "iteration counts");
  if (!(p->eps_round >= 0) || !(p->eps_final >= 0)) return fail(MM_EINVAL, "eps must be >= 0");
  if (p->max_levels < 0 || p->max_levels >= MM_MAX_LEVELS) return fail(MM_EINVAL, "max_levels in [0, 63]");
  if (!(p->b > 1) || !(p->f > 0)) return fail(MM_EINVAL, "b > 1 and f > 0 required");
  if (p->lp_rounds < 0) return fail(MM_EINVAL, "lp_rounds < 0");
  if (!(p->coarse_dist_scale > 0)) return fail(MM_EINVAL, "coarse_dist_scale must be > 0");
  if (p->exact_below < 0) return fail(MM_EINVAL, "exact_below must be >= 0");
  if (p->approx_h < 0) return fail(MM_EINVAL, "approx_h must be >= 0");
  if (p->mlp_weights && (p->theta < 0 || p->q != 0.0))
    return fail(MM_EUNSUPPORTED, "the learned far field needs theta >= 0 and q == 0");
  return MM_OK;
}

struct Timer {
  hipEvent_t a, b;
  hipStream_t s;
  Timer(hipEvent_t a_, hipEvent_t b_, hipStream_t s_) : a(a_), b(b_), s(s_) {}
};

struct LevelGraph {
  mm::GraphDev g;      // owned arrays for coarse levels
  std::vector<int32_t> c_host;
};

// sqrt of node weights (ones when c is NULL)
hipError_t make_sqrtc(int32_t n, const int32_t* c, mm::DevBuf& buf, hipStream_t s) {
  MM_TRY(buf.alloc(sizeof(float) * (size_t)n, s));
  return mm::sqrt_weights(n, c, buf.as<float>(), s);
}

// Times `reps` launches of a sweep variant after one untimed launch; returns ms per launch.
template <typename F>
hipError_t time_variant(mm_context* ctx, hipStream_t s, int reps, F&& launch, float* ms) {
  MM_TRY(launch());
  MM_TRY(hipEventRecord(ctx->ev[0], s));
  for (int r = 0; r < reps; ++r) MM_TRY(launch());
  MM_TRY(hipEventRecord(ctx->ev[1], s));
  MM_TRY(hipEventSynchronize(ctx->ev[1]));
  float t = 0;
  MM_TRY(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]));
  *ms = t / reps;
  return hipSuccess;
}

// Autotuner of one level's sweep: every eligible configuration -- the row
// kernel with 8/16/32/64 lanes per row, the tiled kernel with tiles of 2^11,
// 2^12, 2^13 vertices, 1/2/4/8/16 lanes per chunk and 2/4 blocks per lane and
// step -- is run on the level's own
// sets and coordinates (far field zero, alpha 1, output to scratch) and the
// fastest is kept.  Row-kernel candidates are skipped on levels whose sets are
// too large for that kernel to win (over 2^30 entries).
mm_status tune_level(mm_context* ctx, mm::KhopDev& kh, int32_t lvl, const float* sqrtc,
                     const mm_params* p, const float* xa, float* F, float* xb, double* d2,
                     hipStream_t s, mm_context::TuneChoice* out) {
  const int32_t nl = kh.n;
  HIPCHK(hipMemsetAsync(F, 0, sizeof(float) * 2 * (size_t)nl, s));
  float best = INFINITY;
  mm_context::TuneChoice bc{0, mm::row_group(kh), 0};
  const int reps = kh.total > (1ll << 28) ? 1 : 3;
  // MM_TUNE_VERBOSE=1 prints every candidate's time to stderr
  const char* ev = std::getenv("MM_TUNE_VERBOSE");
  const bool verbose = ev && ev[0] == '1';
  if (kh.total <= (1ll << 30)) {
    mm::DevBuf part;
    for (int32_t G : {8, 16, 32, 64}) {
      float ms = 0;
      HIPCHK(time_variant(ctx, s, reps, [&]() {
        return mm::sweep(kh, lvl, sqrtc, p->coarse_dist_scale, xa, F, 1.0, p->q, xb, d2, s, nullptr,
                         nullptr, nullptr, &part, G);
      }, &ms));
      if (verbose)
        std::fprintf(stderr, "[tune] level %d n %d sets %lld rows lanes %d: %.4f ms\n", lvl, nl,
                     (long long)kh.total, G, ms);
      if (ms < best) { best = ms; bc = {0, G, 0}; }
    }
  }
  mm::DevBuf rho;
  bool have_rho = false;
  for (int32_t tb : {11, 12, 13}) {
    if (!mm::tiled_eligible(kh, tb)) continue;
    if (!have_rho) {
      HIPCHK(rho.alloc(sizeof(float) * (size_t)nl, s));
      HIPCHK(mm::compute_rho(kh, sqrtc, p->coarse_dist_scale, rho.as<float>(), s));
      have_rho = true;
    }
    mm::TiledSet ts;
    HIPCHK(mm::tiled_build(kh, tb, 0.0, &ts, s));
    if (!ts.built) continue;
    for (int32_t G : {1, 2, 4, 8, 16}) {
      for (int32_t NB : {2, 4}) {
        float ms = 0;
        HIPCHK(time_variant(ctx, s, reps, [&]() {
          return mm::sweep_tiled(ts, lvl, sqrtc, p->coarse_dist_scale, rho.as<float>(), xa, F,
                                 1.0, p->q, xb, d2, s, nullptr, G, NB);
        }, &ms));
        if (verbose)
          std::fprintf(stderr, "[tune] level %d n %d sets %lld tiled tbits %d lanes %d blocks %d: %.4f ms\n",
                       lvl, nl, (long long)kh.total, tb, G, NB, ms);
        if (ms < best) { best = ms; bc = {tb, G, NB}; }
      }
    }
    HIPCHK(hipStreamSynchronize(s));
    // the sliced layout of the same tiles
    mm::TiledSet tsl;
    HIPCHK(mm::tiled_build(kh, tb, 0.0, &tsl, s, nullptr, 1.0, nullptr, true));
    if (!tsl.built) continue;
    for (int32_t NB : {2, 4}) {
      float ms = 0;
      HIPCHK(time_variant(ctx, s, reps, [&]() {
        return mm::sweep_tiled(tsl, lvl, sqrtc, p->coarse_dist_scale, rho.as<float>(), xa, F,
                               1.0, p->q, xb, d2, s, nullptr, mm::kSlicedGroup, NB);
      }, &ms));
      if (verbose)
        std::fprintf(stderr, "[tune] level %d n %d sets %lld sliced tbits %d blocks %d: %.4f ms\n",
                     lvl, nl, (long long)kh.total, tb, NB, ms);
      if (ms < best) { best = ms; bc = {tb, mm::kSlicedGroup, NB}; }
    }
    HIPCHK(hipStreamSynchronize(s));
  }
  *out = bc;
  return MM_OK;
}

// One sweep through the C-ABI: mode as mm_sweep_ex; tbits/group/nb > 0 force
// the tile size, lanes and blocks per step (a tile-major copy of another tile
// size is built for the call and dropped).
mm_status sweep_common(mm_context* ctx, mm_khop* kh, int32_t level, const int32_t* node_w,
                       double scale, const float* xy_in, const float* F, double alpha, double q,
                       float* xy_out, double* delta, int32_t mode, int32_t tbits, int32_t group,
                       int32_t nb) {
  try {
    if (!ctx || !kh || !xy_in || !F || !xy_out) return fail(MM_EINVAL, "NULL argument");
    if (xy_in == xy_out) return fail(MM_EINVAL, "Jacobi update needs separate in/out buffers");
    if (level < 0 || !(scale > 0) || std::isnan(alpha) || std::isnan(q)) return fail(MM_EINVAL, "bad level/scale/alpha/q");
    DeviceGuard dg(ctx->device);
    hipStream_t s = ctx->stream;
    mm::DevBuf sq, d2;
    const float* sqrtc = nullptr;
    if (level > 0) {
      HIPCHK(make_sqrtc(kh->kh.n, node_w, sq, s));
      sqrtc = sq.as<float>();
    }
    HIPCHK(d2.alloc(2 * sizeof(double), s));
    const int32_t tb = tbits > 0 ? tbits : mm::kTileBits;
    mm::TiledSet own;
    const mm::TiledSet* ts = nullptr;
    if (mode != MM_SWEEP_ROWS) {
      const bool ok = mm::tiled_eligible(kh->kh, tb);
      if (mode == MM_SWEEP_TILED && !ok) return fail(MM_EUNSUPPORTED, "tiled sweep needs k <= 7 and n <= 2^25");
      if (ok && group == mm::kSlicedGroup) {
        HIPCHK(mm::tiled_build(kh->kh, tb, 0.0, &own, s, nullptr, 1.0, nullptr, true));
        if (own.built) ts = &own;
      } else if (ok && tb != mm::kTileBits) {
        HIPCHK(mm::tiled_build(kh->kh, tb, 0.0, &own, s));
        if (own.built) ts = &own;
      } else if (ok) {
        if (!kh->ts_tried) {
          HIPCHK(mm::tiled_build(kh->kh, tb, mode == MM_SWEEP_TILED ? 0.0 : 8.0, &kh->ts, s));
          kh->ts_tried = true;
        }
        if (!kh->ts.built && mode == MM_SWEEP_TILED) HIPCHK(mm::tiled_build(kh->kh, tb, 0.0, &kh->ts, s));
        if (kh->ts.built) ts = &kh->ts;
      }
      if (!ts && mode == MM_SWEEP_TILED) return fail(MM_EUNSUPPORTED, "tile-major sets not built");
    }
    if (ts) {
      mm::DevBuf rho;
      HIPCHK(rho.alloc(sizeof(float) * (size_t)kh->kh.n, s));
      HIPCHK(mm::compute_rho(kh->kh, sqrtc, scale, rho.as<float>(), s));
      HIPCHK(mm::sweep_tiled(*ts, level, sqrtc, scale, rho.as<float>(), xy_in, F, alpha, q,
                             xy_out, d2.as<double>(), s, nullptr, group, nb));
    } else {
      mm::DevBuf part;
      HIPCHK(mm::sweep(kh->kh, level, sqrtc, scale, xy_in, F, alpha, q, xy_out, d2.as<double>(), s,
                       nullptr, nullptr, nullptr, &part, group));
    }
    HIPCHK(hipMemcpyAsync(ctx->pinned, d2.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (delta) { delta[0] = ctx->pinned[0]; delta[1] = ctx->pinned[1]; }
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in the sweep");
  }
}

}  // namespace

extern "C" {

const char* mm_last_error(void) { return g_err.c_str(); }

mm_status mm_tune_clear(mm_context* ctx) {
  if (!ctx) return fail(MM_EINVAL, "NULL context");
  ctx->tune.clear();
  return MM_OK;
}

mm_status mm_tune_export(mm_context* ctx, int64_t* recs, int32_t cap, int32_t* count) {
  if (!ctx || !count) return fail(MM_EINVAL, "NULL context or count");
  if (cap > 0 && !recs) return fail(MM_EINVAL, "NULL records with cap %d", cap);
  int32_t i = 0;
  for (const auto& [key, c] : ctx->tune) {
    if (i < cap) {
      int64_t* r = recs + (size_t)i * MM_TUNE_FIELDS;
      r[0] = std::get<0>(key);
      r[1] = std::get<1>(key);
      r[2] = std::get<2>(key);
      r[3] = std::get<3>(key);
      r[4] = c.tbits;
      r[5] = c.group;
      r[6] = c.nb;
    }
    ++i;
  }
  *count = i;
  return MM_OK;
}

mm_status mm_tune_import(mm_context* ctx, const int64_t* recs, int32_t count) {
  if (!ctx) return fail(MM_EINVAL, "NULL context");
  if (count < 0 || (count > 0 && !recs)) return fail(MM_EINVAL, "bad record list (%d)", count);
  for (int32_t i = 0; i < count; ++i) {
    if (!mm::check_tune_record(recs + (size_t)i * MM_TUNE_FIELDS, mm::kSlicedGroup))
      return fail(MM_EINVAL, "tune record %d is invalid", i);
  }
  for (int32_t i = 0; i < count; ++i) {
    const int64_t* r = recs + (size_t)i * MM_TUNE_FIELDS;
    ctx->tune[std::make_tuple((int)r[0], (int32_t)r[1], r[2], (int32_t)r[3])] =
        mm_context::TuneChoice{(int32_t)r[4], (int32_t)r[5], (int32_t)r[6]};
  }
  return MM_OK;
}

mm_status mm_params_default(mm_params* p) {
  if (!p) return fail(MM_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->k = 1;
  p->q = 0.0;
  p->theta = 0.5;
  p->alpha0 = 1.0;
  p->alpha_decay = 0.3;
  p->alpha_min = 0.008;
  p->iters_per_round = 2;
  p->eps_round = 1e-4;
  p->eps_final = 1e-4;
  p->max_final_iters = 200;
  p->max_levels = 62;
  p->coarsest_n = 2;
  p->b = 2.0;
  p->f = 20.0;
  p->lp_rounds = 10;
  p->coarse_dist_scale = 1.0;
  p->seed = 1;
  p->validate = 1;
  p->mlp_weights = nullptr;
  p->use_graphs = 1;
  p->autotune = 0;
  p->exact_below = 0;
  p->approx_h = 0;
  p->khop_direct = 1;
  return MM_OK;
}

mm_status mm_context_create(mm_context** out, int32_t device, void* stream) {
  try {
    if (!out) return fail(MM_EINVAL, "out is NULL");
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(MM_EINVAL, "device %d out of range (%d)", device, count);
    DeviceGuard dg(device);
    std::unique_ptr<mm_context> c(new mm_context());
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->bh = mm::bh_work_create();
    HIPCHK(hipHostMalloc((void**)&c->pinned, 16 * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipMalloc((void**)&c->alpha_dev, sizeof(float)));
    HIPCHK(hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device));
    HIPCHK(hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&c->far, hipStreamNonBlocking));
    for (auto& e : c->ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDefault));
    // device address of the no-allocation sweep's scratch (looked up once per
    // device, with the device current); a failure is reported by that call
    c->scratch_err = mm::noalloc_scratch_setup(device, &c->scratch);
    mm::big_register(c->stream);
    mm::big_register(c->work);
    mm::big_register(c->far);
    // the library's buffers come from the device's default pool
    // (stream-ordered); keep freed memory in the pool instead of returning it
    // at every synchronisation, since each level frees and re-allocates sets
    // of tens of GB (mm_context_destroy trims the pool)
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    *out = c.release();
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_context_create");
  }
}

void mm_context_destroy(mm_context* ctx) {
  if (!ctx) return;
  DeviceGuard dg(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  mm::bh_work_destroy(ctx->bh);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->work) (void)hipStreamSynchronize(ctx->work);
  if (ctx->far) (void)hipStreamSynchronize(ctx->far);
  mm::big_unregister(ctx->stream);
  if (ctx->work) mm::big_unregister(ctx->work);
  if (ctx->far) mm::big_unregister(ctx->far);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->alpha_dev) (void)hipFree(ctx->alpha_dev);
  if (ctx->work) (void)hipStreamDestroy(ctx->work);
  if (ctx->far) (void)hipStreamDestroy(ctx->far);
  for (auto& e : ctx->ev) if (e) (void)hipEventDestroy(e);
  (void)hipDeviceSynchronize();
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, ctx->device) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
  delete ctx;
}

mm_status mm_sync(mm_context* ctx) {
  if (!ctx) return fail(MM_EINVAL, "ctx is NULL");
  DeviceGuard dg(ctx->device);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipGetLastError());
  return MM_OK;
}

// ------------------------------------------------------------------ k-hop

mm_status mm_khop_build(mm_context* ctx, const mm_graph* g, int32_t k, mm_khop** out) {
  try {
    if (!ctx || !g || !out) return fail(MM_EINVAL, "NULL argument");
    if (g->mem != MM_DEVICE) return fail(MM_EINVAL, "mm_khop_build needs a device graph");
    if (k < 1 || k > 8) return fail(MM_EINVAL, "k must be in [1, 8]");
    if (g->n < 2) return fail(MM_EINVAL, "n < 2");
    DeviceGuard dg(ctx->device);
    std::unique_ptr<mm_khop> kh(new mm_khop());
    HIPCHK(mm::khop_build(g->n, g->row_ptr, g->col, k, &kh->kh, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *out = kh.release();
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_khop_build");
  }
}

void mm_khop_free(mm_khop* kh) { delete kh; }

mm_status mm_khop_info(const mm_khop* kh, int32_t* n, int32_t* k, int64_t* total) {
  if (!kh) return fail(MM_EINVAL, "kh is NULL");
  if (n) *n = kh->kh.n;
  if (k) *k = kh->kh.k;
  if (total) *total = kh->kh.total;
  return MM_OK;
}

mm_status mm_khop_arrays(const mm_khop* kh, const int64_t** off, const int32_t** hend,
                         const int32_t** nbr) {
  if (!kh) return fail(MM_EINVAL, "kh is NULL");
  if (off) *off = kh->kh.off;
  if (hend) *hend = kh->kh.hend;
  if (nbr) *nbr = kh->kh.nbr;
  return MM_OK;
}

mm_status mm_khop_export(mm_context* ctx, const mm_khop* kh, int64_t* off, int32_t* hend,
                         int32_t* nbr, int32_t mem) {
  if (!ctx || !kh) return fail(MM_EINVAL, "NULL argument");
  if (mem != MM_HOST && mem != MM_DEVICE) return fail(MM_EINVAL, "bad mem kind");
  DeviceGuard dg(ctx->device);
  const hipMemcpyKind kd = mem == MM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const mm::KhopDev& K = kh->kh;
  if (off) HIPCHK(hipMemcpyAsync(off, K.off, sizeof(int64_t) * (size_t)(K.n + 1), kd, ctx->stream));
  if (hend) HIPCHK(hipMemcpyAsync(hend, K.hend, sizeof(int32_t) * (size_t)K.n * K.k, kd, ctx->stream));
  if (nbr && K.total > 0) HIPCHK(hipMemcpyAsync(nbr, K.nbr, sizeof(int32_t) * (size_t)K.total, kd, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return MM_OK;
}

// A general stress set S ⊇ E (footnote to Eq. 1) handed in by the caller, in
// the layout of the k-hop sets: per row the entries are grouped by their
// target distance d_uv = h in 1..k (hend cumulative), ids strictly increasing
// inside a group.  S is a set of unordered pairs: (u, v, h) in row u needs
// (v, u, h) in row v.
mm_status mm_khop_validate(int32_t n, int32_t k, const int64_t* off, const int32_t* hend,
                           const int32_t* nbr) {
  char msg[256];
  if (!mm::check_stress_set(n, k, off, hend, nbr, msg, sizeof(msg))) return fail(MM_EINVAL, "%s", msg);
  return MM_OK;
}

mm_status mm_khop_import(mm_context* ctx, int32_t n, int32_t k, const int64_t* off,
                         const int32_t* hend, const int32_t* nbr, int32_t mem, mm_khop** out) {
  try {
    if (!ctx || !off || !hend || !out) return fail(MM_EINVAL, "NULL argument");
    if (mem != MM_HOST && mem != MM_DEVICE) return fail(MM_EINVAL, "bad mem kind");
    if (n < 2) return fail(MM_EINVAL, "n < 2");
    if (k < 1 || k > 8) return fail(MM_EINVAL, "k must be in [1, 8]");
    DeviceGuard dg(ctx->device);
    hipStream_t s = ctx->stream;
    // host copies for the checks when the caller's arrays live on the device
    std::vector<int64_t> h_off;
    std::vector<int32_t> h_hend, h_nbr;
    const int64_t* ho = off;
    const int32_t* hh = hend;
    const int32_t* hn = nbr;
    if (mem == MM_DEVICE) {
      h_off.resize((size_t)n + 1);
      h_hend.resize((size_t)n * k);
      HIPCHK(hipMemcpyAsync(h_off.data(), off, sizeof(int64_t) * h_off.size(), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(h_hend.data(), hend, sizeof(int32_t) * h_hend.size(), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      const int64_t tot = h_off[(size_t)n];
      if (tot < 0 || h_off[0] != 0) return fail(MM_EINVAL, "off[0] must be 0 and off[n] >= 0");
      if (tot > 0) {
        if (!nbr) return fail(MM_EINVAL, "nbr is NULL");
        h_nbr.resize((size_t)tot);
        HIPCHK(hipMemcpyAsync(h_nbr.data(), nbr, sizeof(int32_t) * h_nbr.size(), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
      }
      ho = h_off.data();
      hh = h_hend.data();
      hn = h_nbr.data();
    }
    STCHK(mm_khop_validate(n, k, ho, hh, hn));
    const int64_t total = ho[n];
    std::unique_ptr<mm_khop> kh(new mm_khop());
    mm::KhopDev& K = kh->kh;
    K.n = n;
    K.k = k;
    K.total = total;
    HIPCHK(K.b_off.alloc(sizeof(int64_t) * (size_t)(n + 1), s));
    HIPCHK(K.b_hend.alloc(sizeof(int32_t) * (size_t)n * k, s));
    HIPCHK(K.b_nbr.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1), s));
    K.off = K.b_off.as<int64_t>();
    K.hend = K.b_hend.as<int32_t>();
    K.nbr = K.b_nbr.as<int32_t>();
    const hipMemcpyKind kd = mem == MM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(hipMemcpyAsync(K.off, off, sizeof(int64_t) * (size_t)(n + 1), kd, s));
    HIPCHK(hipMemcpyAsync(K.hend, hend, sizeof(int32_t) * (size_t)n * k, kd, s));
    if (total > 0) HIPCHK(hipMemcpyAsync(K.nbr, nbr, sizeof(int32_t) * (size_t)total, kd, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = kh.release();
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_khop_import");
  }
}

// ------------------------------------------------------------- far field

mm_status mm_repulsion(mm_context* ctx, int32_t n, const float* xy, double q, double theta,
                       float* F, uint64_t* codes, int32_t* order, int64_t* nodes,
                       int64_t* counters) {
  try {
    if (!ctx || !xy || !F) return fail(MM_EINVAL, "NULL argument");
    if (n < 1) return fail(MM_EINVAL, "n < 1");
    if (std::isnan(theta) || std::isnan(q)) return fail(MM_EINVAL, "theta/q NaN");
    DeviceGuard dg(ctx->device);
    if (theta < 0) {
      HIPCHK(mm::farfield_exact(ctx->bh, n, xy, q, F, ctx->stream));
      if (counters) { counters[0] = 0; counters[1] = (int64_t)n * (n - 1); counters[2] = 0; counters[3] = 0; }
    } else {
      mm::FarStats st{};
      int64_t nn = 0;
      HIPCHK(mm::farfield_bh(ctx->bh, n, xy, q, theta, F, codes, order, nodes, &nn,
                             counters ? 1 : 0, &st, ctx->stream));
      if (counters) { counters[0] = st.accepted; counters[1] = st.leaf_pairs; counters[2] = 0; counters[3] = nn; }
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_repulsion");
  }
}

mm_status mm_repulsion_cluster(mm_context* ctx, int32_t n, const float* xy, const int32_t* node_w,
                               const int32_t* cluster1, int32_t n1, const int32_t* cluster_h,
                               int32_t nh, double q, float* F) {
  try {
    if (!ctx || !xy || !F || !cluster1 || !cluster_h) return fail(MM_EINVAL, "NULL argument");
    if (n < 1 || n1 < 1 || nh < 1) return fail(MM_EINVAL, "n, n1 and nh must be >= 1");
    if (std::isnan(q)) return fail(MM_EINVAL, "q NaN");
    DeviceGuard dg(ctx->device);
    hipStream_t s = ctx->stream;
    bool ok = false;
    HIPCHK(mm::cluster_far_check(n, cluster1, n1, cluster_h, nh, &ok, s));
    if (!ok) return fail(MM_EINVAL, "cluster id out of range");
    mm::ClusterFar cf;
    HIPCHK(mm::cluster_far_setup(n, cluster1, n1, cluster_h, nh, &cf, s));
    HIPCHK(mm::cluster_far(cf, xy, node_w, q, F, s));
    HIPCHK(hipStreamSynchronize(s));
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_repulsion_cluster");
  }
}

// ------------------------------------------------------ learned far field

mm_status mm_repulsion_learned(mm_context* ctx, int32_t n, const float* xy, double theta,
                               const float* weights, float* F) {
  try {
    if (!ctx || !xy || !F || !weights) return fail(MM_EINVAL, "NULL argument");
    if (n < 1) return fail(MM_EINVAL, "n < 1");
    if (!(theta >= 0)) return fail(MM_EINVAL, "theta must be >= 0");
    DeviceGuard dg(ctx->device);
    HIPCHK(mm::farfield_learned(ctx->bh, n, xy, theta, weights, F, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_repulsion_learned");
  }
}

mm_status mm_far_samples(mm_context* ctx, int32_t n, const float* xy, double theta, int64_t cap,
                         int32_t* u_out, int32_t* node_out, float* feat, float* target,
                         float* coef, int64_t* count) {
  try {
    if (!ctx || !xy || !count) return fail(MM_EINVAL, "NULL argument");
    if (n < 1) return fail(MM_EINVAL, "n < 1");
    if (!(theta >= 0)) return fail(MM_EINVAL, "theta must be >= 0");
    if (cap < 0) return fail(MM_EINVAL, "cap < 0");
    if (cap > 0 && (!u_out || !node_out || !feat || !target || !coef))
      return fail(MM_EINVAL, "NULL output with cap > 0");
    DeviceGuard dg(ctx->device);
    int64_t total = 0;
    HIPCHK(mm::far_samples(ctx->bh, n, xy, theta, cap, u_out, node_out, feat, target, coef, &total,
                           ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *count = total;
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_far_samples");
  }
}

mm_status mm_mlp_init(mm_context* ctx, uint64_t seed, double out_scale, float* weights) {
  try {
    if (!ctx || !weights) return fail(MM_EINVAL, "NULL argument");
    if (!(out_scale >= 0) || !std::isfinite(out_scale)) return fail(MM_EINVAL, "out_scale must be finite and >= 0");
    DeviceGuard dg(ctx->device);
    HIPCHK(mm::mlp_init(seed, out_scale, weights, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_mlp_init");
  }
}

mm_status mm_mlp_forward(mm_context* ctx, int64_t count, const float* feat, const float* weights,
                         float* out) {
  try {
    if (!ctx || (count > 0 && (!feat || !weights || !out))) return fail(MM_EINVAL, "NULL argument");
    if (count < 0) return fail(MM_EINVAL, "count < 0");
    DeviceGuard dg(ctx->device);
    HIPCHK(mm::mlp_forward(count, feat, weights, out, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_mlp_forward");
  }
}

mm_status mm_mlp_grad(mm_context* ctx, int64_t count, const float* feat, const float* target,
                      const float* weights, float* grad, float* loss) {
  try {
    if (!ctx || !feat || !target || !weights || !grad || !loss) return fail(MM_EINVAL, "NULL argument");
    if (count < 1) return fail(MM_EINVAL, "count < 1");
    DeviceGuard dg(ctx->device);
    HIPCHK(mm::mlp_grad(count, feat, target, weights, grad, loss, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_mlp_grad");
  }
}

mm_status mm_mlp_train(mm_context* ctx, int64_t count, const float* feat, const float* target,
                       float* weights, float* adam, int32_t steps, int32_t batch, double lr,
                       uint64_t seed, int32_t step0, float* losses) {
  try {
    if (!ctx || !feat || !target || !weights || !adam) return fail(MM_EINVAL, "NULL argument");
    if (count < 1 || steps < 0 || batch < 1 || step0 < 0) return fail(MM_EINVAL, "sizes");
    if (!(lr > 0)) return fail(MM_EINVAL, "lr must be > 0");
    DeviceGuard dg(ctx->device);
    HIPCHK(mm::mlp_train(count, feat, target, weights, adam, steps, batch, lr, seed, step0, losses,
                         ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_mlp_train");
  }
}

// ------------------------------------------------------------------ sweep

mm_status mm_sweep_ex(mm_context* ctx, mm_khop* kh, int32_t level, const int32_t* node_w,
                      double scale, const float* xy_in, const float* F, double alpha, double q,
                      float* xy_out, double* delta, int32_t mode) {
  if (mode < MM_SWEEP_AUTO || mode > MM_SWEEP_TILED) return fail(MM_EINVAL, "bad sweep mode");
  return sweep_common(ctx, kh, level, node_w, scale, xy_in, F, alpha, q, xy_out, delta, mode, 0, 0,
                      0);
}

mm_status mm_sweep_cfg(mm_context* ctx, mm_khop* kh, int32_t level, const int32_t* node_w,
                       double scale, const float* xy_in, const float* F, double alpha, double q,
                       float* xy_out, double* delta, int32_t tile_bits, int32_t group,
                       int32_t blocks) {
  const bool rows_ok = tile_bits == 0 && blocks == 0 &&
                       (group == 8 || group == 16 || group == 32 || group == 64);
  const bool tiled_ok = tile_bits >= 11 && tile_bits <= 13 &&
                        (group == 1 || group == 2 || group == 4 || group == 8 || group == 16 ||
                         group == mm::kSlicedGroup) &&
                        (blocks == 0 || blocks == 2 || blocks == 4);
  if (!rows_ok && !tiled_ok)
    return fail(MM_EINVAL, "bad sweep configuration (%d, %d, %d)", tile_bits, group, blocks);
  return sweep_common(ctx, kh, level, node_w, scale, xy_in, F, alpha, q, xy_out, delta,
                      tile_bits ? MM_SWEEP_TILED : MM_SWEEP_ROWS, tile_bits, group, blocks);
}

mm_status mm_sweep(mm_context* ctx, const mm_khop* kh, int32_t level, const int32_t* node_w,
                   double scale, const float* xy_in, const float* F, double alpha, double q,
                   float* xy_out, double* delta) {
  return mm_sweep_ex(ctx, const_cast<mm_khop*>(kh), level, node_w, scale, xy_in, F, alpha, q,
                     xy_out, delta, MM_SWEEP_ROWS);
}

static_assert(MM_SWEEP_NOALLOC_MAX_N == mm::kNoallocMaxN, "scratch limit");

mm_status mm_sweep_noalloc(mm_context* ctx, const mm_khop* kh, int32_t level,
                           const int32_t* node_w, double scale, const float* xy_in,
                           const float* F, double alpha, double q, float* xy_out, double* delta) {
  try {
    if (!ctx || !kh || !xy_in || !F || !xy_out) return fail(MM_EINVAL, "NULL argument");
    if (xy_in == xy_out) return fail(MM_EINVAL, "Jacobi update needs separate in/out buffers");
    if (level < 0 || !(scale > 0) || std::isnan(alpha) || std::isnan(q)) return fail(MM_EINVAL, "bad level/scale/alpha/q");
    const mm::KhopDev& K = kh->kh;
    if (K.n > MM_SWEEP_NOALLOC_MAX_N)
      return fail(MM_EINVAL, "mm_sweep_noalloc: %d vertices exceed its scratch limit of %d", K.n,
                  MM_SWEEP_NOALLOC_MAX_N);
    if (K.k > 8) return fail(MM_EINVAL, "k must be <= 8");
    if (K.n > 0 && !K.nbr && K.total > 0) return fail(MM_EINVAL, "the sets hold no ids");
    if (!ctx->scratch)
      return fail(MM_EDEVICE, "scratch of device %d unavailable: %s", ctx->device,
                  hipGetErrorString(ctx->scratch_err));
    DeviceGuard dg(ctx->device);
    hipStream_t s = ctx->stream;
    unsigned char* base = static_cast<unsigned char*>(ctx->scratch);
    double* d2 = reinterpret_cast<double*>(base);
    double2* part = reinterpret_cast<double2*>(base + mm::kNoallocPartOff);
    float* sqrtc = nullptr;
    if (level > 0) {
      sqrtc = reinterpret_cast<float*>(base + mm::kNoallocSqrtcOff);
      HIPCHK(mm::sqrt_weights(K.n, node_w, sqrtc, s));
    }
    HIPCHK(mm::sweep_into(K, level, sqrtc, scale, xy_in, F, alpha, q, xy_out, d2, part,
                          mm::kNoallocPartBytes, s));
    HIPCHK(hipMemcpyAsync(ctx->pinned, d2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (delta) { delta[0] = ctx->pinned[0]; delta[1] = ctx->pinned[1]; }
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_sweep_noalloc");
  }
}

// ------------------------------------------------------------- coarsening

mm_status mm_coarsen(mm_context* ctx, const mm_graph* g, double U, int32_t lp_rounds,
                     uint64_t seed, int32_t level_h, int32_t* cluster, mm_coarse** out,
                     int32_t* rounds_run, int64_t* moves) {
  try {
    if (!ctx || !g || !cluster || !out) return fail(MM_EINVAL, "NULL argument");
    if (g->mem != MM_DEVICE) return fail(MM_EINVAL, "mm_coarsen needs a device graph");
    if (g->n < 2 || std::isnan(U) || lp_rounds < 0) return fail(MM_EINVAL, "bad n/U/rounds");
    DeviceGuard dg(ctx->device);
    mm::GraphDev G;
    G.n = g->n; G.nnz = g->nnz;
    G.row_ptr = const_cast<int32_t*>(g->row_ptr);
    G.col = const_cast<int32_t*>(g->col);
    G.c = const_cast<int32_t*>(g->node_w);
    G.w = const_cast<int32_t*>(g->edge_w);
    mm::DevBuf label;
    HIPCHK(label.alloc(sizeof(int32_t) * (size_t)g->n, ctx->stream));
    int32_t rr = 0;
    std::vector<int64_t> mv((size_t)std::max(lp_rounds, 1), 0);
    HIPCHK(mm::lp_cluster(G, U, lp_rounds, seed, level_h, label.as<int32_t>(), &rr, mv.data(),
                          ctx->stream));
    std::unique_ptr<mm_coarse> cg(new mm_coarse());
    HIPCHK(mm::contract(G, label.as<int32_t>(), cluster, &cg->g, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (rounds_run) *rounds_run = rr;
    if (moves) for (int32_t i = 0; i < rr; ++i) moves[i] = mv[(size_t)i];
    *out = cg.release();
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_coarsen");
  }
}

mm_status mm_coarse_graph(const mm_coarse* cg, mm_graph* v) {
  if (!cg || !v) return fail(MM_EINVAL, "NULL argument");
  v->n = cg->g.n;
  v->nnz = cg->g.nnz;
  v->row_ptr = cg->g.row_ptr;
  v->col = cg->g.col;
  v->node_w = cg->g.c;
  v->edge_w = cg->g.w;
  v->mem = MM_DEVICE;
  return MM_OK;
}

void mm_coarse_free(mm_coarse* cg) { delete cg; }

mm_status mm_coarse_export(mm_context* ctx, const mm_coarse* cg, int32_t* row_ptr, int32_t* col,
                           int32_t* node_w, int32_t* edge_w, int32_t mem) {
  if (!ctx || !cg) return fail(MM_EINVAL, "NULL argument");
  if (mem != MM_HOST && mem != MM_DEVICE) return fail(MM_EINVAL, "bad mem kind");
  DeviceGuard dg(ctx->device);
  const hipMemcpyKind kd = mem == MM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const mm::GraphDev& G = cg->g;
  if (row_ptr) HIPCHK(hipMemcpyAsync(row_ptr, G.row_ptr, sizeof(int32_t) * (size_t)(G.n + 1), kd, ctx->stream));
  if (col && G.nnz > 0) HIPCHK(hipMemcpyAsync(col, G.col, sizeof(int32_t) * (size_t)G.nnz, kd, ctx->stream));
  if (node_w) HIPCHK(hipMemcpyAsync(node_w, G.c, sizeof(int32_t) * (size_t)G.n, kd, ctx->stream));
  if (edge_w && G.nnz > 0) HIPCHK(hipMemcpyAsync(edge_w, G.w, sizeof(int32_t) * (size_t)G.nnz, kd, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return MM_OK;
}

// -------------------------------------------------------------- placement

mm_status mm_init_layout(mm_context* ctx, int32_t n, uint64_t seed, int32_t level, float* xy) {
  if (!ctx || !xy || n < 1 || level < 0) return fail(MM_EINVAL, "bad argument");
  DeviceGuard dg(ctx->device);
  HIPCHK(mm::init_layout(n, seed, level, xy, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return MM_OK;
}

mm_status mm_prolong(mm_context* ctx, int32_t n_fine, const int32_t* cluster,
                     const int32_t* coarse_w, const float* coarse_xy, uint64_t seed,
                     int32_t level, float* fine_xy) {
  if (!ctx || !cluster || !coarse_xy || !fine_xy || n_fine < 1 || level < 0)
    return fail(MM_EINVAL, "bad argument");
  DeviceGuard dg(ctx->device);
  HIPCHK(mm::prolong(n_fine, cluster, coarse_w, coarse_xy, seed, level, fine_xy, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return MM_OK;
}

// ------------------------------------------------------------- objectives

mm_status mm_objective(mm_context* ctx, const mm_khop* kh, int32_t level, const int32_t* node_w,
                       double scale, const float* xy, double alpha, double q, double* out) {
  try {
    if (!ctx || !kh || !xy || !out) return fail(MM_EINVAL, "NULL argument");
    if (std::isnan(alpha) || std::isnan(q) || level < 0 || !(scale > 0))
      return fail(MM_EINVAL, "bad level/scale/alpha/q");
    DeviceGuard dg(ctx->device);
    mm::DevBuf sq;
    const float* sqrtc = nullptr;
    if (level > 0) {
      HIPCHK(make_sqrtc(kh->kh.n, node_w, sq, ctx->stream));
      sqrtc = sq.as<float>();
    }
    double parts[3];
    HIPCHK(mm::objective(kh->kh, level, sqrtc, scale, xy, q, parts, ctx->stream));
    // Eq. 1: M = stress over S - alpha * (entropy over the pairs not in S)
    out[0] = parts[0] - alpha * parts[1];
    out[1] = parts[0];
    out[2] = parts[1];
    out[3] = parts[2];
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_objective");
  }
}

mm_status mm_full_stress_ex(mm_context* ctx, const mm_graph* g, const float* xy, int32_t method,
                            double* out) {
  try {
    if (!ctx || !g || !xy || !out) return fail(MM_EINVAL, "NULL argument");
    if (g->mem != MM_DEVICE) return fail(MM_EINVAL, "mm_full_stress needs a device graph");
    if (method < 0 || method > 3) return fail(MM_EINVAL, "method must be 0, 1, 2 or 3");
    if (g->n < 1) return fail(MM_EINVAL, "n < 1");
    if (method == 2 && g->n > 1179648)
      return fail(MM_EUNSUPPORTED, "one BFS per source is limited to n <= 1179648");
    if (method == 3 && g->n > (1 << 23))
      return fail(MM_EUNSUPPORTED, "the banded search is limited to n <= 2^23");
    DeviceGuard dg(ctx->device);
    mm::GraphDev G;
    G.n = g->n; G.nnz = g->nnz;
    G.row_ptr = const_cast<int32_t*>(g->row_ptr);
    G.col = const_cast<int32_t*>(g->col);
    const hipError_t e = mm::full_stress(G, xy, out, ctx->stream, method);
    if (e == hipErrorInvalidValue)
      return fail(MM_EUNSUPPORTED, "graph too large for one BFS per source and of too high a "
                                   "diameter for the multi-source BFS");
    HIPCHK(e);
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_full_stress");
  }
}

mm_status mm_full_stress(mm_context* ctx, const mm_graph* g, const float* xy, double* out) {
  return mm_full_stress_ex(ctx, g, xy, 0, out);
}

// ---------------------------------------------------------------- layout

mm_status mm_layout(mm_context* ctx, const mm_graph* g, const mm_params* p,
                    const float* init_xy, float* out_xy, mm_stats* stats) {
  try {
    if (!ctx || !g || !out_xy) return fail(MM_EINVAL, "NULL argument");
    STCHK(validate_params(p));
    if (g->n < 2) return fail(MM_EINVAL, "graph needs at least 2 vertices (n=%d)", g->n);
    if (g->nnz < 1 || g->nnz >= (1ll << 31)) return fail(MM_EINVAL, "nnz out of range");
    if (g->mem != MM_HOST && g->mem != MM_DEVICE) return fail(MM_EINVAL, "bad mem kind");
    DeviceGuard dg(ctx->device);
    // the layout runs on the context's own stream (capturable into HIP graphs),
    // after the work the caller queued on its stream
    hipStream_t s = ctx->work;
    HIPCHK(hipEventRecord(ctx->ev[3], ctx->stream));
    HIPCHK(hipStreamWaitEvent(s, ctx->ev[3], 0));
    const int32_t n = g->n;
    const int64_t nnz = g->nnz;
    auto t_start = std::chrono::steady_clock::now();

    // host copies for validation and bookkeeping
    std::vector<int32_t> h_rp(n + 1), h_col((size_t)nnz), h_c, h_w;
    const hipMemcpyKind k2h = g->mem == MM_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    HIPCHK(hipMemcpy(h_rp.data(), g->row_ptr, sizeof(int32_t) * (size_t)(n + 1), k2h));
    if (p->validate || g->mem == MM_HOST)
      HIPCHK(hipMemcpy(h_col.data(), g->col, sizeof(int32_t) * (size_t)nnz, k2h));
    if (g->node_w) { h_c.resize(n); HIPCHK(hipMemcpy(h_c.data(), g->node_w, sizeof(int32_t) * (size_t)n, k2h)); }
    if (g->edge_w) { h_w.resize((size_t)nnz); HIPCHK(hipMemcpy(h_w.data(), g->edge_w, sizeof(int32_t) * (size_t)nnz, k2h)); }
    if (p->validate) {
      STCHK(validate_graph(n, nnz, h_rp.data(), h_col.data(), h_c.empty() ? nullptr : h_c.data(),
                           h_w.empty() ? nullptr : h_w.data()));
    } else if (h_rp[0] != 0 || (int64_t)h_rp[n] != nnz) {
      return fail(MM_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] == nnz");
    }
    if (init_xy) {
      std::vector<float> hx(2 * (size_t)n);
      HIPCHK(hipMemcpy(hx.data(), init_xy, sizeof(float) * hx.size(), k2h));
      for (float v : hx) if (!std::isfinite(v)) return fail(MM_EINVAL, "init_xy not finite");
    }

    // level 0 on the device
    std::vector<std::unique_ptr<LevelGraph>> levels;
    levels.emplace_back(new LevelGraph());
    mm::GraphDev& G0 = levels[0]->g;
    G0.n = n;
    G0.nnz = nnz;
    if (g->mem == MM_DEVICE) {
      G0.row_ptr = const_cast<int32_t*>(g->row_ptr);
      G0.col = const_cast<int32_t*>(g->col);
      G0.c = const_cast<int32_t*>(g->node_w);
      G0.w = const_cast<int32_t*>(g->edge_w);
    } else {
      HIPCHK(G0.b_rp.alloc(sizeof(int32_t) * (size_t)(n + 1), s));
      HIPCHK(G0.b_col.alloc(sizeof(int32_t) * (size_t)nnz, s));
      G0.row_ptr = G0.b_rp.as<int32_t>();
      G0.col = G0.b_col.as<int32_t>();
      HIPCHK(hipMemcpyAsync(G0.row_ptr, h_rp.data(), sizeof(int32_t) * (size_t)(n + 1), hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(G0.col, h_col.data(), sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, s));
      if (!h_c.empty()) {
        HIPCHK(G0.b_c.alloc(sizeof(int32_t) * (size_t)n, s));
        G0.c = G0.b_c.as<int32_t>();
        HIPCHK(hipMemcpyAsync(G0.c, h_c.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
      }
      if (!h_w.empty()) {
        HIPCHK(G0.b_w.alloc(sizeof(int32_t) * (size_t)nnz, s));
        G0.w = G0.b_w.as<int32_t>();
        HIPCHK(hipMemcpyAsync(G0.w, h_w.data(), sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, s));
      }
    }
    levels[0]->c_host = h_c;
    HIPCHK(hipStreamSynchronize(s));

    mm_stats st;
    std::memset(&st, 0, sizeof(st));
    double t_coarsen = 0, t_khop = 0, t_far = 0, t_sweep = 0, t_tune = 0;

    // ---- hierarchy (Section 3.1)
    std::vector<mm::DevBuf> clusters;
    auto t0 = std::chrono::steady_clock::now();
    // a warm start refines only the finest level; with approx_h > 0 it still
    // needs the graphs h levels beneath for the cluster far field, so the
    // coarsening stops after h levels (the update protocol of Sec. 4.3)
    const bool cut = init_xy && p->approx_h > 0;
    const int32_t max_lv = cut ? std::min(p->max_levels, p->approx_h) : p->max_levels;
    if (!init_xy || cut) {
      double cV = 0;
      if (h_c.empty()) cV = (double)n;
      else for (int32_t v = 0; v < n; ++v) cV += h_c[v];
      double f = p->f;
      int32_t h = 1, redo = 0;
      while ((int32_t)levels.size() - 1 < max_lv &&
             levels.back()->g.n > std::max(p->coarsest_n, 2)) {
        LevelGraph& L = *levels.back();
        const double W = std::min(std::pow(p->b, (double)h), cV / f);
        int32_t maxc = 1;
        for (int32_t x : L.c_host) maxc = std::max(maxc, x);
        const double U = std::max((double)maxc, W);
        mm::DevBuf label, cluster;
        HIPCHK(label.alloc(sizeof(int32_t) * (size_t)L.g.n, s));
        HIPCHK(cluster.alloc(sizeof(int32_t) * (size_t)L.g.n, s));
        int32_t rr = 0;
        std::vector<int64_t> mv((size_t)std::max(p->lp_rounds, 1), 0);
        HIPCHK(mm::lp_cluster(L.g, U, p->lp_rounds, p->seed, h, label.as<int32_t>(), &rr, mv.data(), s));
        std::unique_ptr<LevelGraph> C(new LevelGraph());
        HIPCHK(mm::contract(L.g, label.as<int32_t>(), cluster.as<int32_t>(), &C->g, s));
        HIPCHK(hipStreamSynchronize(s));
        if (C->g.n > 0.9 * L.g.n) {
          const bool bounded_by_f = (cV / f) < std::pow(p->b, (double)h);
          f = 0.7 * f;
          if (bounded_by_f && redo < 10) { redo++; continue; }
        }
        if (C->g.n >= L.g.n || C->g.n < 2) break;
        C->c_host.resize((size_t)C->g.n);
        HIPCHK(hipMemcpy(C->c_host.data(), C->g.c, sizeof(int32_t) * (size_t)C->g.n, hipMemcpyDeviceToHost));
        levels.push_back(std::move(C));
        clusters.push_back(std::move(cluster));
        h++;
        redo = 0;
      }
    }
    t_coarsen = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    const int32_t Lmax = (int32_t)levels.size() - 1;
    const int32_t top = init_xy ? 0 : Lmax;  // finest-only refinement for a warm start
    st.levels = top + 1;

    // ---- placement of the coarsest level
    mm::DevBuf xa, xb, F, d2;
    const int32_t nL = levels[top]->g.n;
    HIPCHK(xa.alloc(sizeof(float) * 2 * (size_t)nL, s));
    if (init_xy) {
      HIPCHK(hipMemcpyAsync(xa.p, init_xy, sizeof(float) * 2 * (size_t)n,
                            g->mem == MM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    } else {
      HIPCHK(mm::init_layout(nL, p->seed, Lmax, xa.as<float>(), s));
      if (nL == 2) {
        // two vertices: optimal distance (initial layout, Section 3.1)
        float hx[4];
        HIPCHK(hipMemcpyAsync(hx, xa.p, sizeof(hx), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const std::vector<int32_t>& cc = levels[Lmax]->c_host;
        const double c0 = cc.empty() ? 1.0 : cc[0], c1 = cc.empty() ? 1.0 : cc[1];
        const double d = Lmax == 0 ? 1.0 : (std::sqrt(c0) + std::sqrt(c1)) * p->coarse_dist_scale;
        double dx = (double)hx[2] - hx[0], dy = (double)hx[3] - hx[1];
        double D = std::sqrt(dx * dx + dy * dy);
        if (D == 0.0) { dx = 1.0; dy = 0.0; D = 1.0; }
        hx[2] = (float)(hx[0] + d * dx / D);
        hx[3] = (float)(hx[1] + d * dy / D);
        HIPCHK(hipMemcpyAsync(xa.p, hx, sizeof(hx), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
      }
    }
    HIPCHK(d2.alloc(2 * sizeof(double), s));

    // ---- level loop (Section 3.2)
    for (int32_t lvl = top; lvl >= 0; --lvl) {
      mm::GraphDev& G = levels[lvl]->g;
      const int32_t nl = G.n;
      if (lvl < top) {
        HIPCHK(xb.alloc(sizeof(float) * 2 * (size_t)nl, s));
        HIPCHK(mm::prolong(nl, clusters[lvl].as<int32_t>(), levels[lvl + 1]->g.c, xa.as<float>(),
                           p->seed, lvl, xb.as<float>(), s));
        std::swap(xa, xb);
      }
      HIPCHK(xb.alloc(sizeof(float) * 2 * (size_t)nl, s));
      HIPCHK(F.alloc(sizeof(float) * 2 * (size_t)nl, s));
      auto tk = std::chrono::steady_clock::now();
      mm::KhopDev kh;
      mm::KhopCount kc;
      HIPCHK(mm::khop_count(nl, G.row_ptr, G.col, p->k, &kh, &kc, s,
                            p->khop_direct != 0 && p->k == 2));
      // the canonical ids are written only when something reads them: the
      // tuner, the row kernel, or a tile-major copy that cannot be built
      // straight from the search's kept bitmaps
      bool canon = false;
      double khop_ms = 0;
      auto fill_canon = [&]() -> hipError_t {
        if (canon) return hipSuccess;
        canon = true;
        auto tf = std::chrono::steady_clock::now();
        MM_TRY(mm::khop_fill(nl, G.row_ptr, G.col, &kh, &kc, s));
        MM_TRY(hipStreamSynchronize(s));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tf).count();
        khop_ms += ms;
        t_khop += ms;
        return hipSuccess;
      };
      HIPCHK(hipStreamSynchronize(s));
      khop_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tk).count();
      t_khop += khop_ms;
      double lvl_far = 0, lvl_sweep = 0, lvl_wall = 0;
      mm::DevBuf sq;
      const float* sqrtc = nullptr;
      if (lvl > 0) {
        HIPCHK(make_sqrtc(nl, G.c, sq, s));
        sqrtc = sq.as<float>();
      }
      // tile-major sets with LDS-staged coordinates when rows are long enough
      mm::TiledSet ts;
      mm::DevBuf rho;
      // tile size: coarse levels stage sqrt c beside the coordinates (12 B per
      // vertex), so smaller tiles keep two or more work-groups per CU
      int32_t tbits_lvl = lvl == 0 ? mm::kTileBits : (nl >= (1 << 17) ? 12 : 11);
      int32_t group_lvl = 0;  // 0: the sliced layout where tiled, else the row kernel's rule
      int32_t nb_lvl = 0;
      double min_avg = 8.0;
      if (p->autotune) {
        const auto key = std::make_tuple(lvl > 0 ? 1 : 0, nl, kh.total, p->k);
        auto it = ctx->tune.find(key);
        if (it == ctx->tune.end()) {
          HIPCHK(fill_canon());
          auto tt = std::chrono::steady_clock::now();
          mm_context::TuneChoice c;
          STCHK(tune_level(ctx, kh, lvl, sqrtc, p, xa.as<float>(), F.as<float>(), xb.as<float>(),
                           d2.as<double>(), s, &c));
          it = ctx->tune.emplace(key, c).first;
          t_tune += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tt).count();
        }
        tbits_lvl = it->second.tbits;
        group_lvl = it->second.group;
        nb_lvl = it->second.nb;
        min_avg = 0.0;
      }
      if (tbits_lvl > 0 && mm::tiled_eligible(kh, tbits_lvl)) {
        auto tt = std::chrono::steady_clock::now();
        HIPCHK(rho.alloc(sizeof(float) * (size_t)nl, s));
        const bool sliced_lvl = group_lvl == 0 || group_lvl == mm::kSlicedGroup;
        const bool direct = !canon && p->khop_direct && mm::tiled_direct_ok(kh, kc, tbits_lvl);
        if (direct) {
          // big rows straight from their kept bitmaps, the rest from a
          // compact copy of their canonical ids
          mm::DevBuf off_small, nbr_small;
          HIPCHK(mm::khop_fill_small(nl, G.row_ptr, G.col, kh, &kc, &off_small, &nbr_small, s));
          HIPCHK(mm::tiled_build_direct(kh, kc, G.row_ptr, G.col, off_small.as<int64_t>(),
                                        nbr_small.as<int32_t>(), tbits_lvl, min_avg, &ts, s, sqrtc,
                                        p->coarse_dist_scale, rho.as<float>(), sliced_lvl));
        } else {
          HIPCHK(fill_canon());
          tt = std::chrono::steady_clock::now();
          HIPCHK(mm::tiled_build(kh, tbits_lvl, min_avg, &ts, s, sqrtc, p->coarse_dist_scale,
                                 rho.as<float>(), sliced_lvl));
        }
        if (ts.built) kh.b_nbr.release();  // ids now live in the tile-major copy
        HIPCHK(hipStreamSynchronize(s));
        const double tiled_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tt).count();
        t_khop += tiled_ms;
        const char* ev = std::getenv("MM_VERBOSE");
        if (ev && ev[0] == '1')
          std::fprintf(stderr, "[level %d] n %d sets %lld: k-hop build %.1f ms, tile-major copy %.1f ms%s\n",
                       lvl, nl, (long long)kh.total, khop_ms, tiled_ms,
                       direct ? " (straight from the search)" : "");
      }
      // the row kernel reads the canonical ids
      if (!ts.built) HIPCHK(fill_canon());
      kc = mm::KhopCount();  // kept bitmaps no longer needed
      int32_t iters = 0, final_iters = 0, cap_hit = 0;
      double delta = 0;
      mm::DevBuf sweep_part;
      // far field of xin: the cluster far field of Eq. 3 (approx_h > 0, a
      // coarser level exists), else exact all-pairs when theta < 0 or the
      // level has at most exact_below vertices, else Barnes-Hut (with the
      // learned correction when weights are given)
      const bool cf_lvl = p->approx_h > 0 && lvl < Lmax;
      const bool exact_lvl = p->theta < 0 || nl <= p->exact_below;
      mm::ClusterFar cf;
      if (cf_lvl) {
        const int32_t lh = std::min(lvl + p->approx_h, Lmax);
        mm::DevBuf mh, tmp;
        HIPCHK(mh.alloc(sizeof(int32_t) * (size_t)nl, s));
        HIPCHK(hipMemcpyAsync(mh.p, clusters[lvl].p, sizeof(int32_t) * (size_t)nl,
                              hipMemcpyDeviceToDevice, s));
        for (int32_t j = lvl + 1; j < lh; ++j) {
          HIPCHK(tmp.alloc(sizeof(int32_t) * (size_t)nl, s));
          HIPCHK(mm::cluster_compose(nl, mh.as<int32_t>(), clusters[j].as<int32_t>(),
                                     tmp.as<int32_t>(), s));
          std::swap(mh, tmp);
        }
        HIPCHK(mm::cluster_far_setup(nl, clusters[lvl].as<int32_t>(), levels[lvl + 1]->g.n,
                                     mh.as<int32_t>(), levels[lh]->g.n, &cf, s));
        HIPCHK(hipStreamSynchronize(s));
      }
      // The far field runs on the context's far-field stream s2, concurrently
      // with the stress sums of the tiled sweep on s; only the combine (x'
      // from the sums and F) waits for it.  Per iteration: s records ex (xin
      // is final, and the previous combine has read F), s2 waits for ex and
      // computes F, records ej; s runs the stress sums, waits for ej and
      // combines.  The row kernel reads F itself, so on its levels the whole
      // sweep waits for ej.
      hipStream_t s2 = ctx->far;
      auto far = [&](const float* xin) -> hipError_t {
        if (cf_lvl) return mm::cluster_far(cf, xin, G.c, p->q, F.as<float>(), s2);
        if (exact_lvl) return mm::farfield_exact(ctx->bh, nl, xin, p->q, F.as<float>(), s2);
        if (p->mlp_weights)
          return mm::farfield_learned(ctx->bh, nl, xin, p->theta, p->mlp_weights, F.as<float>(), s2);
        return mm::farfield_bh(ctx->bh, nl, xin, p->q, p->theta, F.as<float>(), nullptr, nullptr,
                               nullptr, nullptr, 0, nullptr, s2);
      };
      // The alpha schedule of Section 3.2 runs on the device (the state
      // machine of a batch's graphs, for one graph): after each iteration a
      // one-thread kernel takes the relative change from the combine's sums
      // and writes the alpha of the next iteration, or -1 once the level is
      // done (the sweep then carries x over unchanged).  The host launches
      // up to kIterChunk iterations at a time and reads the state once per
      // chunk, so no iteration waits for a host round trip; a chunk never
      // exceeds the level's largest possible iteration count, so iterations
      // past the stop happen only when the relative change ends it early.
      mm::BatchSched prm;
      prm.alpha_min = p->alpha_min;
      prm.decay = p->alpha_decay;
      prm.eps_round = p->eps_round;
      prm.eps_final = p->eps_final;
      prm.a = p->iters_per_round;
      prm.max_final = p->max_final_iters;
      mm::DevBuf sst, scnt;
      HIPCHK(sst.alloc(sizeof(mm::BatchState), s));
      HIPCHK(scnt.alloc(2 * sizeof(int32_t), s));
      const double alpha_start = init_xy ? p->alpha_min : p->alpha0;
      HIPCHK(mm::batch_sched_init(1, prm, alpha_start, sst.as<mm::BatchState>(), ctx->alpha_dev, s));
      int32_t max_iters = p->max_final_iters;  // every round at full length, then the cap
      for (double a0 = alpha_start; a0 > p->alpha_min; a0 = std::max(a0 * p->alpha_decay, p->alpha_min))
        max_iters += p->iters_per_round;
      // The part of the sweep that does not read F (tiled levels).  On
      // Barnes-Hut levels below kCapMaxN vertices the far field's chain of
      // short kernels takes longer than the sums; there the sums run as
      // kCapPerCU persistent work-groups per compute unit (they fill every
      // wave slot otherwise), so each kernel of the chain finds room at once.
      const bool cap_lvl = !cf_lvl && !exact_lvl && !p->mlp_weights && nl < kCapMaxN;
      const int32_t max_groups = cap_lvl ? (nl < (1 << 16) ? 2 : kCapPerCU) * ctx->cus : 0;
      auto sweep_sums = [&](const float* xin) -> hipError_t {
        if (!ts.built) return hipSuccess;
        return mm::sweep_tiled_partial(ts, lvl, sqrtc, p->coarse_dist_scale, xin, 0.0, p->q, s,
                                       ctx->alpha_dev, group_lvl, nb_lvl, nullptr, nullptr,
                                       max_groups);
      };
      // the part that reads F, the relative-change sums and the schedule step
      auto sweep_finish = [&](const float* xin, float* xout) -> hipError_t {
        if (ts.built)
          MM_TRY(mm::sweep_tiled_combine(ts, rho.as<float>(), xin, F.as<float>(), 0.0, xout,
                                         d2.as<double>(), s, ctx->alpha_dev));
        else
          MM_TRY(mm::sweep(kh, lvl, sqrtc, p->coarse_dist_scale, xin, F.as<float>(), 0.0, p->q,
                           xout, d2.as<double>(), s, nullptr, nullptr, ctx->alpha_dev,
                           &sweep_part, group_lvl));
        return mm::schedule_one(d2.as<double>(), prm, sst.as<mm::BatchState>(), ctx->alpha_dev,
                                scnt.as<int32_t>(), s);
      };
      hipEvent_t ex = ctx->ev[4];
      // After one direct iteration per level (which sizes every buffer), the
      // iteration is captured once per direction (A -> B, B -> A) and
      // replayed.  Levels above kSplitMinN vertices keep three graphs -- far
      // field (launched on s2), stress sums and combine (on s) -- with event
      // records between them, so the far field and the sweep stay timed by
      // HIP events on their own streams; smaller levels, where launches cost
      // more than the work, capture the fork/join of both streams into one
      // graph and split its time in the ratio of the direct iteration.
      float* bufA = xa.as<float>();
      float* bufB = xb.as<float>();
      int parity = 0;  // 0: the current layout is in bufA
      const bool want_graph = p->use_graphs != 0;
      const bool split_graphs = nl > kSplitMinN;
      // far A, far B, sums A, sums B, combine A, combine B
      hipGraphExec_t gx[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
      bool graph_failed = false;
      double split = 0.5;
      struct GraphGuard {
        hipGraphExec_t* g;
        ~GraphGuard() { for (int i = 0; i < 6; ++i) if (g[i]) (void)hipGraphExecDestroy(g[i]); }
      } gguard{gx};
      // six timing events per iteration of a chunk: s before and after the
      // stress sums, before and after the combine; s2 before and after the
      // far field (the last is also the join)
      struct EventSet {
        std::vector<hipEvent_t> e;
        ~EventSet() { for (hipEvent_t x : e) (void)hipEventDestroy(x); }
      } evs;
      evs.e.resize(6 * kIterChunk, nullptr);
      for (auto& x : evs.e) HIPCHK(hipEventCreate(&x));
      struct FarJoin {  // no far-field work outlives the level's graphs and buffers
        hipStream_t s2;
        ~FarJoin() { (void)hipStreamSynchronize(s2); }
      } far_join{s2};
      auto capture_one = [&](hipStream_t cs, hipGraphExec_t* out, auto&& body) -> bool {
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) return false;
        const hipError_t e = body();
        hipGraph_t gr = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &gr);
        if (e != hipSuccess || e2 != hipSuccess || !gr) {
          if (gr) (void)hipGraphDestroy(gr);
          (void)hipGetLastError();
          return false;
        }
        const hipError_t e3 = hipGraphInstantiate(out, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e3 != hipSuccess) { *out = nullptr; (void)hipGetLastError(); return false; }
        return true;
      };
      auto capture = [&]() -> bool {
        hipEvent_t ej = ctx->ev[5];
        for (int d = 0; d < 2; ++d) {
          const float* xin = d ? bufB : bufA;
          float* xout = d ? bufA : bufB;
          if (split_graphs) {
            if (!capture_one(s2, &gx[d], [&]() { return far(xin); })) return false;
            if (!capture_one(s, &gx[2 + d], [&]() { return sweep_sums(xin); })) return false;
            if (!capture_one(s, &gx[4 + d], [&]() { return sweep_finish(xin, xout); })) return false;
          } else {
            if (!capture_one(s, &gx[d], [&]() -> hipError_t {
                  MM_TRY(hipEventRecord(ex, s));
                  MM_TRY(sweep_sums(xin));
                  MM_TRY(hipStreamWaitEvent(s2, ex, 0));
                  MM_TRY(far(xin));
                  MM_TRY(hipEventRecord(ej, s2));
                  MM_TRY(hipStreamWaitEvent(s, ej, 0));
                  return sweep_finish(xin, xout);
                }))
              return false;
          }
        }
        return true;
      };
      // enqueue one iteration (no host wait) with the events of chunk slot r
      int32_t launched = 0;
      auto launch = [&](int r) -> mm_status {
        if (want_graph && launched >= 1 && !gx[0] && !graph_failed) {
          if (!capture()) {
            graph_failed = true;
            for (auto& g2 : gx) if (g2) { (void)hipGraphExecDestroy(g2); g2 = nullptr; }
          }
        }
        const float* xin = parity ? bufB : bufA;
        float* xout = parity ? bufA : bufB;
        hipEvent_t* E = &evs.e[6 * r];
        if (gx[parity] && !split_graphs) {
          HIPCHK(hipEventRecord(E[0], s));
          HIPCHK(hipGraphLaunch(gx[parity], s));
          HIPCHK(hipEventRecord(E[3], s));
        } else {
          // fork: the stress sums on s are enqueued first, so the GPU starts
          // them while the host is still launching the far field of xin on s2
          HIPCHK(hipEventRecord(ex, s));
          HIPCHK(hipEventRecord(E[0], s));
          if (gx[parity]) HIPCHK(hipGraphLaunch(gx[2 + parity], s));
          else HIPCHK(sweep_sums(xin));
          HIPCHK(hipEventRecord(E[1], s));
          HIPCHK(hipStreamWaitEvent(s2, ex, 0));
          HIPCHK(hipEventRecord(E[4], s2));
          if (gx[parity]) HIPCHK(hipGraphLaunch(gx[parity], s2));
          else HIPCHK(far(xin));
          HIPCHK(hipEventRecord(E[5], s2));
          // join, then the combine
          HIPCHK(hipStreamWaitEvent(s, E[5], 0));
          HIPCHK(hipEventRecord(E[2], s));
          if (gx[parity]) HIPCHK(hipGraphLaunch(gx[4 + parity], s));
          else HIPCHK(sweep_finish(xin, xout));
          HIPCHK(hipEventRecord(E[3], s));
        }
        parity ^= 1;
        launched++;
        return MM_OK;
      };
      // the times of an iteration of the chunk (after the chunk's wait)
      auto account = [&](int r, bool direct_split) -> mm_status {
        hipEvent_t* E = &evs.e[6 * r];
        float a = 0, b = 0, wall = 0;
        if (!direct_split) {
          HIPCHK(hipEventElapsedTime(&wall, E[0], E[3]));
          a = (float)(wall * split);
          b = (float)(wall * (1.0 - split));
        } else {
          float b1 = 0, b2 = 0;
          HIPCHK(hipEventElapsedTime(&a, E[4], E[5]));
          HIPCHK(hipEventElapsedTime(&b1, E[0], E[1]));
          HIPCHK(hipEventElapsedTime(&b2, E[2], E[3]));
          HIPCHK(hipEventElapsedTime(&wall, E[0], E[3]));
          b = b1 + b2;
        }
        t_far += a;
        t_sweep += b;
        lvl_far += a;
        lvl_sweep += b;
        lvl_wall += wall;
        return MM_OK;
      };
      mm::BatchState* hstate = reinterpret_cast<mm::BatchState*>(ctx->pinned + 8);
      int32_t* hcnt = reinterpret_cast<int32_t*>(ctx->pinned + 14);
      for (;;) {
        const int32_t chunk = std::max<int32_t>(1, std::min<int32_t>(
            launched == 0 ? 1 : kIterChunk, max_iters - launched));
        const int32_t first = launched;
        bool single_graph[kIterChunk];
        for (int32_t r = 0; r < chunk; ++r) {
          STCHK(launch(r));
          single_graph[r] = gx[(parity ^ 1)] != nullptr && !split_graphs;
        }
        HIPCHK(hipMemcpyAsync(hstate, sst.p, sizeof(mm::BatchState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hcnt, scnt.p, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const mm::BatchState S = *hstate;
        // (the counters describe the chunk's last step; a non-finite layout
        // also leaves the state in phase 3)
        if (hcnt[1] > 0 || S.phase == 3) return fail(MM_EINTERNAL, "non-finite layout at level %d", lvl);
        for (int32_t r = 0; r < chunk; ++r) {
          if (first + r >= S.iters) break;  // past the level's stop: copies only
          STCHK(account(r, !single_graph[r]));
          // the direct iteration sets the far / sweep ratio of single graphs
          if (first + r == 0 && !split_graphs) {
            float a = 0, b1 = 0, b2 = 0;
            HIPCHK(hipEventElapsedTime(&a, evs.e[6 * r + 4], evs.e[6 * r + 5]));
            HIPCHK(hipEventElapsedTime(&b1, evs.e[6 * r], evs.e[6 * r + 1]));
            HIPCHK(hipEventElapsedTime(&b2, evs.e[6 * r + 2], evs.e[6 * r + 3]));
            if (a + b1 + b2 > 0) split = a / (a + b1 + b2);
          }
        }
        iters = S.iters;
        final_iters = S.final_iters;
        cap_hit = S.cap_hit;
        delta = S.delta;
        if (hcnt[0] == 0 || launched >= max_iters) break;
      }
      if (parity) std::swap(xa, xb);  // the level's result in xa
      if (lvl < MM_MAX_LEVELS) {
        st.level_n[lvl] = nl;
        st.level_nnz[lvl] = G.nnz;
        st.level_khop[lvl] = kh.total;
        st.level_iters[lvl] = iters;
        st.level_final_iters[lvl] = final_iters;
        st.level_cap_hit[lvl] = cap_hit;
        st.level_delta[lvl] = delta;
        st.level_sweep_ms[lvl] = lvl_sweep;
        st.level_far_ms[lvl] = lvl_far;
        st.level_wall_ms[lvl] = lvl_wall;
        st.level_khop_ms[lvl] = khop_ms;
        st.level_tile_bits[lvl] = ts.built ? ts.tbits : 0;
        st.level_blocks[lvl] = ts.built ? (nb_lvl > 0 ? nb_lvl : mm::tiled_blocks(ts)) : 0;
        st.level_group[lvl] = group_lvl > 0 ? group_lvl
                                            : (ts.built ? (ts.sliced ? mm::kSlicedGroup : mm::tiled_group(ts))
                                                        : mm::row_group(kh));
      }
      st.vertex_updates += (int64_t)nl * iters;
      st.t_iterate_ms += lvl_wall;
      if (lvl == 0) st.finest_updates = (int64_t)nl * iters;
    }
    HIPCHK(hipMemcpyAsync(out_xy, xa.p, sizeof(float) * 2 * (size_t)n,
                          g->mem == MM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    st.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    st.t_coarsen_ms = t_coarsen;
    st.t_khop_ms = t_khop;
    st.t_farfield_ms = t_far;
    st.t_sweep_ms = t_sweep;
    st.t_tune_ms = t_tune;
    st.t_other_ms = st.t_total_ms - t_coarsen - t_khop - st.t_iterate_ms - t_tune;
    if (stats) *stats = st;
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_layout");
  }
}

}  // extern "C"

// ------------------------------------------------------------------ batches

namespace {

// One level of a batch: the union of the graphs still present at this level.
struct BatchLevel {
  mm::GraphDev g;
  std::vector<int32_t> orig;     // batch index of every member graph
  std::vector<int32_t> goff_h;   // member vertex offsets (M+1)
  mm::DevBuf d_gid, d_goff;      // per-vertex member index, offsets
  mm::DevBuf cl;                 // vertex -> next level vertex, -1 = graph stops here
  std::vector<uint8_t> top;      // member's coarsest level is this one
  int32_t M() const { return (int32_t)orig.size(); }
};

mm_status upload_offsets(BatchLevel& L, hipStream_t s) {
  const int32_t M = L.M();
  HIPCHK(L.d_goff.alloc(sizeof(int32_t) * (size_t)(M + 1), s));
  HIPCHK(hipMemcpyAsync(L.d_goff.p, L.goff_h.data(), sizeof(int32_t) * (size_t)(M + 1),
                        hipMemcpyHostToDevice, s));
  HIPCHK(L.d_gid.alloc(sizeof(int32_t) * (size_t)std::max(L.g.n, 1), s));
  HIPCHK(mm::batch_fill_gid(M, L.d_goff.as<int32_t>(), L.d_gid.as<int32_t>(), s));
  return MM_OK;
}

}  // namespace

extern "C" {

mm_status mm_layout_batch(mm_context* ctx, int32_t G, const int64_t* graph_off, const mm_graph* g,
                          const mm_params* p, const float* init_xy, float* out_xy,
                          int32_t* graph_levels, mm_stats* stats) {
  try {
    if (!ctx || !g || !out_xy || !graph_off) return fail(MM_EINVAL, "NULL argument");
    STCHK(validate_params(p));
    if (p->theta < 0) return fail(MM_EUNSUPPORTED, "batches use the Barnes-Hut far field (theta >= 0)");
    if (p->exact_below != 0) return fail(MM_EUNSUPPORTED, "batches use Barnes-Hut on every level (exact_below must be 0)");
    if (p->mlp_weights) return fail(MM_EUNSUPPORTED, "batches use the plain Barnes-Hut far field");
    if (G < 1) return fail(MM_EINVAL, "G < 1");
    if (g->mem != MM_HOST && g->mem != MM_DEVICE) return fail(MM_EINVAL, "bad mem kind");
    if (graph_off[0] != 0 || graph_off[G] != (int64_t)g->n) return fail(MM_EINVAL, "graph_off must run from 0 to n");
    for (int32_t i = 0; i < G; ++i)
      if (graph_off[i + 1] - graph_off[i] < 2) return fail(MM_EINVAL, "graph %d has fewer than 2 vertices", i);
    if (g->nnz < 1 || g->nnz >= (1ll << 31)) return fail(MM_EINVAL, "nnz out of range");
    DeviceGuard dg(ctx->device);
    hipStream_t s = ctx->work;
    HIPCHK(hipEventRecord(ctx->ev[3], ctx->stream));
    HIPCHK(hipStreamWaitEvent(s, ctx->ev[3], 0));
    const int32_t n = g->n;
    const int64_t nnz = g->nnz;
    auto t_start = std::chrono::steady_clock::now();

    std::vector<int32_t> h_rp(n + 1), h_col((size_t)nnz), h_c;
    const hipMemcpyKind k2h = g->mem == MM_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    HIPCHK(hipMemcpy(h_rp.data(), g->row_ptr, sizeof(int32_t) * (size_t)(n + 1), k2h));
    HIPCHK(hipMemcpy(h_col.data(), g->col, sizeof(int32_t) * (size_t)nnz, k2h));
    if (g->node_w) { h_c.resize(n); HIPCHK(hipMemcpy(h_c.data(), g->node_w, sizeof(int32_t) * (size_t)n, k2h)); }
    if (p->validate) {
      std::vector<int32_t> h_w;
      if (g->edge_w) { h_w.resize((size_t)nnz); HIPCHK(hipMemcpy(h_w.data(), g->edge_w, sizeof(int32_t) * (size_t)nnz, k2h)); }
      STCHK(validate_graph(n, nnz, h_rp.data(), h_col.data(), h_c.empty() ? nullptr : h_c.data(),
                           h_w.empty() ? nullptr : h_w.data()));
    } else if (h_rp[0] != 0 || (int64_t)h_rp[n] != nnz) {
      return fail(MM_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] == nnz");
    }
    // edges stay inside their graph
    for (int32_t i = 0; i < G; ++i)
      for (int64_t v = graph_off[i]; v < graph_off[i + 1]; ++v)
        for (int32_t e = h_rp[v]; e < h_rp[v + 1]; ++e)
          if (h_col[e] < graph_off[i] || h_col[e] >= graph_off[i + 1])
            return fail(MM_EINVAL, "edge %lld-%d leaves graph %d", (long long)v, h_col[e], i);
    if (init_xy) {
      std::vector<float> hx(2 * (size_t)n);
      HIPCHK(hipMemcpy(hx.data(), init_xy, sizeof(float) * hx.size(), k2h));
      for (float v : hx) if (!std::isfinite(v)) return fail(MM_EINVAL, "init_xy not finite");
    }

    // level 0: the whole batch
    std::vector<std::unique_ptr<BatchLevel>> levels;
    levels.emplace_back(new BatchLevel());
    {
      BatchLevel& L0 = *levels[0];
      L0.g.n = n;
      L0.g.nnz = nnz;
      HIPCHK(L0.g.b_rp.alloc(sizeof(int32_t) * (size_t)(n + 1), s));
      HIPCHK(L0.g.b_col.alloc(sizeof(int32_t) * (size_t)nnz, s));
      L0.g.row_ptr = L0.g.b_rp.as<int32_t>();
      L0.g.col = L0.g.b_col.as<int32_t>();
      HIPCHK(hipMemcpyAsync(L0.g.row_ptr, h_rp.data(), sizeof(int32_t) * (size_t)(n + 1), hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(L0.g.col, h_col.data(), sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, s));
      if (!h_c.empty()) {
        HIPCHK(L0.g.b_c.alloc(sizeof(int32_t) * (size_t)n, s));
        L0.g.c = L0.g.b_c.as<int32_t>();
        HIPCHK(hipMemcpyAsync(L0.g.c, h_c.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
      }
      if (g->edge_w) {
        HIPCHK(L0.g.b_w.alloc(sizeof(int32_t) * (size_t)nnz, s));
        L0.g.w = L0.g.b_w.as<int32_t>();
        HIPCHK(hipMemcpyAsync(L0.g.w, g->edge_w, sizeof(int32_t) * (size_t)nnz,
                              g->mem == MM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
      }
      L0.orig.resize(G);
      L0.goff_h.resize(G + 1);
      for (int32_t i = 0; i < G; ++i) L0.orig[i] = i;
      for (int32_t i = 0; i <= G; ++i) L0.goff_h[i] = (int32_t)graph_off[i];
      STCHK(upload_offsets(L0, s));
    }

    // ---- hierarchy, every graph with its own U, f and stopping point
    std::vector<double> cV(G, 0.0), f(G, p->f);
    std::vector<int32_t> redo(G, 0), nlev(G, 1);
    std::vector<uint8_t> alive(G, init_xy ? 0 : 1);
    for (int32_t i = 0; i < G; ++i) {
      if (h_c.empty()) cV[i] = (double)(graph_off[i + 1] - graph_off[i]);
      else for (int64_t v = graph_off[i]; v < graph_off[i + 1]; ++v) cV[i] += h_c[v];
    }
    auto t0 = std::chrono::steady_clock::now();
    for (int32_t h = 1;; ++h) {
      BatchLevel& cur = *levels.back();
      const int32_t M = cur.M();
      std::vector<uint8_t> cand(M, 0);
      bool any = false;
      for (int32_t m = 0; m < M; ++m) {
        const int32_t gi = cur.orig[m];
        const int32_t nm = cur.goff_h[m + 1] - cur.goff_h[m];
        cand[m] = alive[gi] && (h - 1) < p->max_levels && nm > std::max(p->coarsest_n, 2);
        if (!cand[m]) alive[gi] = 0;
        any = any || cand[m];
      }
      if (!any) break;
      std::vector<int32_t> maxc(M, 1);
      if (cur.g.c) {
        mm::DevBuf dm;
        HIPCHK(dm.alloc(sizeof(int32_t) * (size_t)M, s));
        HIPCHK(mm::batch_max_c(M, cur.d_goff.as<int32_t>(), cur.g.c, dm.as<int32_t>(), s));
        HIPCHK(hipMemcpyAsync(maxc.data(), dm.p, sizeof(int32_t) * (size_t)M, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
      }
      auto Uof = [&](int32_t m) {
        const int32_t gi = cur.orig[m];
        const double W = std::min(std::pow(p->b, (double)h), cV[gi] / f[gi]);
        return std::max((double)maxc[m], W);
      };
      std::vector<double> U(M, 1.0);
      for (int32_t m = 0; m < M; ++m) if (cand[m]) U[m] = Uof(m);
      // decision per member: 0 pending, 1 accept, 2 stop
      std::vector<int32_t> decide(M, 0);
      for (int32_t m = 0; m < M; ++m) if (!cand[m]) decide[m] = 2;
      mm::DevBuf d_U, d_stop, label, cluster, gidc, goffc;
      HIPCHK(d_U.alloc(sizeof(double) * (size_t)M, s));
      HIPCHK(d_stop.alloc(sizeof(int32_t) * (size_t)M, s));
      HIPCHK(label.alloc(sizeof(int32_t) * (size_t)cur.g.n, s));
      HIPCHK(cluster.alloc(sizeof(int32_t) * (size_t)cur.g.n, s));
      std::unique_ptr<mm::GraphDev> C;
      std::vector<int32_t> goffc_h(M + 1);
      for (;;) {
        std::vector<int32_t> stop(M);
        for (int32_t m = 0; m < M; ++m) stop[m] = cand[m] ? 0 : 1;
        HIPCHK(hipMemcpyAsync(d_U.p, U.data(), sizeof(double) * (size_t)M, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_stop.p, stop.data(), sizeof(int32_t) * (size_t)M, hipMemcpyHostToDevice, s));
        mm::LpSeg seg;
        seg.M = M;
        seg.gid = cur.d_gid.as<int32_t>();
        seg.goff = cur.d_goff.as<int32_t>();
        seg.Ug = d_U.as<double>();
        seg.gstop = d_stop.as<int32_t>();
        int32_t rr = 0;
        HIPCHK(mm::lp_cluster(cur.g, 0.0, p->lp_rounds, p->seed, h, label.as<int32_t>(), &rr, nullptr,
                              s, &seg));
        C.reset(new mm::GraphDev());
        HIPCHK(mm::contract(cur.g, label.as<int32_t>(), cluster.as<int32_t>(), C.get(), s));
        HIPCHK(gidc.alloc(sizeof(int32_t) * (size_t)std::max(C->n, 1), s));
        HIPCHK(goffc.alloc(sizeof(int32_t) * (size_t)(M + 1), s));
        HIPCHK(mm::batch_coarse_offsets(cur.g.n, M, C->n, cluster.as<int32_t>(), cur.d_gid.as<int32_t>(),
                                        gidc.as<int32_t>(), goffc.as<int32_t>(), s));
        HIPCHK(hipMemcpyAsync(goffc_h.data(), goffc.p, sizeof(int32_t) * (size_t)(M + 1),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        bool any_redo = false;
        for (int32_t m = 0; m < M; ++m) {
          if (decide[m] != 0) continue;
          const int32_t gi = cur.orig[m];
          const int32_t nm = cur.goff_h[m + 1] - cur.goff_h[m];
          const int32_t nc = goffc_h[m + 1] - goffc_h[m];
          if (nc > 0.9 * nm) {
            const bool bounded_by_f = (cV[gi] / f[gi]) < std::pow(p->b, (double)h);
            f[gi] = 0.7 * f[gi];
            if (bounded_by_f && redo[gi] < 10) {
              redo[gi]++;
              U[m] = Uof(m);
              any_redo = true;
              continue;
            }
          }
          decide[m] = (nc >= nm || nc < 2) ? 2 : 1;
        }
        if (!any_redo) break;
      }
      // next level: the accepted graphs
      std::vector<uint8_t> keep(M, 0);
      std::unique_ptr<BatchLevel> next(new BatchLevel());
      next->goff_h.push_back(0);
      for (int32_t m = 0; m < M; ++m) {
        const int32_t gi = cur.orig[m];
        if (decide[m] == 1) {
          keep[m] = 1;
          next->orig.push_back(gi);
          next->goff_h.push_back(next->goff_h.back() + goffc_h[m + 1] - goffc_h[m]);
          redo[gi] = 0;
          nlev[gi]++;
        } else {
          alive[gi] = 0;
        }
      }
      if (next->orig.empty()) break;
      mm::DevBuf d_keep, cflag, cnewid;
      HIPCHK(d_keep.alloc((size_t)M, s));
      HIPCHK(hipMemcpyAsync(d_keep.p, keep.data(), (size_t)M, hipMemcpyHostToDevice, s));
      HIPCHK(cflag.alloc(sizeof(int32_t) * (size_t)C->n, s));
      HIPCHK(cnewid.alloc(sizeof(int64_t) * (size_t)(C->n + 1), s));
      HIPCHK(mm::batch_subset(*C, gidc.as<int32_t>(), d_keep.as<uint8_t>(), &next->g,
                              cflag.as<int32_t>(), cnewid.as<int64_t>(), s));
      HIPCHK(cur.cl.alloc(sizeof(int32_t) * (size_t)cur.g.n, s));
      HIPCHK(mm::batch_cl_map(cur.g.n, cluster.as<int32_t>(), cflag.as<int32_t>(), cnewid.as<int64_t>(),
                              cur.cl.as<int32_t>(), s));
      STCHK(upload_offsets(*next, s));
      HIPCHK(hipStreamSynchronize(s));
      levels.push_back(std::move(next));
    }
    const double t_coarsen = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    const int32_t H = (int32_t)levels.size() - 1;
    // member flags: coarsest level of the graph
    for (int32_t l = 0; l <= H; ++l) {
      BatchLevel& L = *levels[l];
      L.top.assign(L.M(), 1);
      if (l < H) {
        const BatchLevel& N = *levels[l + 1];
        size_t j = 0;
        for (int32_t m = 0; m < L.M(); ++m) {
          while (j < N.orig.size() && N.orig[j] < L.orig[m]) ++j;
          L.top[m] = (j < N.orig.size() && N.orig[j] == L.orig[m]) ? 0 : 1;
        }
      }
    }

    // ---- levels, coarsest first
    mm_stats st;
    std::memset(&st, 0, sizeof(st));
    st.levels = H + 1;
    double t_khop = 0;
    mm::BatchSched prm;
    prm.alpha_min = p->alpha_min;
    prm.decay = p->alpha_decay;
    prm.eps_round = p->eps_round;
    prm.eps_final = p->eps_final;
    prm.a = p->iters_per_round;
    prm.max_final = p->max_final_iters;
    mm::DevBuf xa, xb, F, d2, gd, gst, galpha, cnt;
    HIPCHK(d2.alloc(2 * sizeof(double), s));
    HIPCHK(cnt.alloc(2 * sizeof(int32_t), s));
    for (int32_t lvl = H; lvl >= 0; --lvl) {
      BatchLevel& L = *levels[lvl];
      const int32_t nl = L.g.n, M = L.M();
      HIPCHK(xb.alloc(sizeof(float) * 2 * (size_t)nl, s));
      if (init_xy) {
        HIPCHK(hipMemcpyAsync(xb.p, init_xy, sizeof(float) * 2 * (size_t)n,
                              g->mem == MM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
      } else {
        if (lvl < H)
          HIPCHK(mm::prolong_seg(nl, L.cl.as<int32_t>(), levels[lvl + 1]->g.c, xa.as<float>(), p->seed,
                                 lvl, L.d_gid.as<int32_t>(), L.d_goff.as<int32_t>(), xb.as<float>(), s));
        mm::DevBuf d_top;
        HIPCHK(d_top.alloc((size_t)M, s));
        HIPCHK(hipMemcpyAsync(d_top.p, L.top.data(), (size_t)M, hipMemcpyHostToDevice, s));
        HIPCHK(mm::init_layout_seg(nl, p->seed, lvl, L.d_gid.as<int32_t>(), L.d_goff.as<int32_t>(),
                                   d_top.as<uint8_t>(), xb.as<float>(), s));
        HIPCHK(mm::place_pairs_seg(M, L.d_goff.as<int32_t>(), d_top.as<uint8_t>(), L.g.c, lvl,
                                   p->coarse_dist_scale, xb.as<float>(), s));
        HIPCHK(hipStreamSynchronize(s));
      }
      std::swap(xa, xb);
      HIPCHK(xb.alloc(sizeof(float) * 2 * (size_t)nl, s));
      HIPCHK(F.alloc(sizeof(float) * 2 * (size_t)nl, s));
      auto tk = std::chrono::steady_clock::now();
      mm::KhopDev kh;
      HIPCHK(mm::khop_build(nl, L.g.row_ptr, L.g.col, p->k, &kh, s));
      HIPCHK(hipStreamSynchronize(s));
      t_khop += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tk).count();
      mm::DevBuf sq;
      const float* sqrtc = nullptr;
      if (lvl > 0) {
        HIPCHK(make_sqrtc(nl, L.g.c, sq, s));
        sqrtc = sq.as<float>();
      }
      HIPCHK(gd.alloc(2 * sizeof(double) * (size_t)M, s));
      HIPCHK(gst.alloc(sizeof(mm::BatchState) * (size_t)M, s));
      HIPCHK(galpha.alloc(sizeof(float) * (size_t)M, s));
      HIPCHK(mm::batch_sched_init(M, prm, init_xy ? p->alpha_min : p->alpha0, gst.as<mm::BatchState>(),
                                  galpha.as<float>(), s));
      // sweep configuration of the union level, as in mm_layout: the tuner's
      // choice for the level's shape (autotune), else the tile-major sliced
      // sweep when the mean (row, tile) chunk has at least 8 entries
      int32_t tbits_lvl = lvl == 0 ? mm::kTileBits : (nl >= (1 << 17) ? 12 : 11);
      int32_t group_lvl = 0, nb_lvl = 0;
      double min_avg = 8.0;
      if (p->autotune) {
        const auto key = std::make_tuple(lvl > 0 ? 1 : 0, nl, kh.total, p->k);
        auto it = ctx->tune.find(key);
        if (it == ctx->tune.end()) {
          mm_context::TuneChoice c;
          STCHK(tune_level(ctx, kh, lvl, sqrtc, p, xa.as<float>(), F.as<float>(), xb.as<float>(),
                           d2.as<double>(), s, &c));
          it = ctx->tune.emplace(key, c).first;
        }
        tbits_lvl = it->second.tbits;
        group_lvl = it->second.group;
        nb_lvl = it->second.nb;
        min_avg = 0.0;
      }
      mm::TiledSet ts;
      mm::DevBuf rho;
      if (tbits_lvl > 0 && mm::tiled_eligible(kh, tbits_lvl)) {
        HIPCHK(rho.alloc(sizeof(float) * (size_t)nl, s));
        HIPCHK(mm::tiled_build(kh, tbits_lvl, min_avg, &ts, s, sqrtc, p->coarse_dist_scale,
                               rho.as<float>(), group_lvl == 0 || group_lvl == mm::kSlicedGroup));
        if (ts.built) kh.b_nbr.release();
        HIPCHK(hipStreamSynchronize(s));
      }
      mm::BHSeg bseg;
      bseg.M = M;
      bseg.gid = L.d_gid.as<int32_t>();
      bseg.goff = L.d_goff.as<int32_t>();
      int32_t launched = 0;  // iterations launched (finished graphs only copy)
      mm::DevBuf sweep_part;
      float* bufA = xa.as<float>();
      float* bufB = xb.as<float>();
      int parity = 0;
      int32_t* hc = reinterpret_cast<int32_t*>(ctx->pinned + 2);
      const int32_t* gidp = L.d_gid.as<int32_t>();
      // one iteration of every graph still running: far field, sweep with the
      // graph's alpha, per-graph relative change, schedule step (counters:
      // graphs still running, graphs with a non-finite layout)
      auto enqueue = [&](const float* xin, float* xout) -> hipError_t {
        MM_TRY(mm::farfield_bh(ctx->bh, nl, xin, p->q, p->theta, F.as<float>(), nullptr, nullptr,
                               nullptr, nullptr, 0, nullptr, s, &bseg));
        if (ts.built) {
          MM_TRY(mm::sweep_tiled_partial(ts, lvl, sqrtc, p->coarse_dist_scale, xin, 0.0, p->q, s,
                                         nullptr, group_lvl, nb_lvl, gidp, galpha.as<float>()));
          MM_TRY(mm::sweep_tiled_combine(ts, rho.as<float>(), xin, F.as<float>(), 0.0, xout,
                                         nullptr, s, nullptr, gidp, galpha.as<float>()));
        } else {
          MM_TRY(mm::sweep(kh, lvl, sqrtc, p->coarse_dist_scale, xin, F.as<float>(), 0.0, p->q,
                           xout, d2.as<double>(), s, gidp, galpha.as<float>(), nullptr,
                           &sweep_part, group_lvl));
        }
        MM_TRY(mm::batch_delta(M, L.d_goff.as<int32_t>(), xin, xout, gd.as<double>(), s,
                               cnt.as<int32_t>()));
        return mm::batch_schedule(M, gd.as<double>(), prm, gst.as<mm::BatchState>(),
                                  galpha.as<float>(), cnt.as<int32_t>(), s);
      };
      auto readback = [&]() -> hipError_t {
        return hipMemcpyAsync(hc, cnt.p, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
      };
      // The union iterates until its last graph is done; the device-side
      // schedule decides each graph's alpha and stop, so the host only needs
      // the count of running graphs.  After two direct iterations (the first
      // sizes every buffer; two keep the parity), kBatchReplay iterations are
      // captured into one HIP graph and replayed with one host check per
      // replay; iterations past the last graph's stop copy the coordinates
      // of the finished graphs and leave the layout unchanged.
      hipGraphExec_t gxr = nullptr;
      struct GraphGuard {
        hipGraphExec_t* g;
        ~GraphGuard() { if (*g) (void)hipGraphExecDestroy(*g); }
      } gguard{&gxr};
      bool gfail = !p->use_graphs;
      for (;;) {
        if (launched >= 2 && !gxr && !gfail) {
          hipGraph_t gr = nullptr;
          if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
            gfail = true;
          } else {
            hipError_t e = hipSuccess;
            for (int32_t r = 0; r < kBatchReplay && e == hipSuccess; ++r)
              e = enqueue((r & 1) ? bufB : bufA, (r & 1) ? bufA : bufB);
            if (e == hipSuccess) e = readback();
            const hipError_t e2 = hipStreamEndCapture(s, &gr);
            if (e != hipSuccess || e2 != hipSuccess || !gr ||
                hipGraphInstantiate(&gxr, gr, nullptr, nullptr, 0) != hipSuccess) {
              gfail = true;
              gxr = nullptr;
            }
            if (gr) (void)hipGraphDestroy(gr);
            if (gfail) (void)hipGetLastError();
          }
        }
        if (gxr && parity == 0) {
          HIPCHK(hipGraphLaunch(gxr, s));
          launched += kBatchReplay;
        } else {
          HIPCHK(enqueue(parity ? bufB : bufA, parity ? bufA : bufB));
          HIPCHK(readback());
          parity ^= 1;
          launched++;
        }
        HIPCHK(hipStreamSynchronize(s));
        if (hc[1] > 0) return fail(MM_EINTERNAL, "non-finite layout at level %d", lvl);
        if (hc[0] == 0) break;
      }
      if (parity) std::swap(xa, xb);
      // per-graph iteration counts from the device-side schedule
      std::vector<mm::BatchState> hs((size_t)M);
      HIPCHK(hipMemcpy(hs.data(), gst.p, sizeof(mm::BatchState) * (size_t)M, hipMemcpyDeviceToHost));
      int32_t iters = 0, final_iters = 0, caps = 0;
      int64_t updates = 0;
      for (int32_t m = 0; m < M; ++m) {
        iters = std::max(iters, hs[m].iters);
        final_iters = std::max(final_iters, hs[m].final_iters);
        caps += hs[m].cap_hit;
        updates += (int64_t)(L.goff_h[m + 1] - L.goff_h[m]) * hs[m].iters;
      }
      if (lvl < MM_MAX_LEVELS) {
        st.level_n[lvl] = nl;
        st.level_nnz[lvl] = L.g.nnz;
        st.level_khop[lvl] = kh.total;
        st.level_iters[lvl] = iters;
        st.level_final_iters[lvl] = final_iters;
        st.level_cap_hit[lvl] = caps;
        st.level_tile_bits[lvl] = ts.built ? ts.tbits : 0;
        st.level_group[lvl] = group_lvl > 0 ? group_lvl
                                            : (ts.built ? (ts.sliced ? mm::kSlicedGroup : mm::tiled_group(ts))
                                                        : mm::row_group(kh));
        st.level_blocks[lvl] = ts.built ? (nb_lvl > 0 ? nb_lvl : mm::tiled_blocks(ts)) : 0;
      }
      st.vertex_updates += updates;
      if (lvl == 0) st.finest_updates = updates;
    }
    HIPCHK(hipMemcpyAsync(out_xy, xa.p, sizeof(float) * 2 * (size_t)n,
                          g->mem == MM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (graph_levels) for (int32_t i = 0; i < G; ++i) graph_levels[i] = nlev[i];
    st.t_coarsen_ms = t_coarsen;
    st.t_khop_ms = t_khop;
    st.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (stats) *stats = st;
    return MM_OK;
  } catch (...) {
    return fail(MM_EINTERNAL, "exception in mm_layout_batch");
  }
}

}  // extern "C"
