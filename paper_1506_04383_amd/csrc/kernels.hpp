// Host-side launchers of the HIP kernels (internal to libmulment).
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <stdint.h>

namespace mm {

// Blocks of kBigBlock bytes and more are kept for reuse, per device and
// stream: the levels of a layout free and allocate blocks of tens of GB, and
// the device memory pool occasionally takes seconds to provide a fresh one.
// big_alloc hands out the smallest cached block of the caller's device and
// stream that holds b bytes and is at most twice b (else a new block; *cap
// receives the block's size); big_free returns a block to the cache, which
// frees (stream-ordered) its largest blocks beyond 40% of device memory.
// Reuse on the same stream keeps the stream order of the frees.
constexpr size_t kBigBlock = size_t(1) << 30;
hipError_t big_alloc(void** p, size_t b, size_t* cap, hipStream_t s);
void big_free(void* p, size_t cap, hipStream_t s);
size_t big_cached_bytes(int device);
void big_flush(int device);  // frees every cached block of the device
// Blocks are cached only for registered streams (those of live contexts);
// unregistering (reference-counted) frees the stream's cached blocks, so it
// must precede the stream's destruction.
void big_register(hipStream_t s);
void big_unregister(hipStream_t s);

// Stream-ordered temporary device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  size_t cap = 0;  // size of the block behind p (>= bytes for cached blocks)
  hipStream_t s = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), cap(o.cap), s(o.s) {
    o.p = nullptr;
    o.bytes = o.cap = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; cap = o.cap; s = o.s;
      o.p = nullptr;
      o.bytes = o.cap = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  hipError_t alloc(size_t b, hipStream_t st) {
    release();
    s = st;
    bytes = cap = b;
    if (b == 0) return hipSuccess;
    if (b >= kBigBlock) return big_alloc(&p, b, &cap, st);
    return hipMallocAsync(&p, b, st);
  }
  void release() {
    if (p) {
      if (cap >= kBigBlock) big_free(p, cap, s);
      else (void)hipFreeAsync(p, s);
    }
    p = nullptr;
    bytes = cap = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

#define MM_TRY(expr)                                  \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return _e;                  \
  } while (0)

// ---- primitives (prims.hip)
// out[0..n]: exclusive prefix sums of in (out[n] = total).
hipError_t scan_excl_i32(const int32_t* in, int64_t* out, int64_t n, hipStream_t s);
hipError_t scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
// Stable LSD radix sort of (key, val) pairs on the low `bits` bits of key.
// Sorted result ends in keys/vals (the buffers are ping-ponged internally).
// Growable temporaries of the sort, kept by callers that sort every
// iteration (no allocation after the first call: graph-capture safe as long
// as the histogram scan stays on its single-launch path, <= 2^16 entries).
struct SortWork {
  DevBuf k2, v2, hist, offs, sparts;  // sparts: partial sums of the histogram scan
};
// Stable LSD sort of (keys, vals) by the low `bits` bits of the keys.  The
// result is in keys/vals, or, when kout and vout are given, wherever the
// passes left it (*kout, *vout: keys/vals or the work buffers), with no copy.
hipError_t radix_sort_pairs(uint64_t* keys, int32_t* vals, int64_t n, int bits, hipStream_t s,
                            SortWork* ws = nullptr, uint64_t** kout = nullptr,
                            int32_t** vout = nullptr);
hipError_t iota_i32(int32_t* out, int64_t n, hipStream_t s);
hipError_t widen_i32_u64(const int32_t* in, uint64_t* out, int64_t n, hipStream_t s);

// ---- k-hop distance sets (khop.hip)
struct KhopDev {
  int32_t n = 0, k = 0;
  int64_t total = 0;
  int64_t* off = nullptr;  // n+1
  int32_t* hend = nullptr; // n*k
  int32_t* nbr = nullptr;  // total
  DevBuf b_off, b_hend, b_nbr;
};
hipError_t khop_build(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t k,
                      KhopDev* out, hipStream_t s);
// The build in two steps.  khop_count fills off, hend and total; rows whose
// breadth-first search outgrows the per-wave lists ("big" rows, ids in rows)
// are searched with n-bit bitmaps, and for k = 2 their hop-2 bitmaps are
// kept (bmk: row r of rows at bmk + r * Wp, W = ceil(n / 32) words) when
// device memory allows (row pitch Wp = W rounded up to 4 words, so rows
// start 16-byte aligned).  khop_fill writes the canonical ids (nbr) from that
// state; khop_fill_small gives only the other rows' ids, with their own
// offsets (off_small: n + 1 values; the rows' lengths are their last hop
// ends): the fixed slots the counting pass kept (keep_short, k = 2), else a
// compact array.
struct KhopCount {
  int32_t k = 0, W = 0, Wp = 0, slots = 0;
  int64_t nbig = 0;
  size_t shm = 0;
  bool lds_bm = false, one = false, keep = false, test = false;
  int32_t hthr = 0x7fffffff;  // k = 2: vertices with more neighbours have bitmaps in hb
  int32_t orcap = 0;          // hub bitmaps a row may OR (LDS list length)
  DevBuf cnt, big, bigpos, rows, bmk, gbm, gscr, hubidx, hb;
  DevBuf slots_short;  // keep_short, k = 2: short row u's ids at u * 2048 (n * 2048 ids)
};
hipError_t khop_count(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t k,
                      KhopDev* out, KhopCount* st, hipStream_t s, bool keep_short = false);
hipError_t khop_fill(int32_t n, const int32_t* row_ptr, const int32_t* col, KhopDev* out,
                     KhopCount* st, hipStream_t s);
hipError_t khop_fill_small(int32_t n, const int32_t* row_ptr, const int32_t* col,
                           const KhopDev& kh, KhopCount* st, DevBuf* off_small,
                           DevBuf* nbr_small, hipStream_t s);

// ---- tile-major stress sets and the LDS-tiled sweep (tiled.hip)
struct TiledSet {
  int32_t n = 0, tbits = 0, ntiles = 0, nunits = 0;
  int64_t nchunks = 0, total = 0, padded = 0;
  double avg_chunk = 0;
  bool built = false;
  int64_t* rc_ptr = nullptr;     // n+1: row-major chunk slots of each row
  int32_t* chunk_row = nullptr;  // chunks by tile, largest first within a tile
  int64_t* chunk_off = nullptr;  // nchunks+1: entry offsets (multiples of 8)
  int32_t* chunk_slot = nullptr; // row-major slot of each chunk
  uint16_t* ent = nullptr;       // ((v - tile * 2^tbits) << 3) | hop
  int32_t* unit_c0 = nullptr;    // nunits+1: first chunk (sliced: slice) of each work unit
  int32_t* unit_tile = nullptr;  // tile of each work unit
  // sliced layout: the chunks of a tile in slices of 64; block j of the
  // slice's chunk i at block slice_base + 64 j + i (chunk_off = the entry
  // offset of its block 0)
  bool sliced = false;
  int64_t nslices = 0;
  int32_t* slice_c0 = nullptr;   // nslices+1: first chunk of each slice
  int32_t* slice_h = nullptr;    // blocks per chunk of the slice (its first chunk's)
  int64_t* slice_base = nullptr; // nslices+1: first block of each slice
  DevBuf b_rc_ptr, b_chunk_row, b_chunk_off, b_chunk_slot, b_ent, b_unit_c0, b_unit_tile, b_partial,
      b_dpart, b_slice_c0, b_slice_h, b_slice_base;
};
bool tiled_eligible(const KhopDev& kh, int32_t tbits);
// rho_u = sum_{v in S(u)} w_uv (sqrtc null: finest level, d = hop)
hipError_t compute_rho(const KhopDev& kh, const float* sqrtc, double scale, float* rho,
                       hipStream_t s);
// Builds the tile-major copy of kh; when the mean chunk length is below
// min_avg_chunk it stops after counting (ts->built stays false).  With rho
// non-null and the copy built it also fills rho_u: on the finest level
// (sqrtc null) from the hop counts (compute_rho's bits), on coarse levels
// as per-chunk sums added per row in slot order (the same value up to
// rounding order).
// sliced: the sliced layout (k_sweep_sliced) instead of consecutive chunks.
hipError_t tiled_build(const KhopDev& kh, int32_t tbits, double min_avg_chunk, TiledSet* ts,
                       hipStream_t s, const float* sqrtc = nullptr, double scale = 1.0,
                       float* rho = nullptr, bool sliced = false);
// The same tile-major copy built without the canonical ids of the big rows
// (k = 2 with kept hop-2 bitmaps): those rows are read from their CSR row
// and bitmap, the others from off_small / nbr_small (khop_fill_small).  The
// result (entries, chunk order, rho) is identical to tiled_build's on the
// canonical sets.  tiled_direct_ok says whether the state allows it.
bool tiled_direct_ok(const KhopDev& kh, const KhopCount& st, int32_t tbits);
hipError_t tiled_build_direct(const KhopDev& kh, const KhopCount& st, const int32_t* row_ptr,
                              const int32_t* col, const int64_t* off_small,
                              const int32_t* nbr_small, int32_t tbits, double min_avg_chunk,
                              TiledSet* ts, hipStream_t s, const float* sqrtc = nullptr,
                              double scale = 1.0, float* rho = nullptr, bool sliced = false);
// lanes-per-chunk code of the sliced layout in tuner records and forced
// configurations (one lane per chunk, 64 chunks per wave)
constexpr int32_t kSlicedGroup = 64;
constexpr int32_t kTileBits = 13;  // tiled sets need k <= 7 and tbits <= 13
constexpr int32_t kTiledMaxTiles = 4096;  // tiles per level (per-tile counters in LDS)
constexpr int32_t kUnitChunks = 768;      // chunks per work unit (consecutive layout)
constexpr int32_t kUnitSlices = 64;       // slices per work unit (sliced layout)
hipError_t sweep_tiled(const TiledSet& ts, int32_t level, const float* sqrtc, double scale,
                       const float* rho, const float* xy, const float* F, double alpha, double q,
                       float* xy_out, double* delta2_dev, hipStream_t s,
                       const float* alpha_dev = nullptr, int32_t group = 0, int32_t nb = 0);
// The two halves of sweep_tiled: the stress sums of every chunk (reads xy
// only, into the set's partial slots), then the combine of each row with the
// far field F (x' and the relative-change sums).  Only the second needs F, so
// the far field of the same iteration may run concurrently with the first.
// gid/galpha (batches, may be null): alpha of each row's graph, < 0 for a
// finished graph (its rows are copied by the combine).
hipError_t sweep_tiled_partial(const TiledSet& ts, int32_t level, const float* sqrtc, double scale,
                               const float* xy, double alpha, double q, hipStream_t s,
                               const float* alpha_dev = nullptr, int32_t group = 0, int32_t nb = 0,
                               const int32_t* gid = nullptr, const float* galpha = nullptr,
                               int32_t max_groups = 0);
hipError_t sweep_tiled_combine(const TiledSet& ts, const float* rho, const float* xy,
                               const float* F, double alpha, float* xy_out, double* delta2_dev,
                               hipStream_t s, const float* alpha_dev = nullptr,
                               const int32_t* gid = nullptr, const float* galpha = nullptr);
// lanes per chunk (4, 8, 16) the heuristic picks; group = 0 above means this
inline int32_t tiled_group(const TiledSet& ts) {
  return ts.avg_chunk >= 512 ? 16 : ts.avg_chunk >= 128 ? 8 : 4;
}
// 16-byte blocks per lane and step (2, 4) the heuristic picks; nb = 0 above
// means this
inline int32_t tiled_blocks(const TiledSet& ts) { return ts.tbits >= 12 ? 4 : 2; }

// ---- far field (farfield.hip)
struct FarStats { int64_t accepted, leaf_pairs, coincident, nodes; };
struct BHWork;  // persistent buffers, sized by n
// Exact all-pairs far field; w holds the per-slab partial sums (sized here,
// so a first direct call sizes it before any graph capture).
hipError_t farfield_exact(BHWork* w, int32_t n, const float* xy, double q, float* F, hipStream_t s);
// A batch of independent graphs laid out together: graph g owns points
// [goff[g], goff[g+1]) (device arrays; gid[v] = graph of point v).  Each
// graph gets its own box and its own tree.
struct BHSeg {
  int32_t M = 0;
  const int32_t* gid = nullptr;
  const int32_t* goff = nullptr;
};
BHWork* bh_work_create();
void bh_work_destroy(BHWork*);
// Barnes-Hut quadtree far field; optional exports (device pointers, may be null):
// codes[n], order[n], nodes[5*(2n)] (depth, first, count, leaf, prefix per node in pre-order),
// stats (host) receives counters (nodes always; interaction counters when count_stats).
hipError_t farfield_bh(BHWork* w, int32_t n, const float* xy, double q, double theta, float* F,
                       uint64_t* codes_out, int32_t* order_out, int64_t* nodes_out,
                       int64_t* n_nodes_out, int count_stats, FarStats* st, hipStream_t s,
                       const BHSeg* seg = nullptr);

// ---- cluster far field of Eq. 3 (clusterfar.hip)
struct ClusterFar {
  int32_t n = 0, n1 = 0, nh = 0;  // level size, next coarser level, approximation level
  int32_t S = 1, L = 1;           // source slabs and representatives per slab
  DevBuf cl1, clh;                // cluster maps (copies)
  DevBuf ord1, off1, ordh, offh;  // members sorted by cluster, cluster start offsets
  DevBuf rep;                     // float4 (midpoint x, y, nu, 0) per representative
  DevBuf part;                    // slab partial sums
};
// true in *ok when every cl1 value is in [0, n1) and every clh value in [0, nh)
hipError_t cluster_far_check(int32_t n, const int32_t* cl1, int32_t n1, const int32_t* clh,
                             int32_t nh, bool* ok, hipStream_t s);
// out[v] = cl[in[v]]
hipError_t cluster_compose(int32_t n, const int32_t* in, const int32_t* cl, int32_t* out,
                           hipStream_t s);
hipError_t cluster_far_setup(int32_t n, const int32_t* cl1, int32_t n1, const int32_t* clh,
                             int32_t nh, ClusterFar* cf, hipStream_t s);
// allocation-free after the setup (capturable)
hipError_t cluster_far(ClusterFar& cf, const float* xy, const int32_t* c, double q, float* F,
                       hipStream_t s);

// ---- learned far-field correction (learned.hip), q = 0
constexpr int32_t kMlpParams = 4866;  // W1 64x8, b1, W2 64x64, b2, W3 2x64, b3
hipError_t farfield_learned(BHWork* w, int32_t n, const float* xy, double theta, const float* wts,
                            float* F, hipStream_t s);
hipError_t far_samples(BHWork* w, int32_t n, const float* xy, double theta, int64_t cap,
                       int32_t* u_out, int32_t* node_out, float* feat, float* tgt, float* coef,
                       int64_t* count_host, hipStream_t s);
hipError_t mlp_forward(int64_t count, const float* feat, const float* wts, float* out,
                       hipStream_t s);
hipError_t mlp_grad(int64_t count, const float* feat, const float* tgt, const float* wts,
                    float* grad, float* loss_dev, hipStream_t s);
// Initial weights: W1 ~ N(0, 2/8), W2 ~ N(0, 2/64) (He), W3 ~ N(0,
// (out_scale/8)^2), zero biases; normal draws by Box-Muller from SplitMix64
// stream (seed, level 0, tag 65), draws 2p and 2p+1 for parameter p.
hipError_t mlp_init(uint64_t seed, double out_scale, float* wts, hipStream_t s);
hipError_t mlp_train(int64_t N, const float* feat, const float* tgt, float* wts, float* adam,
                     int32_t steps, int32_t batch, double lr, uint64_t seed, int32_t step0,
                     float* losses, hipStream_t s);

// ---- sweep (sweep.hip)
// One Jacobi iteration of Eq. 2 over the k-hop sets. sqrtc: sqrt of node
// weights (null at level 0 => d = hop). delta2 (device, 2 doubles) receives
// sum |x'-x|^2 and sum |x|^2.
// gid/galpha (batches, may be null): alpha of each graph; < 0 = finished
// graph (coordinates copied).  alpha_dev (may be null): alpha read from
// device memory (graph replays).  part_ws: reusable reduction buffer.
hipError_t sweep(const KhopDev& kh, int32_t level, const float* sqrtc, double scale,
                 const float* xy, const float* F, double alpha, double q, float* xy_out,
                 double* delta2_dev, hipStream_t s, const int32_t* gid = nullptr,
                 const float* galpha = nullptr, const float* alpha_dev = nullptr,
                 DevBuf* part_ws = nullptr, int32_t group = 0);
// lanes per row (8, 16, 32, 64) the heuristic picks for the row kernel
inline int32_t row_group(const KhopDev& kh) {
  const double avg = kh.n > 0 ? (double)kh.total / (double)kh.n : 0.0;
  return avg >= 96 ? 64 : avg >= 40 ? 32 : avg >= 16 ? 16 : 8;
}
// work-groups of the row kernel (256 threads, 256/G rows each) = entries of
// its reduction buffer (one double2 per work-group)
inline int32_t sweep_blocks(int32_t n, int32_t G) {
  const int32_t rpb = 256 / G;
  return (n + rpb - 1) / rpb;
}
// The row kernel with a caller-provided reduction buffer (part: part_bytes,
// at least sweep_blocks(n, G) double2) and no allocation; group 0 = the
// heuristic.  hipErrorInvalidValue if the buffer is too small or k > 8.
hipError_t sweep_into(const KhopDev& kh, int32_t level, const float* sqrtc, double scale,
                      const float* xy, const float* F, double alpha, double q, float* xy_out,
                      double* delta2_dev, double2* part, size_t part_bytes, hipStream_t s,
                      const int32_t* gid = nullptr, const float* galpha = nullptr,
                      const float* alpha_dev = nullptr, int32_t group = 0);

// ---- fixed scratch of the no-allocation sweep (noalloc.hip)
// Layout: [0, 16) the two FP64 relative-change sums; [kNoallocPartOff, +
// kNoallocPartBytes) the row kernel's per-work-group partials (at most
// sweep_blocks(n, 64) = n/4 double2); [kNoallocSqrtcOff, + 4n) sqrt of the
// node weights on coarse levels.
constexpr int32_t kNoallocMaxN = 1 << 20;
constexpr size_t kNoallocPartOff = 256;
constexpr size_t kNoallocPartBytes = 16 * (size_t)(kNoallocMaxN / 4);
constexpr size_t kNoallocSqrtcOff = kNoallocPartOff + kNoallocPartBytes;
constexpr size_t kNoallocScratchBytes = kNoallocSqrtcOff + 4 * (size_t)kNoallocMaxN;
// Device address of the scratch copy of `device`, which must be the current
// device; looked up once per device (later calls return the first result).
hipError_t noalloc_scratch_setup(int device, void** out);

// ---- coarsening (coarsen.hip)
struct GraphDev {
  int32_t n = 0;
  int64_t nnz = 0;
  int32_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  int32_t* c = nullptr;  // node weights (null = 1)
  int32_t* w = nullptr;  // edge weights (null = 1)
  DevBuf b_rp, b_col, b_c, b_w;
};
// Runs synchronous size-constrained label propagation; label[n] (device) is
// initialised to v. Returns rounds run in *rounds_run.
// Batches (block-diagonal union of M graphs): graph of each vertex gid,
// vertex offsets goff (M+1), per-graph U (Ug) and stop flags (gstop, in/out:
// graphs flagged take no part; a graph stops after a round without moves).
// Draws are keyed by the local vertex id, so every graph is clustered as it
// would be alone.
struct LpSeg {
  int32_t M = 0;
  const int32_t* gid = nullptr;
  const int32_t* goff = nullptr;
  const double* Ug = nullptr;
  int32_t* gstop = nullptr;
};
hipError_t lp_cluster(const GraphDev& g, double U, int32_t rounds, uint64_t seed, int32_t level_h,
                      int32_t* label, int32_t* rounds_run, int64_t* moves_host, hipStream_t s,
                      const LpSeg* seg = nullptr);
hipError_t contract(const GraphDev& g, const int32_t* label, int32_t* cluster, GraphDev* out,
                    hipStream_t s);

// ---- placement (layout.hip)
hipError_t init_layout(int32_t n, uint64_t seed, int32_t level, float* xy, hipStream_t s);
hipError_t prolong(int32_t n_fine, const int32_t* cluster, const int32_t* coarse_c,
                   const float* coarse_xy, uint64_t seed, int32_t level, float* fine_xy,
                   hipStream_t s);
hipError_t sqrt_weights(int32_t n, const int32_t* c, float* out, hipStream_t s);
// Batches: draws keyed by local vertex ids.  init: graphs flagged in top;
// prolong: vertices with cluster >= 0; pairs: flagged two-vertex graphs.
hipError_t init_layout_seg(int32_t n, uint64_t seed, int32_t level, const int32_t* gid,
                           const int32_t* goff, const uint8_t* top, float* xy, hipStream_t s);
hipError_t prolong_seg(int32_t n_fine, const int32_t* cluster, const int32_t* coarse_c,
                       const float* coarse_xy, uint64_t seed, int32_t level, const int32_t* gid,
                       const int32_t* goff, float* fine_xy, hipStream_t s);
hipError_t place_pairs_seg(int32_t M, const int32_t* goff, const uint8_t* top, const int32_t* c,
                           int32_t level, double scale, float* xy, hipStream_t s);

// ---- batches of independent graphs (batch.hip)
struct BatchSched {
  double alpha_min, decay, eps_round, eps_final;
  int32_t a, max_final;
};
struct BatchState {
  double alpha, delta;
  int32_t phase;  // 0 rounds, 1 final phase at alpha_min, 2 done, 3 non-finite layout
  int32_t k, iters, final_iters, cap_hit, pad;
};
hipError_t batch_fill_gid(int32_t M, const int32_t* goff, int32_t* gid, hipStream_t s);
hipError_t batch_max_c(int32_t M, const int32_t* goff, const int32_t* c, int32_t* out,
                       hipStream_t s);
// out: 2 doubles per graph (sum |x'-x|^2, sum |x|^2)
hipError_t batch_delta(int32_t M, const int32_t* goff, const float* x, const float* xn,
                       double* out, hipStream_t s, int32_t* zero2 = nullptr);
hipError_t batch_sched_init(int32_t M, const BatchSched& prm, double alpha_start, BatchState* st,
                            float* galpha, hipStream_t s);
// counters[0] += graphs still iterating, counters[1] += graphs with a non-finite layout
hipError_t batch_schedule(int32_t M, const double* gd, const BatchSched& prm, BatchState* st,
                          float* galpha, int32_t* counters, hipStream_t s);
// The same step for a single layout (d2: sum |x'-x|^2, sum |x|^2; counters
// zeroed first; alpha: the next iteration's alpha, -1 once finished).
hipError_t schedule_one(const double* d2, const BatchSched& prm, BatchState* st, float* alpha,
                        int32_t* counters, hipStream_t s);
hipError_t batch_coarse_offsets(int32_t n, int32_t M, int32_t nc, const int32_t* cluster,
                                const int32_t* gid, int32_t* gidc, int32_t* goffc, hipStream_t s);
// The graphs flagged in keep (vertex flags / new ids into flag[n], newid[n+1]).
hipError_t batch_subset(const GraphDev& g, const int32_t* gid, const uint8_t* keep, GraphDev* out,
                        int32_t* flag, int64_t* newid, hipStream_t s);
hipError_t batch_cl_map(int32_t n, const int32_t* cluster, const int32_t* cflag,
                        const int64_t* cnewid, int32_t* cl, hipStream_t s);

// ---- objectives (objective.hip)
// out (host, 3 doubles): stress over S, entropy sum over pairs not in S, coincident pairs.
hipError_t objective(const KhopDev& kh, int32_t level, const float* sqrtc, double scale,
                     const float* xy, double q, double* out_host, hipStream_t s);
// out (host, 3 doubles): F unscaled, s*, F(s* x).
// method 0: n <= 65536 one BFS per source; larger graphs the multi-source BFS
// when the diameter is low (at most 64 levels from the first 256 sources),
// else the banded search; 1: multi-source BFS; 2: one BFS per source
// (n <= 1179648); 3: banded search (n <= 2^23)
hipError_t full_stress(const GraphDev& g, const float* xy, double* out_host, hipStream_t s,
                       int32_t method = 0);

}  // namespace mm
