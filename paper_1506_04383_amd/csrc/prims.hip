// Scan and radix-sort primitives (deterministic: fixed tiles, fixed order).
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {

namespace {

constexpr int SCAN_T = 256;          // threads per block
constexpr int SCAN_I = 8;            // items per thread
constexpr int SCAN_TILE = SCAN_T * SCAN_I;

template <typename Tin>
__global__ __launch_bounds__(SCAN_T) void k_tile_sums(const Tin* __restrict__ in, int64_t n,
                                                      int64_t* __restrict__ part) {
  __shared__ int64_t sh[SCAN_T / 64 + 1];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_I; ++i) {
    int64_t j = base + i;
    if (j < n) s += (int64_t)in[j];
  }
  int64_t tot;
  block_excl_scan<int64_t>(s, sh, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Single-block exclusive scan of the tile sums (any count), in place.
__global__ __launch_bounds__(1024) void k_scan_parts(int64_t* part, int64_t m) {
  __shared__ int64_t sh[1024 / 64 + 1];
  int64_t carry = 0;
  for (int64_t b = 0; b < m; b += blockDim.x) {
    int64_t j = b + threadIdx.x;
    int64_t v = j < m ? part[j] : 0;
    int64_t tot;
    int64_t ex = block_excl_scan<int64_t>(v, sh, &tot);
    if (j < m) part[j] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[m] = carry;
}

template <typename Tin>
__global__ __launch_bounds__(SCAN_T) void k_tile_scan(const Tin* __restrict__ in, int64_t n,
                                                      const int64_t* __restrict__ part,
                                                      int64_t* __restrict__ out) {
  __shared__ int64_t sh[SCAN_T / 64 + 1];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
  int64_t v[SCAN_I];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_I; ++i) {
    int64_t j = base + i;
    v[i] = j < n ? (int64_t)in[j] : 0;
    s += v[i];
  }
  int64_t tot;
  int64_t ex = block_excl_scan<int64_t>(s, sh, &tot) + part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_I; ++i) {
    int64_t j = base + i;
    if (j < n) out[j] = ex;
    ex += v[i];
  }
}

// As k_tile_scan, for few tiles (m <= SCAN_FUSE_MAX): each block adds the
// sums of the tiles before it itself (so no separate scan of the sums), and
// the last block also writes the total to out[n].
constexpr int64_t SCAN_FUSE_MAX = 512;
template <typename Tin>
__global__ __launch_bounds__(SCAN_T) void k_tile_scan_fused(const Tin* __restrict__ in, int64_t n,
                                                            const int64_t* __restrict__ part,
                                                            int64_t m, int64_t* __restrict__ out) {
  __shared__ int64_t sh[SCAN_T / 64 + 1];
  int64_t c = 0;
  for (int64_t j = threadIdx.x; j < (int64_t)blockIdx.x; j += SCAN_T) c += part[j];
  int64_t carry;
  block_excl_scan<int64_t>(c, sh, &carry);
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
  int64_t v[SCAN_I];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_I; ++i) {
    int64_t j = base + i;
    v[i] = j < n ? (int64_t)in[j] : 0;
    s += v[i];
  }
  int64_t tot;
  int64_t ex = block_excl_scan<int64_t>(s, sh, &tot) + carry;
#pragma unroll
  for (int i = 0; i < SCAN_I; ++i) {
    int64_t j = base + i;
    if (j < n) out[j] = ex;
    ex += v[i];
  }
  if ((int64_t)blockIdx.x == m - 1 && threadIdx.x == 0) out[n] = carry + tot;
}

__global__ void k_set_last(int64_t* out, int64_t n, const int64_t* part, int64_t m) {
  out[n] = part[m];
}

// Small inputs (n <= 8192): one workgroup, one step of 1024 threads x 8
// consecutive elements.
constexpr int64_t SCAN_SMALL_MAX = 8192;
template <typename Tin>
__global__ __launch_bounds__(1024) void k_scan_small(const Tin* __restrict__ in, int64_t n,
                                                     int64_t* __restrict__ out) {
  constexpr int E = 8;
  __shared__ int64_t sh[1024 / 64 + 1];
  const int64_t j0 = (int64_t)threadIdx.x * E;
  int64_t v[E], t = 0;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    v[i] = j0 + i < n ? (int64_t)in[j0 + i] : 0;
    t += v[i];
  }
  int64_t tot;
  int64_t ex = block_excl_scan<int64_t>(t, sh, &tot);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    if (j0 + i < n) out[j0 + i] = ex;
    ex += v[i];
  }
  if (threadIdx.x == 0) out[n] = tot;
}

template <typename Tin>
hipError_t scan_excl_impl(const Tin* in, int64_t* out, int64_t n, hipStream_t s,
                          DevBuf* ws = nullptr) {
  if (n <= SCAN_SMALL_MAX) {
    k_scan_small<Tin><<<1, 1024, 0, s>>>(in, n, out);
    return hipGetLastError();
  }
  int64_t m = (n + SCAN_TILE - 1) / SCAN_TILE;
  DevBuf local;
  DevBuf& part = ws ? *ws : local;
  if (part.bytes < sizeof(int64_t) * (size_t)(m + 1))
    MM_TRY(part.alloc(sizeof(int64_t) * (size_t)(m + 1), s));
  if (m <= SCAN_FUSE_MAX) {  // two launches instead of four (n > SCAN_SMALL_MAX, so m >= 1)
    k_tile_sums<Tin><<<(unsigned)m, SCAN_T, 0, s>>>(in, n, part.as<int64_t>());
    k_tile_scan_fused<Tin><<<(unsigned)m, SCAN_T, 0, s>>>(in, n, part.as<int64_t>(), m, out);
    return hipGetLastError();
  }
  if (m > 0) {
    k_tile_sums<Tin><<<(unsigned)m, SCAN_T, 0, s>>>(in, n, part.as<int64_t>());
  }
  k_scan_parts<<<1, 1024, 0, s>>>(part.as<int64_t>(), m);
  if (m > 0) {
    k_tile_scan<Tin><<<(unsigned)m, SCAN_T, 0, s>>>(in, n, part.as<int64_t>(), out);
  }
  k_set_last<<<1, 1, 0, s>>>(out, n, part.as<int64_t>(), m);
  return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort
// LSD radix sort of (key, value) pairs, 8 bits per pass; block b holds
// RS_TILE consecutive elements, and its output base for digit d is the count
// of all digits below d plus the counts of digit d in blocks before b; the
// scatter ranks equal digits in input order (stable).  Two forms of the
// per-pass counts, chosen by the block count:
// * up to RS_ONE_MAX blocks (few keys: the launch count matters): digit
//   counts block-major (hist[b * 256 + d]); per pass one 256-thread work-group
//   computes every block's bases, and the scatter also counts the next pass's
//   digits of the elements it writes, per output block (integer atomics into
//   the other of two histogram buffers, which the offset kernel of the pass
//   has cleared: the counts, and so the sort, do not depend on the order of
//   the atomics), so only the first pass has a histogram launch;
// * more blocks: digit-major counts (hist[d * nb + b]) from a histogram
//   launch per pass and their exclusive scan, which are the bases.
constexpr int RS_T = 256;
constexpr int RS_TILE = 1024;  // elements per block (4 steps of RS_T; >= 2 blocks per CU from 2^19 keys)
constexpr int RS_TILE_SH = 10;
constexpr int RS_NW = RS_T / 64;
constexpr int64_t RS_ONE_MAX = 256;  // block-major form up to this many blocks

template <bool BM>
__global__ __launch_bounds__(RS_T) void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                  int shift, int64_t nb,
                                                  int32_t* __restrict__ hist) {
  raise_wave_priority();
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  int64_t end = base + RS_TILE < n ? base + RS_TILE : n;
  for (int64_t j = base + threadIdx.x; j < end; j += RS_T) {
    int d = (int)((keys[j] >> shift) & 255u);
    atomicAdd(&h[d], 1);
  }
  __syncthreads();
  if (BM) hist[(int64_t)blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];
  else hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Block-major form: bases of all nb <= RS_ONE_MAX blocks in one work-group of
// 256 threads (one per digit; a small work-group finds room beside a running
// kernel sooner than a large one); also clears the next pass's histogram
// buffer (if any).
__global__ __launch_bounds__(256) void k_rs_offs_one(const int32_t* __restrict__ hist, int64_t nb,
                                                     int64_t* __restrict__ offs,
                                                     int32_t* __restrict__ clear) {
  raise_wave_priority();
  __shared__ int64_t sh[256 / 64 + 1];
  const int d = threadIdx.x;
  int64_t tot = 0;
#pragma unroll 8
  for (int64_t b = 0; b < nb; ++b) tot += hist[b * 256 + d];
  int64_t all;
  int64_t run = block_excl_scan<int64_t>(tot, sh, &all);
#pragma unroll 8
  for (int64_t b = 0; b < nb; ++b) {
    offs[b * 256 + d] = run;
    run += hist[b * 256 + d];
  }
  if (clear) {
    int4* c4 = reinterpret_cast<int4*>(clear);  // 256 ints per block: 64 int4
    for (int64_t j = d; j < nb * 64; j += 256) c4[j] = make_int4(0, 0, 0, 0);
  }
}

template <bool BM>
__global__ __launch_bounds__(RS_T) void k_rs_scatter(const uint64_t* __restrict__ keys,
                                                     const int32_t* __restrict__ vals, int64_t n,
                                                     int shift, int64_t nb,
                                                     const int64_t* __restrict__ offs,
                                                     uint64_t* __restrict__ okeys,
                                                     int32_t* __restrict__ ovals,
                                                     int32_t* __restrict__ nhist) {
  raise_wave_priority();
  __shared__ int64_t base_d[256];
  __shared__ int32_t wc[RS_NW][256];
  const int t = threadIdx.x, w = t >> 6, l = lane_id();
  base_d[t] = BM ? offs[(int64_t)blockIdx.x * 256 + t] : offs[(int64_t)t * nb + blockIdx.x];
  int64_t tile0 = (int64_t)blockIdx.x * RS_TILE;
  int64_t end = tile0 + RS_TILE < n ? tile0 + RS_TILE : n;
  const uint64_t lt = lanemask_lt();
  for (int64_t c0 = tile0; c0 < end; c0 += RS_T) {
#pragma unroll
    for (int i = 0; i < RS_NW; ++i) wc[i][t] = 0;
    __syncthreads();
    int64_t j = c0 + t;
    bool valid = j < end;
    uint64_t key = valid ? keys[j] : 0;
    int32_t val = valid ? vals[j] : 0;
    int d = (int)((key >> shift) & 255u);
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bb = __ballot((d >> b) & 1);
      m &= ((d >> b) & 1) ? bb : ~bb;
    }
    int rank = __popcll(m & lt);
    if (valid && (m >> l) == 1ull) wc[w][d] = __popcll(m);  // highest lane of its digit group
    __syncthreads();
    if (valid) {
      int64_t pos = base_d[d] + rank;
      for (int i = 0; i < w; ++i) pos += wc[i][d];
      okeys[pos] = key;
      ovals[pos] = val;
      if (BM && nhist)
        atomicAdd(&nhist[(pos >> RS_TILE_SH) * 256 + (int)((key >> (shift + 8)) & 255u)], 1);
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int i = 0; i < RS_NW; ++i) add += wc[i][t];
    base_d[t] += add;
    __syncthreads();
  }
}

__global__ void k_widen(const int32_t* in, uint64_t* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (uint64_t)(uint32_t)in[i];
}

__global__ void k_iota(int32_t* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int32_t)i;
}

}  // namespace

hipError_t scan_excl_i32(const int32_t* in, int64_t* out, int64_t n, hipStream_t s) {
  return scan_excl_impl<int32_t>(in, out, n, s);
}
hipError_t scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  return scan_excl_impl<int64_t>(in, out, n, s);
}

hipError_t iota_i32(int32_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_iota<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, n);
  return hipGetLastError();
}

hipError_t widen_i32_u64(const int32_t* in, uint64_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_widen<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, out, n);
  return hipGetLastError();
}

hipError_t radix_sort_pairs(uint64_t* keys, int32_t* vals, int64_t n, int bits, hipStream_t s,
                            SortWork* ws, uint64_t** kout, int32_t** vout) {
  if (kout) *kout = keys;
  if (vout) *vout = vals;
  if (n <= 1 || bits <= 0) return hipSuccess;
  int passes = (bits + 7) / 8;
  int64_t nb = (n + RS_TILE - 1) / RS_TILE;
  if (nb > (1ll << 30)) return hipErrorInvalidValue;
  const bool bm = nb <= RS_ONE_MAX;
  SortWork local;
  SortWork& W = ws ? *ws : local;
  auto grow = [&](DevBuf& b, size_t bytes) -> hipError_t {
    return b.bytes >= bytes ? hipSuccess : b.alloc(bytes, s);
  };
  MM_TRY(grow(W.k2, sizeof(uint64_t) * (size_t)n));
  MM_TRY(grow(W.v2, sizeof(int32_t) * (size_t)n));
  MM_TRY(grow(W.hist, sizeof(int32_t) * (size_t)((bm ? 2 : 1) * 256 * nb)));
  MM_TRY(grow(W.offs, sizeof(int64_t) * (size_t)(256 * nb + 1)));
  if (!bm && 256 * nb > SCAN_SMALL_MAX)
    MM_TRY(grow(W.sparts, sizeof(int64_t) * (size_t)((256 * nb + SCAN_TILE - 1) / SCAN_TILE + 1)));
  int32_t* hb[2] = {W.hist.as<int32_t>(), W.hist.as<int32_t>() + (bm ? 256 * nb : 0)};
  int64_t* offs = W.offs.as<int64_t>();
  uint64_t* ka = keys; int32_t* va = vals;
  uint64_t* kb = W.k2.as<uint64_t>(); int32_t* vb = W.v2.as<int32_t>();
  if (bm) k_rs_hist<true><<<(unsigned)nb, RS_T, 0, s>>>(ka, n, 0, nb, hb[0]);
  for (int p = 0; p < passes; ++p) {
    if (bm) {
      int32_t* nxt = p + 1 < passes ? hb[(p + 1) & 1] : nullptr;
      k_rs_offs_one<<<1, 256, 0, s>>>(hb[p & 1], nb, offs, nxt);
      k_rs_scatter<true><<<(unsigned)nb, RS_T, 0, s>>>(ka, va, n, 8 * p, nb, offs, kb, vb, nxt);
    } else {
      k_rs_hist<false><<<(unsigned)nb, RS_T, 0, s>>>(ka, n, 8 * p, nb, hb[0]);
      MM_TRY(scan_excl_impl<int32_t>(hb[0], offs, 256 * nb, s, &W.sparts));
      k_rs_scatter<false><<<(unsigned)nb, RS_T, 0, s>>>(ka, va, n, 8 * p, nb, offs, kb, vb,
                                                        nullptr);
    }
    MM_TRY(hipGetLastError());
    uint64_t* tk = ka; ka = kb; kb = tk;
    int32_t* tv = va; va = vb; vb = tv;
  }
  if (ka != keys) {
    if (kout && vout) {  // the caller reads the result where it is
      *kout = ka;
      *vout = va;
    } else {
      MM_TRY(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
      MM_TRY(hipMemcpyAsync(vals, va, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    }
  }
  return hipGetLastError();
}

// ---- cache of big device blocks (see kernels.hpp)
namespace {
struct BigBlock {
  void* p;
  size_t cap;
  hipStream_t s;
  int dev;
};
std::mutex g_big_mu;
std::vector<BigBlock> g_big;
std::vector<std::pair<hipStream_t, int>> g_big_streams;  // registered streams, counts
bool verbose_allocs() {
  static const bool v = [] { const char* e = std::getenv("MM_VERBOSE"); return e && e[0] == '1'; }();
  return v;
}
void big_flush_locked(int dev) {
  for (size_t i = 0; i < g_big.size();) {
    if (g_big[i].dev == dev) {
      (void)hipFreeAsync(g_big[i].p, g_big[i].s);
      g_big[i] = g_big.back();
      g_big.pop_back();
    } else {
      ++i;
    }
  }
}
}  // namespace

hipError_t big_alloc(void** p, size_t b, size_t* cap, hipStream_t s) {
  int dev = 0;
  MM_TRY(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_big_mu);
    size_t best = SIZE_MAX;
    for (size_t i = 0; i < g_big.size(); ++i) {
      const BigBlock& k = g_big[i];
      if (k.dev == dev && k.s == s && k.cap >= b && k.cap / 2 <= b &&
          (best == SIZE_MAX || k.cap < g_big[best].cap))
        best = i;
    }
    if (best != SIZE_MAX) {
      *p = g_big[best].p;
      *cap = g_big[best].cap;
      g_big[best] = g_big.back();
      g_big.pop_back();
      return hipSuccess;
    }
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t e = hipMallocAsync(p, b, s);
  if (e == hipErrorOutOfMemory) {
    // give the cached blocks back and try once more
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(g_big_mu);
      big_flush_locked(dev);
    }
    MM_TRY(hipDeviceSynchronize());
    e = hipMallocAsync(p, b, s);
  }
  *cap = b;
  if (verbose_allocs())
    std::fprintf(stderr, "[alloc] %.2f GB in %.1f ms\n", b / 1e9,
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  return e;
}

void big_free(void* p, size_t cap, hipStream_t s) {
  int dev = 0;
  bool reg = false;
  {
    std::lock_guard<std::mutex> lk(g_big_mu);
    for (const auto& r : g_big_streams) reg = reg || r.first == s;
  }
  // blocks are kept only for streams of live contexts
  if (!reg || hipGetDevice(&dev) != hipSuccess) {
    (void)hipFreeAsync(p, s);
    return;
  }
  size_t freeb = 0, totb = 0;
  (void)hipMemGetInfo(&freeb, &totb);
  const size_t limit = totb / 10 * 4;
  std::lock_guard<std::mutex> lk(g_big_mu);
  g_big.push_back({p, cap, s, dev});
  for (;;) {
    size_t total = 0, big = SIZE_MAX;
    for (size_t i = 0; i < g_big.size(); ++i) {
      if (g_big[i].dev != dev) continue;
      total += g_big[i].cap;
      if (big == SIZE_MAX || g_big[i].cap > g_big[big].cap) big = i;
    }
    if (total <= limit || big == SIZE_MAX) break;
    (void)hipFreeAsync(g_big[big].p, g_big[big].s);
    g_big[big] = g_big.back();
    g_big.pop_back();
  }
}

size_t big_cached_bytes(int device) {
  std::lock_guard<std::mutex> lk(g_big_mu);
  size_t t = 0;
  for (const BigBlock& k : g_big)
    if (k.dev == device) t += k.cap;
  return t;
}

void big_flush(int device) {
  std::lock_guard<std::mutex> lk(g_big_mu);
  big_flush_locked(device);
}

void big_register(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_big_mu);
  for (auto& r : g_big_streams)
    if (r.first == s) { r.second++; return; }
  g_big_streams.push_back({s, 1});
}

void big_unregister(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_big_mu);
  for (size_t i = 0; i < g_big_streams.size(); ++i) {
    if (g_big_streams[i].first != s) continue;
    if (--g_big_streams[i].second > 0) return;
    g_big_streams[i] = g_big_streams.back();
    g_big_streams.pop_back();
    break;
  }
  // the stream may be destroyed next: free its blocks while it is valid
  for (size_t i = 0; i < g_big.size();) {
    if (g_big[i].s == s) {
      (void)hipFreeAsync(g_big[i].p, g_big[i].s);
      g_big[i] = g_big.back();
      g_big.pop_back();
    } else {
      ++i;
    }
  }
}

}  // namespace mm
