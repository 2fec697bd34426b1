// Layout quality measures (Section 4, methodology): the maxent-stress of Eq. 1
// over the stress set S and the full stress over all pairs with BFS hop
// distances at the optimal scale s*.
//
// Maxent-stress: M = sum_{u<v, v in S(u)} w (D - d)^2 - alpha sum_{u<v, v not in S(u)} E_q(D),
// E_0 = ln D, E_q = -D^-q / q.  The entropy sum is taken as (all pairs) minus
// (pairs in S): an LDS-tiled all-pairs kernel plus a pass over the k-hop sets.
// Full stress: one workgroup per source runs a BFS with an LDS bitmap, then
// sums D/d, (D/d)^2 and (D-d)^2/d^2 over v > u; s* = sum(D/d) / sum((D/d)^2)
// minimises sum w (s D - d)^2 for w = d^-2 and
// F(s*) = s*^2 sum (D/d)^2 - 2 s* sum D/d + #pairs.
// All sums are FP64 in a fixed order.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

constexpr int OB_T = 256;

__device__ inline double ent_q(double D, double q) { return q == 0.0 ? log(D) : -pow(D, -q) / q; }

// per block: {stress_S, ent_S, coincident_S} over rows u, pairs v > u
__global__ __launch_bounds__(OB_T) void k_obj_sets(
    int32_t n, int32_t k, const int64_t* __restrict__ off, const int32_t* __restrict__ hend,
    const int32_t* __restrict__ nbr, const float* __restrict__ sqrtc, double scale, int coarse,
    const float2* __restrict__ xy, double q, double* __restrict__ part) {
  __shared__ double sh[3][OB_T];
  const int32_t u = blockIdx.x * OB_T + threadIdx.x;
  double st = 0.0, en = 0.0, co = 0.0;
  if (u < n) {
    const int64_t beg = off[u];
    const float2 xu = xy[u];
    int32_t e = 0;
    for (int h = 1; h <= k; ++h) {
      const int32_t he = hend[(int64_t)u * k + h - 1];
      for (; e < he; ++e) {
        const int32_t v = nbr[beg + e];
        if (v <= u) continue;
        const float2 xv = xy[v];
        const double dx = (double)xu.x - (double)xv.x, dy = (double)xu.y - (double)xv.y;
        const double D = sqrt(dx * dx + dy * dy);
        const double d = coarse ? (double)h * ((double)sqrtc[u] + (double)sqrtc[v]) * scale : (double)h;
        st += (D - d) * (D - d) / (d * d);
        if (D > 0.0) en += ent_q(D, q); else co += 1.0;
      }
    }
  }
  sh[0][threadIdx.x] = st; sh[1][threadIdx.x] = en; sh[2][threadIdx.x] = co;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0, c = 0;
    for (int i = 0; i < OB_T; ++i) { a += sh[0][i]; b += sh[1][i]; c += sh[2][i]; }
    part[3 * blockIdx.x] = a; part[3 * blockIdx.x + 1] = b; part[3 * blockIdx.x + 2] = c;
  }
}

// all pairs u < v: {sum E(D) over D > 0, coincident count}; grid (u-tile, v-tile >= u-tile)
__global__ __launch_bounds__(OB_T) void k_obj_all(int32_t n, const float2* __restrict__ xy, float q,
                                                  int32_t ntiles, double* __restrict__ part) {
  __shared__ float2 tile[OB_T];
  __shared__ double sh[2][OB_T];
  const int32_t tu = blockIdx.y, tv = blockIdx.x;
  double en = 0.0, co = 0.0;
  if (tv >= tu) {
    const int32_t u = tu * OB_T + threadIdx.x;
    const int32_t v0 = tv * OB_T;
    if (v0 + threadIdx.x < n) tile[threadIdx.x] = xy[v0 + threadIdx.x];
    __syncthreads();
    if (u < n) {
      const float2 xu = xy[u];
      const int32_t m = min(OB_T, n - v0);
      for (int32_t j = 0; j < m; ++j) {
        if (v0 + j <= u) continue;
        const float dx = xu.x - tile[j].x, dy = xu.y - tile[j].y;
        const float D2 = dx * dx + dy * dy;
        if (D2 > 0.f) en += (q == 0.f) ? 0.5 * (double)logf(D2) : (double)(-powf(D2, -0.5f * q) / q);
        else co += 1.0;
      }
    }
  }
  sh[0][threadIdx.x] = en; sh[1][threadIdx.x] = co;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int i = 0; i < OB_T; ++i) { a += sh[0][i]; b += sh[1][i]; }
    const int64_t id = (int64_t)tu * ntiles + tv;
    part[2 * id] = a; part[2 * id + 1] = b;
  }
}

constexpr int FS_T = 256;
constexpr int FS_MAXW = 36864;  // LDS bitmap words (n <= 1179648); + 8 KB static < 160 KB

// BIG: the visited bitmap is a static LDS array of FS_MAXW words (dynamic LDS
// is limited to 64 KB per work-group); otherwise it is sized at launch.
template <bool BIG>
__global__ __launch_bounds__(FS_T) void k_full_stress(int32_t n, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      const float2* __restrict__ xy,
                                                      int32_t* __restrict__ gq, int32_t* __restrict__ ghop,
                                                      double* __restrict__ per) {
  extern __shared__ uint32_t bm_dyn[];
  __shared__ uint32_t bm_big[BIG ? FS_MAXW : 1];
  uint32_t* bm = BIG ? bm_big : bm_dyn;
  __shared__ int32_t tail;
  __shared__ double sh[4][FS_T];
  const int32_t W = (n + 31) >> 5;
  int32_t* queue = gq + (size_t)blockIdx.x * n;
  int32_t* hop = ghop + (size_t)blockIdx.x * n;
  for (int32_t i = threadIdx.x; i < W; i += FS_T) bm[i] = 0u;
  __syncthreads();
  for (int32_t u = blockIdx.x; u < n; u += gridDim.x) {
    if (threadIdx.x == 0) {
      bm[u >> 5] |= 1u << (u & 31);
      queue[0] = u;
      hop[u] = 0;
      tail = 1;
    }
    __syncthreads();
    int32_t lo = 0, hi = 1, h = 0;
    while (lo < hi) {
      h++;
      for (int32_t i = lo + threadIdx.x; i < hi; i += FS_T) {
        const int32_t x = queue[i];
        for (int32_t e = rp[x]; e < rp[x + 1]; ++e) {
          const int32_t y = col[e];
          const uint32_t bit = 1u << (y & 31);
          if (bm[y >> 5] & bit) continue;
          const uint32_t old = atomicOr(&bm[y >> 5], bit);
          if (!(old & bit)) {
            const int32_t p = atomicAdd(&tail, 1);
            queue[p] = y;
            hop[y] = h;
          }
        }
      }
      __syncthreads();
      lo = hi;
      hi = tail;
      __syncthreads();
    }
    const float2 xu = xy[u];
    double a1 = 0.0, a2 = 0.0, a0 = 0.0, a3 = 0.0;
    for (int32_t v = u + 1 + threadIdx.x; v < n; v += FS_T) {
      if (!(bm[v >> 5] & (1u << (v & 31)))) continue;
      a3 += 1.0;
      const double d = (double)hop[v];
      const float2 xv = xy[v];
      const double dx = (double)xu.x - (double)xv.x, dy = (double)xu.y - (double)xv.y;
      const double D = sqrt(dx * dx + dy * dy);
      a1 += D / d;
      a2 += (D / d) * (D / d);
      a0 += (D - d) * (D - d) / (d * d);
    }
    sh[0][threadIdx.x] = a1; sh[1][threadIdx.x] = a2; sh[2][threadIdx.x] = a0;
    sh[3][threadIdx.x] = a3;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s1 = 0, s2 = 0, s0 = 0, s3 = 0;
      for (int i = 0; i < FS_T; ++i) { s1 += sh[0][i]; s2 += sh[1][i]; s0 += sh[2][i]; s3 += sh[3][i]; }
      per[4 * (int64_t)u] = s1; per[4 * (int64_t)u + 1] = s2; per[4 * (int64_t)u + 2] = s0;
      per[4 * (int64_t)u + 3] = s3;
    }
    // clear the visited bits of this source
    for (int32_t i = threadIdx.x; i < tail; i += FS_T) {
      const int32_t y = queue[i];
      bm[y >> 5] = 0u;
    }
    __syncthreads();
  }
}

// ---- full stress by bit-parallel multi-source BFS (low-diameter graphs)
// A batch of MS_B = 256 sources advances one level per launch: vertex v's
// sources-reached mask (4 x 64 bits) grows by the OR of its neighbours'
// frontier masks; each newly reached (source, v) pair at level h adds its
// terms with d = h to v's own FP64 accumulators (one wave per vertex, so each
// accumulator has one writer and a fixed order).  Ordered pairs: every
// unordered pair is counted from both ends and the sums are halved.
constexpr int MS_W = 4;           // 64-bit words per vertex mask
constexpr int MS_B = 64 * MS_W;   // sources per batch

__global__ void k_ms_init(int32_t n, int32_t s0, uint64_t* __restrict__ vis,
                          uint64_t* __restrict__ fr) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t b = v - s0;
#pragma unroll
  for (int w = 0; w < MS_W; ++w) {
    const uint64_t m = (b >= 0 && b < MS_B && (b >> 6) == w) ? (1ull << (b & 63)) : 0ull;
    vis[(size_t)v * MS_W + w] = m;
    fr[(size_t)v * MS_W + w] = m;
  }
}

__global__ __launch_bounds__(256) void k_ms_step(
    int32_t n, int32_t s0, int32_t h, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ col, const float2* __restrict__ xy,
    const uint64_t* __restrict__ fr, uint64_t* __restrict__ nx, uint64_t* __restrict__ vis,
    double* __restrict__ acc, int32_t* __restrict__ more) {
  const int32_t v = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = lane_id();
  if (v >= n) return;
  uint64_t a[MS_W] = {0ull, 0ull, 0ull, 0ull};
  for (int32_t e = rp[v] + l; e < rp[v + 1]; e += 64) {
    const uint64_t* f = fr + (size_t)col[e] * MS_W;
#pragma unroll
    for (int w = 0; w < MS_W; ++w) a[w] |= f[w];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int w = 0; w < MS_W; ++w) a[w] |= __shfl_xor(a[w], o, 64);
  uint64_t nw[MS_W];
  bool any = false;
#pragma unroll
  for (int w = 0; w < MS_W; ++w) {
    nw[w] = a[w] & ~vis[(size_t)v * MS_W + w];
    any |= nw[w] != 0ull;
  }
  if (l < MS_W) {
    nx[(size_t)v * MS_W + l] = nw[l];
    vis[(size_t)v * MS_W + l] |= nw[l];
  }
  if (!any) return;
  if (l == 0) *more = 1;
  // pair terms: lane l takes source bit l of every word
  const float2 xv = xy[v];
  const double d = (double)h;
  double a1 = 0.0, a2 = 0.0, a0 = 0.0, np = 0.0;
#pragma unroll
  for (int w = 0; w < MS_W; ++w) {
    if ((nw[w] >> l) & 1ull) {
      const float2 xs = xy[s0 + 64 * w + l];
      const double dx = (double)xs.x - (double)xv.x, dy = (double)xs.y - (double)xv.y;
      const double D = sqrt(dx * dx + dy * dy);
      a1 += D / d;
      a2 += (D / d) * (D / d);
      a0 += (D - d) * (D - d) / (d * d);
      np += 1.0;
    }
  }
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  a0 = wave_sum(a0);
  np = wave_sum(np);
  if (l == 0) {
    acc[4 * (size_t)v] += a1;
    acc[4 * (size_t)v + 1] += a2;
    acc[4 * (size_t)v + 2] += a0;
    acc[4 * (size_t)v + 3] += np;
  }
}

}  // namespace

// Returns false in *done (and leaves out_host alone) when the first batch
// needs more than max_levels levels: a high-diameter graph, for which the
// per-source kernel is the better choice.
hipError_t full_stress_msbfs(const GraphDev& g, const float* xy, int32_t max_levels,
                             double* out_host, bool* done, hipStream_t s) {
  const int32_t n = g.n;
  *done = false;
  DevBuf vis, fr, nx, acc, more;
  MM_TRY(vis.alloc(sizeof(uint64_t) * MS_W * (size_t)n, s));
  MM_TRY(fr.alloc(sizeof(uint64_t) * MS_W * (size_t)n, s));
  MM_TRY(nx.alloc(sizeof(uint64_t) * MS_W * (size_t)n, s));
  MM_TRY(acc.alloc(sizeof(double) * 4 * (size_t)n, s));
  MM_TRY(more.alloc(sizeof(int32_t), s));
  MM_TRY(hipMemsetAsync(acc.p, 0, sizeof(double) * 4 * (size_t)n, s));
  const unsigned nb = (unsigned)((n + 255) / 256), nw = (unsigned)((n + 3) / 4);
  for (int32_t s0 = 0; s0 < n; s0 += MS_B) {
    k_ms_init<<<nb, 256, 0, s>>>(n, s0, vis.as<uint64_t>(), fr.as<uint64_t>());
    MM_TRY(hipGetLastError());
    for (int32_t h = 1;; ++h) {
      if (s0 == 0 && h > max_levels) return hipStreamSynchronize(s);  // *done stays false
      MM_TRY(hipMemsetAsync(more.p, 0, sizeof(int32_t), s));
      k_ms_step<<<nw, 256, 0, s>>>(n, s0, h, g.row_ptr, g.col, (const float2*)xy,
                                   fr.as<uint64_t>(), nx.as<uint64_t>(), vis.as<uint64_t>(),
                                   acc.as<double>(), more.as<int32_t>());
      MM_TRY(hipGetLastError());
      std::swap(fr, nx);
      int32_t hm = 0;
      MM_TRY(hipMemcpyAsync(&hm, more.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      MM_TRY(hipStreamSynchronize(s));
      if (!hm) break;
    }
  }
  std::vector<double> h(4 * (size_t)n);
  MM_TRY(hipMemcpyAsync(h.data(), acc.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  double s1 = 0, s2 = 0, s0s = 0, np = 0;
  for (int32_t u = 0; u < n; ++u) {
    s1 += h[4 * u]; s2 += h[4 * u + 1]; s0s += h[4 * u + 2]; np += h[4 * u + 3];
  }
  s1 *= 0.5; s2 *= 0.5; s0s *= 0.5; np *= 0.5;  // ordered -> unordered pairs
  const double sstar = s2 > 0 ? s1 / s2 : 1.0;
  out_host[0] = s0s;
  out_host[1] = sstar;
  out_host[2] = sstar * sstar * s2 - 2.0 * sstar * s1 + np;
  *done = true;
  return hipSuccess;
}

hipError_t objective(const KhopDev& kh, int32_t level, const float* sqrtc, double scale,
                     const float* xy, double q, double* out_host, hipStream_t s) {
  const int32_t n = kh.n;
  const int32_t nb = (n + OB_T - 1) / OB_T;
  DevBuf p1, p2;
  MM_TRY(p1.alloc(sizeof(double) * 3 * (size_t)nb, s));
  MM_TRY(p2.alloc(sizeof(double) * 2 * (size_t)nb * (size_t)nb, s));
  const int coarse = (level > 0 && sqrtc) ? 1 : 0;
  k_obj_sets<<<nb, OB_T, 0, s>>>(n, kh.k, kh.off, kh.hend, kh.nbr, sqrtc, scale, coarse,
                                 (const float2*)xy, q, p1.as<double>());
  dim3 grid(nb, nb);
  k_obj_all<<<grid, OB_T, 0, s>>>(n, (const float2*)xy, (float)q, nb, p2.as<double>());
  MM_TRY(hipGetLastError());
  std::vector<double> h1(3 * (size_t)nb), h2(2 * (size_t)nb * (size_t)nb);
  MM_TRY(hipMemcpyAsync(h1.data(), p1.p, sizeof(double) * h1.size(), hipMemcpyDeviceToHost, s));
  MM_TRY(hipMemcpyAsync(h2.data(), p2.p, sizeof(double) * h2.size(), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  double st = 0, ens = 0, cos_ = 0, ena = 0, coa = 0;
  for (int32_t b = 0; b < nb; ++b) { st += h1[3 * b]; ens += h1[3 * b + 1]; cos_ += h1[3 * b + 2]; }
  for (size_t b = 0; b < (size_t)nb * nb; ++b) { ena += h2[2 * b]; coa += h2[2 * b + 1]; }
  out_host[0] = st;
  out_host[1] = ena - ens;
  out_host[2] = coa - cos_;
  return hipSuccess;
}

hipError_t full_stress(const GraphDev& g, const float* xy, double* out_host, hipStream_t s,
                       int32_t method) {
  const int32_t n = g.n;
  const int32_t W = (n + 31) >> 5;
  // large graphs of low diameter: the multi-source BFS (tried first, given up
  // after 64 levels of its first batch)
  if (method == 1 || (method == 0 && n > 65536)) {
    bool done = false;
    MM_TRY(full_stress_msbfs(g, xy, method == 1 ? INT32_MAX : 64, out_host, &done, s));
    if (done) return hipSuccess;
  }
  if (W > FS_MAXW) return hipErrorInvalidValue;
  int dev = 0, ncu = 0;
  MM_TRY(hipGetDevice(&dev));
  MM_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int32_t slots = std::min<int32_t>(n, 4 * ncu);
  DevBuf q, hop, per;
  MM_TRY(q.alloc(sizeof(int32_t) * (size_t)n * (size_t)slots, s));
  MM_TRY(hop.alloc(sizeof(int32_t) * (size_t)n * (size_t)slots, s));
  MM_TRY(per.alloc(sizeof(double) * 4 * (size_t)n, s));
  const size_t shm = sizeof(uint32_t) * (size_t)W;
  if (shm <= 65536)
    k_full_stress<false><<<slots, FS_T, shm, s>>>(n, g.row_ptr, g.col, (const float2*)xy,
                                                  q.as<int32_t>(), hop.as<int32_t>(), per.as<double>());
  else
    k_full_stress<true><<<slots, FS_T, 0, s>>>(n, g.row_ptr, g.col, (const float2*)xy,
                                               q.as<int32_t>(), hop.as<int32_t>(), per.as<double>());
  MM_TRY(hipGetLastError());
  std::vector<double> h(4 * (size_t)n);
  MM_TRY(hipMemcpyAsync(h.data(), per.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  double s1 = 0, s2 = 0, s0 = 0, np = 0;
  for (int32_t u = 0; u < n; ++u) {
    s1 += h[4 * u]; s2 += h[4 * u + 1]; s0 += h[4 * u + 2]; np += h[4 * u + 3];
  }
  const double sstar = s2 > 0 ? s1 / s2 : 1.0;
  out_host[0] = s0;
  out_host[1] = sstar;
  out_host[2] = sstar * sstar * s2 - 2.0 * sstar * s1 + np;
  return hipSuccess;
}

}  // namespace mm
