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
  // every source already reached v: nothing new can arrive (late levels of
  // low-diameter graphs, where most vertices are done)
  uint64_t all = ~0ull;
#pragma unroll
  for (int w = 0; w < MS_W; ++w) all &= vis[(size_t)v * MS_W + w];
  if (all == ~0ull) {
    if (l < MS_W) nx[(size_t)v * MS_W + l] = 0ull;
    return;
  }
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


// ---- full stress by banded multi-source search (high-diameter graphs)
// Vertices are renumbered in Morton order of the layout and cut into tiles of
// 64 consecutive ids; batch b takes the 64 vertices of tile b as its sources
// (one bit each).  On a graph whose layout follows its distances the sources
// of a batch are close together, so at level h the vertices that gain bits
// form a thin band around the batch and only the tiles it crosses are
// visited: a tile is visited at level h + 1 when some vertex with new bits at
// level h has a neighbour in it.  One work-group runs a batch from start to
// end with its own frontier and visited masks (work-group barriers between
// levels, no host round trips).  A frontier buffer may keep masks written two
// or more levels earlier; those bits are already in every neighbour's visited
// mask, so they add nothing.  Each unordered pair is counted once, from the
// batch of its smaller new id; every sum has a fixed order (levels, tiles
// ascending, fixed lanes, fixed reductions), so results are reproducible.
constexpr int BS_T = 1024;
constexpr int BS_WAVES = BS_T / 64;
constexpr int BS_U = 8;                 // neighbours gathered at once
constexpr int32_t BS_MAX_WORDS = 2048;  // tile bitmap words (n <= 2^23), 2 x 16 KB LDS

__global__ __launch_bounds__(256) void k_bs_bbox_part(int32_t n, const float2* __restrict__ xy,
                                                     float4* __restrict__ part) {
  __shared__ float4 sh[4];
  float4 m = make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY);
  for (int32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float2 p = xy[i];
    m.x = fminf(m.x, p.x); m.y = fminf(m.y, p.y); m.z = fmaxf(m.z, p.x); m.w = fmaxf(m.w, p.y);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m.x = fminf(m.x, __shfl_xor(m.x, o, 64)); m.y = fminf(m.y, __shfl_xor(m.y, o, 64));
    m.z = fmaxf(m.z, __shfl_xor(m.z, o, 64)); m.w = fmaxf(m.w, __shfl_xor(m.w, o, 64));
  }
  if (lane_id() == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      m.x = fminf(m.x, sh[w].x); m.y = fminf(m.y, sh[w].y);
      m.z = fmaxf(m.z, sh[w].z); m.w = fmaxf(m.w, sh[w].w);
    }
    part[blockIdx.x] = m;
  }
}

__global__ __launch_bounds__(64) void k_bs_bbox_final(int32_t np, float4* __restrict__ part) {
  float4 m = make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY);
  for (int32_t i = threadIdx.x; i < np; i += 64) {
    const float4 q = part[i];
    m.x = fminf(m.x, q.x); m.y = fminf(m.y, q.y); m.z = fmaxf(m.z, q.z); m.w = fmaxf(m.w, q.w);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m.x = fminf(m.x, __shfl_xor(m.x, o, 64)); m.y = fminf(m.y, __shfl_xor(m.y, o, 64));
    m.z = fmaxf(m.z, __shfl_xor(m.z, o, 64)); m.w = fmaxf(m.w, __shfl_xor(m.w, o, 64));
  }
  __syncthreads();
  if (threadIdx.x == 0) part[0] = m;
}

__device__ inline uint32_t bs_spread16(uint32_t a) {
  a = (a | (a << 8)) & 0x00FF00FFu;
  a = (a | (a << 4)) & 0x0F0F0F0Fu;
  a = (a | (a << 2)) & 0x33333333u;
  a = (a | (a << 1)) & 0x55555555u;
  return a;
}

// Morton key of 16-bit cell coordinates in the bounding box box[0]
__global__ void k_bs_keys(int32_t n, const float2* __restrict__ xy, const float4* __restrict__ box,
                          uint64_t* __restrict__ keys, int32_t* __restrict__ ids) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 m = box[0];
  const float ext = fmaxf(fmaxf(m.z - m.x, m.w - m.y), 1e-30f);
  const float sc = 65536.0f / ext;
  const float2 p = xy[i];
  const uint32_t qx = (uint32_t)fminf(fmaxf((p.x - m.x) * sc, 0.0f), 65535.0f);
  const uint32_t qy = (uint32_t)fminf(fmaxf((p.y - m.y) * sc, 0.0f), 65535.0f);
  keys[i] = (uint64_t)(bs_spread16(qx) | (bs_spread16(qy) << 1));
  ids[i] = i;
}

// perm[new] = old: inverse map, renumbered coordinates and degrees
__global__ void k_bs_relabel(int32_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ rp,
                             const float2* __restrict__ xy, int32_t* __restrict__ inv,
                             float2* __restrict__ xy2, int32_t* __restrict__ deg2) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t o = perm[i];
  inv[o] = i;
  xy2[i] = xy[o];
  deg2[i] = rp[o + 1] - rp[o];
}

__global__ void k_bs_fill(int32_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ inv,
                          const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const int64_t* __restrict__ rp2, int32_t* __restrict__ col2) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t o = perm[i];
  const int32_t e0 = rp[o], d = rp[o + 1] - e0;
  const int64_t f0 = rp2[i];
  for (int32_t j = 0; j < d; ++j) col2[f0 + j] = inv[col[e0 + j]];
}

// Neighbour ids per tile, lane-interleaved: entry k of the vertex in lane l
// of tile T at ell[base[T] + 64 k + l] for k < K[T] (the tile's largest
// degree), -1 past the vertex's degree and for lanes past n.
__global__ void k_bs_tile_deg(int32_t n, int32_t tiles, const int64_t* __restrict__ rp2,
                              int32_t* __restrict__ tk, int32_t* __restrict__ tcnt) {
  const int32_t T = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (T >= tiles) return;
  const int32_t v = 64 * T + lane_id();
  int32_t d = v < n ? (int32_t)(rp2[v + 1] - rp2[v]) : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) d = max(d, __shfl_xor(d, o, 64));
  if (lane_id() == 0) {
    tk[T] = d;
    tcnt[T] = 64 * d;
  }
}

__global__ void k_bs_ell_fill(int32_t n, int32_t tiles, const int64_t* __restrict__ rp2,
                              const int32_t* __restrict__ col2, const int32_t* __restrict__ tk,
                              const int64_t* __restrict__ tbase, int32_t* __restrict__ ell) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 64 * (int64_t)tiles) return;
  const int32_t T = (int32_t)(i >> 6), l = (int32_t)(i & 63);
  const int32_t v = (int32_t)i;
  const int32_t K = tk[T];
  const int64_t e0 = v < n ? rp2[v] : 0;
  const int32_t d = v < n ? (int32_t)(rp2[v + 1] - e0) : 0;
  int32_t* out = ell + tbase[T] + l;
  for (int32_t k = 0; k < K; ++k) out[64 * (int64_t)k] = k < d ? col2[e0 + k] : -1;
}

// One work-group per batch slot; state holds 3 n masks per slot (visited,
// frontier of even levels, frontier of odd levels); part[4 b + 0..3] gets the
// batch's sums of D/d, (D/d)^2, (D-d)^2/d^2 and its pair count.
__global__ __launch_bounds__(BS_T, 8) void k_bs_search(int32_t n, int32_t tiles, int32_t words,
                                                   const int32_t* __restrict__ tk,
                                                   const int64_t* __restrict__ tbase,
                                                   const int32_t* __restrict__ ell,
                                                   const float2* __restrict__ xy,
                                                   uint64_t* __restrict__ state,
                                                   double* __restrict__ part) {
  extern __shared__ uint64_t bs_bm[];  // 2 x words: tiles to visit at this level / the next
  __shared__ float2 sx[64];
  __shared__ int32_t s_any[2];
  __shared__ double sred[4][BS_WAVES];
  __shared__ double sacc[4][BS_T];  // each lane's pair sums over the batch
  const int l = lane_id(), w = threadIdx.x >> 6;
  uint64_t* vis = state + (size_t)blockIdx.x * 3 * (size_t)n;
  uint64_t* const fb0 = vis + n;             // frontier masks of even levels
  uint64_t* const fb1 = vis + 2 * (size_t)n;  // of odd levels
  const uint64_t resid = 0x0001000100010001ull << w;  // tiles T with T % 16 == w
  for (int32_t b = blockIdx.x; b < tiles; b += gridDim.x) {
    for (size_t i = threadIdx.x; i < 3 * (size_t)n; i += BS_T) vis[i] = 0ull;
    for (int32_t i = threadIdx.x; i < 2 * words; i += BS_T) bs_bm[i] = 0ull;
    const int32_t s0 = 64 * b;
    const int ns = min(64, n - s0);
    const uint64_t full = ns == 64 ? ~0ull : (1ull << ns) - 1ull;
    if (threadIdx.x < 64) sx[threadIdx.x] = threadIdx.x < ns ? xy[s0 + threadIdx.x] : make_float2(0.f, 0.f);
    if (threadIdx.x < 2) s_any[threadIdx.x] = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) sacc[k][threadIdx.x] = 0.0;
    __syncthreads();
    // level 0: the sources; level 1 visits the tiles of their neighbours
    if (threadIdx.x < ns) {
      const int32_t v = s0 + threadIdx.x;
      const uint64_t bit = 1ull << threadIdx.x;
      vis[v] = bit;
      fb0[v] = bit;
      const int32_t* ce = ell + tbase[b] + threadIdx.x;
      for (int32_t k = 0; k < tk[b]; ++k) {
        const int32_t u = ce[64 * k];
        if (u >= 0) atomicOr(&bs_bm[u >> 12], 1ull << ((u >> 6) & 63));
      }
    }
    __syncthreads();
    uint64_t* cur = bs_bm;
    uint64_t* nxt = bs_bm + words;
    for (int32_t h = 1;; ++h) {
      const uint64_t* R = (h & 1) ? fb0 : fb1;  // masks of level h - 1
      uint64_t* Wm = (h & 1) ? fb1 : fb0;
      const double inv_h = 1.0 / (double)h;
      for (int32_t i0 = 0; i0 < words; i0 += 64) {
        const uint64_t m = (i0 + l < words) ? (cur[i0 + l] & resid) : 0ull;
        uint64_t lanes = __ballot(m != 0ull);
        while (lanes) {
          const int src = __ffsll((unsigned long long)lanes) - 1;
          lanes &= lanes - 1;
          uint64_t mm = __shfl(m, src, 64);
          while (mm) {
            const int j = __ffsll((unsigned long long)mm) - 1;
            mm &= mm - 1;
            const int32_t T = 64 * (i0 + src) + j;
            const int32_t v = 64 * T + l;
            const int32_t K = tk[T];  // uniform over the wave
            const int32_t* ce = ell + tbase[T] + l;
            if (v < n) {
              // the first BS_U neighbours' loads are all issued before any is
              // used (one memory round trip instead of one per edge)
              int32_t cu[BS_U];
#pragma unroll
              for (int k = 0; k < BS_U; ++k) cu[k] = k < K ? ce[64 * k] : -1;
              const uint64_t vv = vis[v];
              uint64_t a = 0ull;
              if (vv != full) {  // a vertex every source has reached gains nothing
#pragma unroll
                for (int k = 0; k < BS_U; ++k) a |= cu[k] >= 0 ? R[cu[k]] : 0ull;
                for (int32_t k = BS_U; k < K; ++k) {
                  const int32_t u = ce[64 * k];
                  if (u >= 0) a |= R[u];
                }
              }
              const uint64_t nw = a & ~vv;
              Wm[v] = nw;
              if (nw) {
                vis[v] = vv | nw;
                s_any[h & 1] = 1;
#pragma unroll
                for (int k = 0; k < BS_U; ++k) {
                  if (cu[k] >= 0) {
                    const uint64_t tb = 1ull << ((cu[k] >> 6) & 63);
                    if (!(nxt[cu[k] >> 12] & tb)) atomicOr(&nxt[cu[k] >> 12], tb);
                  }
                }
                for (int32_t k = BS_U; k < K; ++k) {
                  const int32_t u = ce[64 * k];
                  if (u < 0) continue;
                  const uint64_t tb = 1ull << ((u >> 6) & 63);
                  if (!(nxt[u >> 12] & tb)) atomicOr(&nxt[u >> 12], tb);
                }
                // pairs (s, v) with s < v: sources of tile b below lane l
                uint64_t pm = T > b ? nw : (T == b ? (nw & ((1ull << l) - 1ull)) : 0ull);
                if (pm) {
                  const float2 xv = xy[v];
                  double a1 = 0.0, a2 = 0.0, a0 = 0.0, np = 0.0;
                  while (pm) {
                    const int i = __ffsll((unsigned long long)pm) - 1;
                    pm &= pm - 1;
                    const float2 xs = sx[i];
                    const double dx = (double)xs.x - (double)xv.x, dy = (double)xs.y - (double)xv.y;
                    const double t = sqrt(dx * dx + dy * dy) * inv_h;
                    const double tm = t - 1.0;
                    a1 += t;
                    a2 += t * t;
                    a0 += tm * tm;
                    np += 1.0;
                  }
                  sacc[0][threadIdx.x] += a1;
                  sacc[1][threadIdx.x] += a2;
                  sacc[2][threadIdx.x] += a0;
                  sacc[3][threadIdx.x] += np;
                }
              }
            }
          }
        }
      }
      __syncthreads();
      const int any = s_any[h & 1];
      if (threadIdx.x == 0) s_any[(h + 1) & 1] = 0;
      for (int32_t i = threadIdx.x; i < words; i += BS_T) cur[i] = 0ull;
      uint64_t* t = cur;
      cur = nxt;
      nxt = t;
      __syncthreads();
      if (!any) break;
    }
    const double a1 = wave_sum(sacc[0][threadIdx.x]);
    const double a2 = wave_sum(sacc[1][threadIdx.x]);
    const double a0 = wave_sum(sacc[2][threadIdx.x]);
    const double np = wave_sum(sacc[3][threadIdx.x]);
    if (l == 0) { sred[0][w] = a1; sred[1][w] = a2; sred[2][w] = a0; sred[3][w] = np; }
    __syncthreads();
    if (threadIdx.x < 4) {
      double acc = 0.0;
      for (int k = 0; k < BS_WAVES; ++k) acc += sred[threadIdx.x][k];
      part[4 * (size_t)b + threadIdx.x] = acc;
    }
    __syncthreads();
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

// Banded multi-source search (see the kernels above).  *done = false when the
// tile bitmap does not fit (n > 2^23) or the padded per-tile neighbour lists
// would take more than a quarter of the free device memory.
hipError_t full_stress_banded(const GraphDev& g, const float* xy, double* out_host, bool* done,
                              hipStream_t s) {
  const int32_t n = g.n;
  *done = false;
  const int32_t tiles = (n + 63) / 64;
  const int32_t words = (tiles + 63) / 64;
  if (words > BS_MAX_WORDS) return hipSuccess;
  // renumber in Morton order of the layout
  const int32_t nbb = std::min<int32_t>(1024, (n + 255) / 256);
  DevBuf bbp, keys, perm, inv, xy2, deg2, rp2, col2;
  MM_TRY(bbp.alloc(sizeof(float4) * (size_t)nbb, s));
  MM_TRY(keys.alloc(sizeof(uint64_t) * (size_t)n, s));
  MM_TRY(perm.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(inv.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(xy2.alloc(sizeof(float2) * (size_t)n, s));
  MM_TRY(deg2.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(rp2.alloc(sizeof(int64_t) * ((size_t)n + 1), s));
  MM_TRY(col2.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(g.nnz, 1), s));
  const unsigned nb = (unsigned)((n + 255) / 256);
  k_bs_bbox_part<<<nbb, 256, 0, s>>>(n, (const float2*)xy, bbp.as<float4>());
  k_bs_bbox_final<<<1, 64, 0, s>>>(nbb, bbp.as<float4>());
  k_bs_keys<<<nb, 256, 0, s>>>(n, (const float2*)xy, bbp.as<float4>(), keys.as<uint64_t>(),
                               perm.as<int32_t>());
  MM_TRY(hipGetLastError());
  MM_TRY(radix_sort_pairs(keys.as<uint64_t>(), perm.as<int32_t>(), n, 32, s));
  k_bs_relabel<<<nb, 256, 0, s>>>(n, perm.as<int32_t>(), g.row_ptr, (const float2*)xy,
                                  inv.as<int32_t>(), xy2.as<float2>(), deg2.as<int32_t>());
  MM_TRY(hipGetLastError());
  MM_TRY(scan_excl_i32(deg2.as<int32_t>(), rp2.as<int64_t>(), n, s));
  k_bs_fill<<<nb, 256, 0, s>>>(n, perm.as<int32_t>(), inv.as<int32_t>(), g.row_ptr, g.col,
                               rp2.as<int64_t>(), col2.as<int32_t>());
  MM_TRY(hipGetLastError());
  keys.release();
  DevBuf tk, tcnt, tbase, ell;
  MM_TRY(tk.alloc(sizeof(int32_t) * (size_t)tiles, s));
  MM_TRY(tcnt.alloc(sizeof(int32_t) * (size_t)tiles, s));
  MM_TRY(tbase.alloc(sizeof(int64_t) * ((size_t)tiles + 1), s));
  k_bs_tile_deg<<<(unsigned)((tiles + 3) / 4), 256, 0, s>>>(n, tiles, rp2.as<int64_t>(),
                                                            tk.as<int32_t>(), tcnt.as<int32_t>());
  MM_TRY(hipGetLastError());
  MM_TRY(scan_excl_i32(tcnt.as<int32_t>(), tbase.as<int64_t>(), tiles, s));
  int64_t ell_n = 0;
  MM_TRY(hipMemcpyAsync(&ell_n, tbase.as<int64_t>() + tiles, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  {
    // tiles holding a hub pad every lane to the hub's degree: give up when
    // that does not fit comfortably
    size_t fb = 0, tb = 0;
    MM_TRY(hipMemGetInfo(&fb, &tb));
    if (sizeof(int32_t) * (size_t)ell_n > fb / 4) return hipSuccess;  // *done stays false
  }
  MM_TRY(ell.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(ell_n, 1), s));
  k_bs_ell_fill<<<(unsigned)(((int64_t)tiles * 64 + 255) / 256), 256, 0, s>>>(
      n, tiles, rp2.as<int64_t>(), col2.as<int32_t>(), tk.as<int32_t>(), tbase.as<int64_t>(),
      ell.as<int32_t>());
  MM_TRY(hipGetLastError());
  MM_TRY(hipStreamSynchronize(s));
  col2.release();
  rp2.release();
  // batch slots: two work-groups per CU, within a third of the free memory
  int dev = 0, ncu = 0;
  MM_TRY(hipGetDevice(&dev));
  MM_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  size_t freeb = 0, totb = 0;
  MM_TRY(hipMemGetInfo(&freeb, &totb));
  const size_t per_slot = 3 * sizeof(uint64_t) * (size_t)n;
  const int64_t fit = (int64_t)(freeb / 3 / per_slot);
  const int32_t slots = (int32_t)std::max<int64_t>(1, std::min<int64_t>({2 * (int64_t)ncu, tiles, fit}));
  DevBuf state, part;
  MM_TRY(state.alloc(per_slot * (size_t)slots, s));
  MM_TRY(part.alloc(sizeof(double) * 4 * (size_t)tiles, s));
  const size_t shm = 2 * sizeof(uint64_t) * (size_t)words;
  k_bs_search<<<slots, BS_T, shm, s>>>(n, tiles, words, tk.as<int32_t>(), tbase.as<int64_t>(),
                                       ell.as<int32_t>(), xy2.as<float2>(), state.as<uint64_t>(),
                                       part.as<double>());
  MM_TRY(hipGetLastError());
  std::vector<double> h(4 * (size_t)tiles);
  MM_TRY(hipMemcpyAsync(h.data(), part.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  double s1 = 0, s2 = 0, s0 = 0, np = 0;
  for (int32_t b = 0; b < tiles; ++b) {
    s1 += h[4 * (size_t)b]; s2 += h[4 * (size_t)b + 1]; s0 += h[4 * (size_t)b + 2]; np += h[4 * (size_t)b + 3];
  }
  const double sstar = s2 > 0 ? s1 / s2 : 1.0;
  out_host[0] = s0;
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
  // high diameter (or asked for): the banded search
  if (method == 3 || (method == 0 && n > 65536)) {
    bool done = false;
    MM_TRY(full_stress_banded(g, xy, out_host, &done, s));
    if (done) return hipSuccess;
    if (method == 3) return hipErrorInvalidValue;
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
