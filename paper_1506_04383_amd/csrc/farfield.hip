// Far field of Eq. 2: F_u = sum_{v != u} r_q(u, v), r_q = (x_u - x_v)/|x_u - x_v|^(q+2).
//
// Exact mode: LDS-tiled all-pairs sum (one thread per target, sources staged
// through LDS in ascending order).
//
// Barnes-Hut mode (the quadtree approximation the paper cites for long-range
// forces):
//  1. bounding box -> square box with power-of-two side 2^e, origin (xmin, ymin);
//     cell index floor((x - xmin) * 2^(24-e)) in FP64, clamped to 24 bits;
//     48-bit Morton code (x bits even, y bits odd);
//  2. stable radix sort of (code, id);
//  3. compressed quadtree from the sorted codes: every adjacent pair with
//     different codes splits at depth floor(lcp/2); the leftmost such pair of
//     a cell owns the internal node; runs of equal codes are leaves.  Nodes
//     are sorted into pre-order by (first point, depth); each node stores a
//     skip index (next node after its subtree), so traversal is stackless;
//  4. moments: mass = point count, centre of mass from FP64 prefix sums of the
//     sorted coordinates (exact to FP64 rounding, independent of tree shape);
//  5. traversal: one wavefront walks the pre-order array for 64 targets that
//     are consecutive in Morton order.  Each lane keeps its own next-node
//     index; the wave visits the smallest one, so every node record is a
//     wave-uniform load.  Lanes that accept a cell or finish a leaf jump to its
//     skip index, which masks them for the whole subtree: each lane sees
//     exactly the nodes its own depth-first traversal would, in the same
//     order.  The opening test is exact integer geometry evaluated in FP64:
//     accept cell C (not containing u) iff
//       theta^2 * |(2 iu + 1) - (2 o_C + S_C)|^2 > 4 S_C^2.
#include <algorithm>

#include "bh.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace mm {

BHWork* bh_work_create() { return new BHWork(); }
void bh_work_destroy(BHWork* w) { delete w; }

namespace {

constexpr int BB_T = 256;

__global__ __launch_bounds__(BB_T) void k_bbox_partial(const float2* __restrict__ xy, int32_t n,
                                                       float4* __restrict__ part) {
  raise_wave_priority();
  float xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
  for (int32_t i = blockIdx.x * BB_T + threadIdx.x; i < n; i += gridDim.x * BB_T) {
    float2 p = xy[i];
    xmin = fminf(xmin, p.x); xmax = fmaxf(xmax, p.x);
    ymin = fminf(ymin, p.y); ymax = fmaxf(ymax, p.y);
  }
  for (int o = 32; o > 0; o >>= 1) {
    xmin = fminf(xmin, __shfl_xor(xmin, o, 64)); xmax = fmaxf(xmax, __shfl_xor(xmax, o, 64));
    ymin = fminf(ymin, __shfl_xor(ymin, o, 64)); ymax = fmaxf(ymax, __shfl_xor(ymax, o, 64));
  }
  __shared__ float4 sh[BB_T / 64];
  if (lane_id() == 0) sh[threadIdx.x >> 6] = make_float4(xmin, ymin, xmax, ymax);
  __syncthreads();
  if (threadIdx.x == 0) {
    float4 r = sh[0];
    for (int i = 1; i < BB_T / 64; ++i) {
      r.x = fminf(r.x, sh[i].x); r.y = fminf(r.y, sh[i].y);
      r.z = fmaxf(r.z, sh[i].z); r.w = fmaxf(r.w, sh[i].w);
    }
    part[blockIdx.x] = r;
  }
}

__device__ void make_box(float4 r, BoxInfo* box);

// One wave reduces the block partials (min / max are exact in any order).
__global__ void k_bbox_final(const float4* __restrict__ part, int nb, BoxInfo* box) {
  raise_wave_priority();
  float4 r = part[0];
  for (int i = threadIdx.x; i < nb; i += 64) {
    const float4 p = part[i];
    r.x = fminf(r.x, p.x); r.y = fminf(r.y, p.y);
    r.z = fmaxf(r.z, p.z); r.w = fmaxf(r.w, p.w);
  }
  for (int o = 32; o > 0; o >>= 1) {
    r.x = fminf(r.x, __shfl_xor(r.x, o, 64)); r.y = fminf(r.y, __shfl_xor(r.y, o, 64));
    r.z = fmaxf(r.z, __shfl_xor(r.z, o, 64)); r.w = fmaxf(r.w, __shfl_xor(r.w, o, 64));
  }
  if (threadIdx.x == 0) make_box(r, box);
}

// One box per graph of a batch (block per graph).
__global__ __launch_bounds__(BB_T) void k_bbox_seg(const float2* __restrict__ xy,
                                                   const int32_t* __restrict__ goff,
                                                   BoxInfo* __restrict__ box) {
  raise_wave_priority();
  const int32_t a = goff[blockIdx.x], b = goff[blockIdx.x + 1];
  float xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
  for (int32_t i = a + threadIdx.x; i < b; i += BB_T) {
    float2 p = xy[i];
    xmin = fminf(xmin, p.x); xmax = fmaxf(xmax, p.x);
    ymin = fminf(ymin, p.y); ymax = fmaxf(ymax, p.y);
  }
  for (int o = 32; o > 0; o >>= 1) {
    xmin = fminf(xmin, __shfl_xor(xmin, o, 64)); xmax = fmaxf(xmax, __shfl_xor(xmax, o, 64));
    ymin = fminf(ymin, __shfl_xor(ymin, o, 64)); ymax = fmaxf(ymax, __shfl_xor(ymax, o, 64));
  }
  __shared__ float4 sh[BB_T / 64];
  if (lane_id() == 0) sh[threadIdx.x >> 6] = make_float4(xmin, ymin, xmax, ymax);
  __syncthreads();
  if (threadIdx.x == 0) {
    float4 r = sh[0];
    for (int i = 1; i < BB_T / 64; ++i) {
      r.x = fminf(r.x, sh[i].x); r.y = fminf(r.y, sh[i].y);
      r.z = fmaxf(r.z, sh[i].z); r.w = fmaxf(r.w, sh[i].w);
    }
    make_box(r, box + blockIdx.x);
  }
}

// Square box with power-of-two side over the extent r = (xmin, ymin, xmax, ymax).
__device__ void make_box(float4 r, BoxInfo* box) {
  double xmin = r.x, ymin = r.y;
  double ext = fmax((double)r.z - xmin, (double)r.w - ymin);
  int e = 0;
  if (ext > 0.0) {
    int ex;
    double m = frexp(ext, &ex);
    e = (m == 0.5) ? ex - 1 : ex;
  }
  box->xmin = xmin;
  box->ymin = ymin;
  box->scale = ldexp(1.0, 24 - e);
  box->e = e;
}

__device__ inline uint64_t spread24(uint32_t v) {
  uint64_t x = v & 0xFFFFFFull;
  x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
  x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
  x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}
__device__ inline uint32_t compact24(uint64_t x) {
  x &= 0x5555555555555555ull;
  x = (x | (x >> 1)) & 0x3333333333333333ull;
  x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
  x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
  x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
  return (uint32_t)x & 0xFFFFFFu;
}

// gid (may be null): graph of each point in a batch; its index goes above
// the 48 code bits and its own box is used.
__global__ void k_morton(const float2* __restrict__ xy, int32_t n, const BoxInfo* __restrict__ box,
                         const int32_t* __restrict__ gid, uint64_t* __restrict__ codes,
                         int32_t* __restrict__ ids, uint32_t* __restrict__ nmask) {
  raise_wave_priority();
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (nmask) nmask[i] = 0;  // node-start masks of k_emit_nodes
  const int32_t g = gid ? gid[i] : 0;
  const BoxInfo b = box[g];
  float2 p = xy[i];
  double fx = floor(((double)p.x - b.xmin) * b.scale);
  double fy = floor(((double)p.y - b.ymin) * b.scale);
  fx = fmin(fmax(fx, 0.0), 16777215.0);
  fy = fmin(fmax(fy, 0.0), 16777215.0);
  codes[i] = spread24((uint32_t)fx) | (spread24((uint32_t)fy) << 1) | ((uint64_t)g << 48);
  ids[i] = i;
}

// Inclusive-exclusive FP64 prefix sums of the sorted coordinates (fixed
// tiles of PS_TILE points, both axes): tile sums, a scan of the tile sums,
// then each tile's own scan.
constexpr int PS_T = 256, PS_I = 8, PS_TILE = PS_T * PS_I;

// Points in sorted order (coordinates and quantum cells) and the FP64 sums
// of both coordinates per tile (part[t], part[stride + t]); each thread takes
// PS_I consecutive points and adds them in order.
__global__ __launch_bounds__(PS_T) void k_gather_tiles(const float2* __restrict__ xy,
                                                       const int32_t* __restrict__ order,
                                                       const uint64_t* __restrict__ codes,
                                                       int32_t n, float* __restrict__ xsx,
                                                       float* __restrict__ xsy,
                                                       uint2* __restrict__ ixy,
                                                       double* __restrict__ part, int32_t stride,
                                                       int32_t* __restrict__ counter) {
  raise_wave_priority();
  __shared__ double sh[PS_T / 64 + 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;  // node count of k_emit_nodes
  const int64_t base = (int64_t)blockIdx.x * PS_TILE + threadIdx.x * PS_I;
  double sx = 0.0, sy = 0.0;
  for (int i = 0; i < PS_I; ++i) {
    const int64_t j = base + i;
    if (j < n) {
      const float2 p = xy[order[j]];
      xsx[j] = p.x;
      xsy[j] = p.y;
      const uint64_t c = codes[j];
      ixy[j] = make_uint2(compact24(c), compact24(c >> 1));
      sx += (double)p.x;
      sy += (double)p.y;
    }
  }
  double tx, ty;
  block_excl_scan<double>(sx, sh, &tx);
  block_excl_scan<double>(sy, sh, &ty);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = tx;
    part[stride + blockIdx.x] = ty;
  }
}
// exclusive scan of one axis's m tile sums in place (block b: axis b, at
// part + b * (m + 1)), the total in part[m]
__global__ __launch_bounds__(1024) void k_fsum_parts(double* parts, int32_t m) {
  raise_wave_priority();
  __shared__ double sh[1024 / 64 + 1];
  double* part = parts + (int64_t)blockIdx.x * (m + 1);
  double carry = 0.0;
  for (int32_t b = 0; b < m; b += blockDim.x) {
    int32_t j = b + threadIdx.x;
    double v = j < m ? part[j] : 0.0;
    double tot;
    double ex = block_excl_scan<double>(v, sh, &tot);
    if (j < m) part[j] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[m] = carry;
}
// each tile's scan of one axis (m tiles)
__device__ inline void fsum_scan_tile(const float* __restrict__ a, int32_t n,
                                      const double* __restrict__ part, int32_t m,
                                      double* __restrict__ out, double* sh) {
  int64_t base = (int64_t)blockIdx.x * PS_TILE + threadIdx.x * PS_I;
  double v[PS_I], s = 0.0;
  for (int i = 0; i < PS_I; ++i) { v[i] = base + i < n ? (double)a[base + i] : 0.0; s += v[i]; }
  double tot;
  double ex = block_excl_scan<double>(s, sh, &tot) + part[blockIdx.x];
  for (int i = 0; i < PS_I; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
  if ((int32_t)blockIdx.x == m - 1 && threadIdx.x == 0) out[n] = part[m];
}

__device__ inline int lcp48(uint64_t a, uint64_t b) {
  uint64_t x = (a ^ b) << 16;  // codes live in the low 48 bits
  return x == 0 ? 48 : __clzll(x);
}

// Emit nodes: leaves at bucket starts, internal nodes at owner pairs.
// Node records at fixed slots: the leaf of the run of equal codes starting
// at i in slot 2i, the internal node owned by the pair (i, i+1) in slot
// 2i+1 (a slot without a node is marked empty).  Pre-order is the order of
// (first point, depth), a leaf after every internal node with the same first
// point; so each point a keeps a mask of the depths of the nodes that start
// at it (bit 31: its leaf), and a node's pre-order index is the number of
// nodes that start before a (a prefix sum over the masks' bit counts) plus
// the number of shallower nodes that start at a.  This gives exactly the
// order of a sort of the keys (first << 5 | depth code).  Range ends are
// found by galloping from i (steps 1, 2, 4, ... then a binary search inside
// the last step), so a node spanning m points costs O(log m) loads.  The node
// count is added once per wave.
//
// first index j in [lo, hi) at or after `from` whose key exceeds `key` under
// the prefix shift sh (codes are sorted; the answer is > from)
__device__ inline int32_t gallop_up(const uint64_t* __restrict__ codes, int32_t from, int32_t n,
                                    uint64_t key, int sh) {
  int32_t lo = from + 1, step = 1, hi = n;
  while (lo < n) {
    const int32_t probe = min(n - 1, from + step);
    if ((codes[probe] >> sh) > key) { hi = probe; break; }
    lo = probe + 1;
    step <<= 1;
  }
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if ((codes[mid] >> sh) <= key) lo = mid + 1; else hi = mid;
  }
  return lo;
}
// first index j <= from with (codes[j] >> sh) == key (codes[from] >> sh == key)
__device__ inline int32_t gallop_down(const uint64_t* __restrict__ codes, int32_t from,
                                      uint64_t key, int sh) {
  int32_t hi = from, step = 1, lo = 0;
  while (hi > 0) {
    const int32_t probe = max(0, from - step);
    if ((codes[probe] >> sh) < key) { lo = probe + 1; break; }
    hi = probe;
    step <<= 1;
  }
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if ((codes[mid] >> sh) < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void k_emit_nodes(const uint64_t* __restrict__ codes, int32_t n,
                             int4* __restrict__ tmp, uint32_t* __restrict__ nmask,
                             int32_t* __restrict__ counter) {
  raise_wave_priority();
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t made = 0;
  if (i < n) {
    const uint64_t ci = codes[i];
    int4 leafrec = make_int4(0, 0, 0, -1), intrec = make_int4(0, 0, 0, -1);
    if (i == 0 || codes[i - 1] != ci) {
      // leaf: run of equal codes starting at i
      const int32_t end = gallop_up(codes, i, n, ci, 0);
      leafrec = make_int4(i, end - 1, 24, 1);
      atomicOr(&nmask[i], 1u << 31);
      ++made;
    }
    if (i + 1 < n && codes[i + 1] != ci && (codes[i + 1] >> 48) == (ci >> 48)) {
      const int t = lcp48(ci, codes[i + 1]) >> 1;
      const int sh = 48 - 2 * t;
      const uint64_t pre = ci >> sh;
      // a: first index with the same 2t-bit prefix
      const int32_t a = gallop_down(codes, i, pre, sh);
      // owner iff points a..i lie in the same child (no split of depth t left of i)
      if ((codes[a] >> (sh - 2)) == (ci >> (sh - 2))) {
        const int32_t end = gallop_up(codes, i, n, pre, sh);
        intrec = make_int4(a, end - 1, t, 0);
        atomicOr(&nmask[a], 1u << t);
        ++made;
      }
    }
    tmp[2 * i] = leafrec;
    tmp[2 * i + 1] = intrec;
  }
  made = wave_sum(made);
  if (lane_id() == 0 && made) atomicAdd(counter, made);
}

// Node-start counts per tile of PS_TILE points (bit counts of the masks).
__global__ __launch_bounds__(PS_T) void k_node_tiles(const uint32_t* __restrict__ nmask, int32_t n,
                                                     int32_t* __restrict__ part) {
  raise_wave_priority();
  __shared__ int32_t sh[PS_T / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * PS_TILE + threadIdx.x * PS_I;
  int32_t c = 0;
  for (int i = 0; i < PS_I; ++i)
    if (base + i < n) c += __popc(nmask[base + i]);
  int32_t tot;
  block_excl_scan<int32_t>(c, sh, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}
// Exclusive scan of m tile counts in place (one work-group), total in part[m].
__global__ __launch_bounds__(1024) void k_node_parts(int32_t* part, int32_t m) {
  raise_wave_priority();
  __shared__ int32_t sh[1024 / 64 + 1];
  int32_t carry = 0;
  for (int32_t b = 0; b < m; b += blockDim.x) {
    const int32_t j = b + threadIdx.x;
    const int32_t v = j < m ? part[j] : 0;
    int32_t tot;
    const int32_t ex = block_excl_scan<int32_t>(v, sh, &tot);
    if (j < m) part[j] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[m] = carry;
}
// first_at[a] = pre-order index of the first node that starts at point a
// (the nodes starting before a); first_at[n] = the node count.  FUSED: each
// tile adds the counts of the tiles before it itself (m <= NODE_FUSE_MAX),
// else part holds their exclusive scan.  Shares its grid with the two FP64
// coordinate scans (blockIdx.y 0, 1: k_fsum_scan's work; 2: this one).
constexpr int32_t NODE_FUSE_MAX = 512;
template <bool FUSED>
__device__ inline void node_base(const uint32_t* __restrict__ nmask, int32_t n,
                                 const int32_t* __restrict__ part, int32_t m,
                                 int32_t* __restrict__ first_at, int32_t* sh) {
  int32_t carry;
  if (FUSED) {
    int32_t c = 0;
    for (int32_t j = threadIdx.x; j < (int32_t)blockIdx.x; j += PS_T) c += part[j];
    block_excl_scan<int32_t>(c, sh, &carry);
  } else {
    carry = part[blockIdx.x];
  }
  const int64_t base = (int64_t)blockIdx.x * PS_TILE + threadIdx.x * PS_I;
  int32_t v[PS_I], c = 0;
  for (int i = 0; i < PS_I; ++i) {
    v[i] = base + i < n ? __popc(nmask[base + i]) : 0;
    c += v[i];
  }
  int32_t tot;
  int32_t ex = block_excl_scan<int32_t>(c, sh, &tot) + carry;
  for (int i = 0; i < PS_I; ++i) {
    if (base + i < n) first_at[base + i] = ex;
    ex += v[i];
  }
  if ((int32_t)blockIdx.x == m - 1 && threadIdx.x == 0) first_at[n] = carry + tot;
}

// The last three scans of the build in one grid (m tiles x 3): rows 0 and 1
// the FP64 prefix sums of x and y, row 2 the node bases.
template <bool FUSED>
__global__ __launch_bounds__(PS_T) void k_tile_scans(const float* __restrict__ ax,
                                                     const float* __restrict__ ay, int32_t n,
                                                     const double* __restrict__ parts,
                                                     double* __restrict__ ox,
                                                     double* __restrict__ oy,
                                                     const uint32_t* __restrict__ nmask,
                                                     const int32_t* __restrict__ npart,
                                                     int32_t* __restrict__ first_at) {
  raise_wave_priority();
  __shared__ double sh[PS_T / 64 + 1];
  const int32_t m = gridDim.x;
  if (blockIdx.y < 2) {
    fsum_scan_tile(blockIdx.y ? ay : ax, n, parts + (int64_t)blockIdx.y * (m + 1), m,
                   blockIdx.y ? oy : ox, sh);
  } else {
    node_base<FUSED>(nmask, n, npart, m, first_at, reinterpret_cast<int32_t*>(sh));
  }
}

// Node records in pre-order, one thread per slot of k_emit_nodes.
__global__ void k_finalize_nodes(const int4* __restrict__ tmp, const uint32_t* __restrict__ nmask,
                                 int32_t n, const int32_t* __restrict__ first_at,
                                 const double* __restrict__ px, const double* __restrict__ py,
                                 const float* __restrict__ xsx, const float* __restrict__ xsy,
                                 const uint2* __restrict__ ixy, BHNode* __restrict__ nodes,
                                 int64_t* __restrict__ export_nodes,
                                 const uint64_t* __restrict__ codes) {
  raise_wave_priority();
  const int32_t sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= 2 * n) return;
  const int4 t = tmp[sl];
  if (t.w < 0) return;  // no node in this slot
  const int32_t first = t.x, last = t.y, depth = t.z, leaf = t.w;
  const int32_t N = first_at[n];
  // pre-order index: nodes starting before `first`, then the shallower ones
  // starting at it (a leaf's depth code is 31)
  const uint32_t below = leaf ? 0x7fffffffu : (1u << depth) - 1u;
  const int32_t p = first_at[first] + __popc(nmask[first] & below);
  const int32_t cnt = last - first + 1;
  BHNode nd;
  // a single point keeps its own coordinates exactly (the traversal reads
  // them from here instead of the point arrays)
  nd.cx = cnt == 1 ? (double)xsx[first] : (px[last + 1] - px[first]) / (double)cnt;
  nd.cy = cnt == 1 ? (double)xsy[first] : (py[last + 1] - py[first]) / (double)cnt;
  nd.mass = (float)cnt;
  nd.skip = (last + 1 < n) ? first_at[last + 1] : N;
  const uint32_t mask = depth >= 24 ? 0xFFFFFFu : ~((1u << (24 - depth)) - 1u) & 0xFFFFFFu;
  uint2 q = ixy[first];
  nd.ox = q.x & mask;
  nd.oy = q.y & mask;
  nd.meta = depth | ((leaf ? min(cnt, kLeafCountSat) : 0) << 8);
  nd.first = first;
  nodes[p] = nd;
  if (export_nodes) {
    int64_t* o = export_nodes + 5 * (int64_t)p;
    o[0] = depth; o[1] = first; o[2] = cnt; o[3] = leaf;
    o[4] = (int64_t)(codes[first] >> (2 * (24 - depth)));
  }
}

// ---- small trees: the whole build in one work-group (n <= BHS_MAX)
// Same tree as the multi-kernel build: (code, id) sorted by one bitonic sort
// of code << 12 | id in LDS, the same leaves and owner pairs, node keys
// (first << 5 | depth code) sorted by a second bitonic sort, then the same
// pre-order records.  Only the FP64 prefix sums run in a different order.
constexpr int BHS_T = 1024;
constexpr int BHS_MAX = 4096;

__device__ inline void bitonic_sort_lds(uint64_t* a, int m) {  // m: power of two
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < m; i += BHS_T) {
        const int l = i ^ j;
        if (l > i) {
          const uint64_t x = a[i], y = a[l];
          const bool asc = (i & k) == 0;
          if ((x > y) == asc) { a[i] = y; a[l] = x; }
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(BHS_T) void k_bh_small(
    const float2* __restrict__ xy, int32_t n, BoxInfo* __restrict__ boxo,
    uint64_t* __restrict__ codes, int32_t* __restrict__ order, float* __restrict__ xsx,
    float* __restrict__ xsy, uint2* __restrict__ ixy, double* __restrict__ px,
    double* __restrict__ py, BHNode* __restrict__ nodes, int32_t* __restrict__ Np,
    int64_t* __restrict__ export_nodes) {
  raise_wave_priority();
  // static LDS (112 KB for BHS_MAX = 4096; gfx950 work-groups may hold 160 KB)
  __shared__ uint64_t sk[BHS_MAX];      // code << 12 | id, then codes
  __shared__ uint64_t nk[2 * BHS_MAX];  // node keys
  __shared__ int32_t fat[BHS_MAX];      // first node of each first point
  int m = 1;
  while (m < n) m <<= 1;
  __shared__ float4 red[BHS_T / 64];
  __shared__ BoxInfo sbox;
  __shared__ int32_t ncount;
  __shared__ double dsh[BHS_T / 64 + 1];
  const int tid = threadIdx.x;
  // 1. box
  float xmin = INFINITY, ymin = INFINITY, xmax = -INFINITY, ymax = -INFINITY;
  for (int i = tid; i < n; i += BHS_T) {
    const float2 p = xy[i];
    xmin = fminf(xmin, p.x); xmax = fmaxf(xmax, p.x);
    ymin = fminf(ymin, p.y); ymax = fmaxf(ymax, p.y);
  }
  for (int o = 32; o > 0; o >>= 1) {
    xmin = fminf(xmin, __shfl_xor(xmin, o, 64)); xmax = fmaxf(xmax, __shfl_xor(xmax, o, 64));
    ymin = fminf(ymin, __shfl_xor(ymin, o, 64)); ymax = fmaxf(ymax, __shfl_xor(ymax, o, 64));
  }
  if (lane_id() == 0) red[tid >> 6] = make_float4(xmin, ymin, xmax, ymax);
  if (tid == 0) ncount = 0;
  __syncthreads();
  if (tid == 0) {
    float4 r = red[0];
    for (int i = 1; i < BHS_T / 64; ++i) {
      r.x = fminf(r.x, red[i].x); r.y = fminf(r.y, red[i].y);
      r.z = fmaxf(r.z, red[i].z); r.w = fmaxf(r.w, red[i].w);
    }
    make_box(r, &sbox);
    *boxo = sbox;
  }
  __syncthreads();
  // 2. codes, 3. sort (code, id)
  const BoxInfo b = sbox;
  for (int i = tid; i < m; i += BHS_T) {
    if (i < n) {
      const float2 p = xy[i];
      double fx = floor(((double)p.x - b.xmin) * b.scale);
      double fy = floor(((double)p.y - b.ymin) * b.scale);
      fx = fmin(fmax(fx, 0.0), 16777215.0);
      fy = fmin(fmax(fy, 0.0), 16777215.0);
      const uint64_t c = spread24((uint32_t)fx) | (spread24((uint32_t)fy) << 1);
      sk[i] = (c << 12) | (uint64_t)i;
    } else {
      sk[i] = ~0ull;
    }
  }
  __syncthreads();
  bitonic_sort_lds(sk, m);
  // 4. sorted points
  for (int i = tid; i < n; i += BHS_T) {
    const uint64_t kv = sk[i];
    const uint64_t c = kv >> 12;
    const int32_t id = (int32_t)(kv & 0xFFFu);
    const float2 p = xy[id];
    codes[i] = c;
    order[i] = id;
    xsx[i] = p.x;
    xsy[i] = p.y;
    ixy[i] = make_uint2(compact24(c), compact24(c >> 1));
  }
  __syncthreads();
  for (int i = tid; i < n; i += BHS_T) sk[i] = sk[i] >> 12;  // codes from here on
  // 5. FP64 prefix sums of the sorted coordinates (4 consecutive points per thread)
  {
    const int i0 = tid * 4;
    double vx[4], vy[4], tx = 0.0, ty = 0.0;
    for (int j = 0; j < 4; ++j) {
      const int i = i0 + j;
      vx[j] = vy[j] = 0.0;
      if (i < n) {
        const float2 p = xy[(int32_t)(order[i])];
        vx[j] = p.x;
        vy[j] = p.y;
      }
      tx += vx[j];
      ty += vy[j];
    }
    double totx, toty;
    double ex = block_excl_scan<double>(tx, dsh, &totx);
    double ey = block_excl_scan<double>(ty, dsh, &toty);
    for (int j = 0; j < 4; ++j) {
      const int i = i0 + j;
      if (i < n) { px[i] = ex; py[i] = ey; }
      ex += vx[j];
      ey += vy[j];
    }
    if (tid == 0) { px[n] = totx; py[n] = toty; }
  }
  __syncthreads();
  // 6. node keys: leaves at runs of equal codes, internal nodes at owner pairs
  for (int i = tid; i < 2 * m; i += BHS_T) nk[i] = ~0ull;
  __syncthreads();
  for (int i = tid; i < n; i += BHS_T) {
    const uint64_t ci = sk[i];
    if (i == 0 || sk[i - 1] != ci) nk[atomicAdd(&ncount, 1)] = ((uint64_t)i << 5) | 31u;
    if (i + 1 < n && sk[i + 1] != ci) {
      const int t = lcp48(ci, sk[i + 1]) >> 1;
      const int sh = 48 - 2 * t;
      const uint64_t pre = ci >> sh;
      int lo = 0, hi = i;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((sk[mid] >> sh) < pre) lo = mid + 1; else hi = mid;
      }
      if ((sk[lo] >> (sh - 2)) == (ci >> (sh - 2)))
        nk[atomicAdd(&ncount, 1)] = ((uint64_t)lo << 5) | (uint32_t)t;
    }
  }
  __syncthreads();
  const int32_t N = ncount;
  // 7. pre-order: sort by (first point, depth code)
  bitonic_sort_lds(nk, 2 * m);
  for (int p = tid; p < N; p += BHS_T) {
    const int32_t f = (int32_t)(nk[p] >> 5);
    if (p == 0 || (int32_t)(nk[p - 1] >> 5) != f) fat[f] = p;
  }
  __syncthreads();
  // 8. node records
  for (int p = tid; p < N; p += BHS_T) {
    const uint64_t key = nk[p];
    const int32_t first = (int32_t)(key >> 5);
    const int dcode = (int)(key & 31u);
    const bool leaf = dcode == 31;
    const int depth = leaf ? 24 : dcode;
    const uint64_t c0 = sk[first];
    int lo = first + 1, hi = n;  // last point: end of the equal code run / prefix
    if (leaf) {
      while (lo < hi) { const int mid = (lo + hi) >> 1; if (sk[mid] <= c0) lo = mid + 1; else hi = mid; }
    } else {
      const int sh = 48 - 2 * depth;
      const uint64_t pre = c0 >> sh;
      while (lo < hi) { const int mid = (lo + hi) >> 1; if ((sk[mid] >> sh) <= pre) lo = mid + 1; else hi = mid; }
    }
    const int32_t last = lo - 1;
    const int32_t cnt = last - first + 1;
    BHNode nd;
    nd.cx = cnt == 1 ? (double)xsx[first] : (px[last + 1] - px[first]) / (double)cnt;
    nd.cy = cnt == 1 ? (double)xsy[first] : (py[last + 1] - py[first]) / (double)cnt;
    nd.mass = (float)cnt;
    nd.skip = (last + 1 < n) ? fat[last + 1] : N;
    const uint32_t mask = depth >= 24 ? 0xFFFFFFu : ~((1u << (24 - depth)) - 1u) & 0xFFFFFFu;
    nd.ox = compact24(c0) & mask;
    nd.oy = compact24(c0 >> 1) & mask;
    nd.meta = depth | ((leaf ? min(cnt, kLeafCountSat) : 0) << 8);
    nd.first = first;
    nodes[p] = nd;
    if (export_nodes) {
      int64_t* o = export_nodes + 5 * (int64_t)p;
      o[0] = depth; o[1] = first; o[2] = cnt; o[3] = leaf ? 1 : 0;
      o[4] = (int64_t)(c0 >> (2 * (24 - depth)));
    }
  }
  if (tid == 0) *Np = N;
}

constexpr int TR_WAVES = 4;

// Interactions of one lane's target (xt, yt; quantum cell (qx2i, qy2i)
// doubled) with node nd at index p: leaf terms, or the opening test and the
// cell term.  Returns true when the lane opens the node.  CT: test whether
// the cell contains u.  Without it the decisions are the same for
// theta^2 <= 2: u in C means |d| <= S - 1 on both axes, so theta^2 d4 <=
// 4 (S - 1)^2 < 4 S^2 (rounding is monotone and 4 (S - 1)^2 is exact), and
// the cell fails the distance test anyway.
template <bool STATS, bool CT>
__device__ inline void visit_node(const BHNode& nd, bool act, int32_t i, float xt, float yt,
                                  int32_t qx2i, int32_t qy2i, float q, double theta2,
                                  const float* __restrict__ xsx, const float* __restrict__ xsy,
                                  int32_t skipv, int32_t& wait, float& fx, float& fy,
                                  unsigned long long& acc, unsigned long long& pairs) {
  // An accepted cell and a single-point leaf (whose record holds the
  // point's coordinates and mass 1) add the same term: rounding the FP64
  // difference of two floats to FP32 gives their FP32 difference
  // (53 >= 2 * 24 + 2).  The record is wave-uniform, so the node kind,
  // mass and cell centre are scalars and the kind is a scalar branch.
  const float m = __builtin_bit_cast(
      float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int32_t, nd.mass)));
  const int32_t lc = __builtin_amdgcn_readfirstlane(nd.meta >> 8);
  if (lc == 0) {
    // opening test in exact integers: offsets of u's quantum-cell centre
    // from the cell centre (doubled); |d| < S on both axes <=> u in C;
    // d4 < 2^52 and 4 S^2 are exact doubles, so theta^2 d4 > 4 S^2 rounds
    // exactly as the same test written with 64-bit integers.  4 S^2 =
    // 2^(2 sh + 2) is assembled from its exponent bits.
    const int sh = 24 - (nd.meta & 0xff);
    const int32_t S = 1 << sh;
    const int32_t cx2 = __builtin_amdgcn_readfirstlane((int32_t)(2u * nd.ox + (uint32_t)S));
    const int32_t cy2 = __builtin_amdgcn_readfirstlane((int32_t)(2u * nd.oy + (uint32_t)S));
    const double s4 = __hiloint2double((1023 + 2 * sh + 2) << 20, 0);
    if (act) {
      const int32_t dxi = qx2i - cx2;
      const int32_t dyi = qy2i - cy2;
      const bool contains = CT && abs(dxi) < S && abs(dyi) < S;
      const double dxd = (double)dxi, dyd = (double)dyi;
      const double d4 = fma(dxd, dxd, dyd * dyd);
      if (!contains && theta2 * d4 > s4) {
        // accepted: the lane does not descend
        wait = skipv;
        rq_add((float)((double)xt - nd.cx), (float)((double)yt - nd.cy), q, m, fx, fy);
        if (STATS) acc++;
      }
    }
  } else if (lc == 1) {
    if (act) {
      wait = skipv;
      if (nd.first != i) {
        const bool added =
            rq_add((float)((double)xt - nd.cx), (float)((double)yt - nd.cy), q, 1.f, fx, fy);
        if (STATS && added) pairs++;
      }
    }
  } else if (act) {
    // leaf of several points: exact terms from the point arrays
    wait = skipv;
    const int32_t cnt = lc == kLeafCountSat ? (int32_t)m : lc;
    for (int32_t j = nd.first; j < nd.first + cnt; ++j) {
      const float sx = xsx[j], sy = xsy[j];
      if (j != i) {
        const bool added = rq_add(xt - sx, yt - sy, q, 1.f, fx, fy);
        if (STATS && added) pairs++;
      }
    }
  }
}

// One wavefront walks the pre-order node array once for 64 Morton-consecutive
// targets; a lane takes part at node p when its own walk is at p.
// One tree (no batch): the wave's next node is p + 1 when some lane opens p,
// else skip(p) -- a lane that is not at p waits at a node after p's subtree
// (its walk never entered that subtree), i.e. at or after skip(p).  So a lane
// keeps only the node it waits for, `wait`, set when it does not open: a lane
// that opens p is at p + 1, the wave's next node, and the lanes at the
// wave's node p are exactly those with wait <= p.  Both candidate records
// are loaded as soon as p's record is there, so their latency overlaps p's
// work.  Batches (one tree per graph, per-lane root and end) take the
// minimum of the lanes' next nodes instead.
template <bool STATS, bool SEG, bool CT>
__global__ __launch_bounds__(64 * TR_WAVES) void k_traverse(
    const BHNode* __restrict__ nodes, const int32_t* __restrict__ Np, const float* __restrict__ xsx,
    const float* __restrict__ xsy, const uint2* __restrict__ ixy, const int32_t* __restrict__ order,
    int32_t n, float q, double theta2, float2* __restrict__ F, unsigned long long* __restrict__ stats,
    const uint64_t* __restrict__ scodes, const int32_t* __restrict__ goff,
    const int32_t* __restrict__ first_at) {
  raise_wave_priority();
  const int l = lane_id();
  const int32_t i = (blockIdx.x * TR_WAVES + (threadIdx.x >> 6)) * 64 + l;
  if ((blockIdx.x * TR_WAVES + (threadIdx.x >> 6)) * 64 >= n) return;
  const int32_t N = *Np;
  const bool valid = i < n;
  const float xt = valid ? xsx[i] : 0.f, yt = valid ? xsy[i] : 0.f;
  const uint2 qt = valid ? ixy[i] : make_uint2(0, 0);
  const int32_t qx2i = 2 * (int32_t)qt.x + 1, qy2i = 2 * (int32_t)qt.y + 1;
  float fx = 0.f, fy = 0.f;
  unsigned long long acc = 0, pairs = 0;
  if (!SEG) {
    int32_t wait = valid ? 0 : 0x7fffffff;
    int32_t p = 0;
    BHNode nd = nodes[0];
    while (p < N) {
      const BHNode na = nodes[min(p + 1, N - 1)];
      const BHNode nb = nodes[min(nd.skip, N - 1)];
      visit_node<STATS, CT>(nd, wait <= p, i, xt, yt, qx2i, qy2i, q, theta2, xsx, xsy,
                            nd.skip >= N ? 0x7fffffff : nd.skip, wait, fx, fy, acc, pairs);
      // the lanes that opened p are the ones still at or before it
      const bool down = __builtin_amdgcn_ballot_w64(wait <= p) != 0;
      p = down ? p + 1 : nd.skip;
      nd = down ? na : nb;
    }
  } else {
    // nodes of this lane's tree: [root, end) (graph g owns sorted points
    // [goff[g], goff[g+1]))
    int32_t root = 0, end = N;
    if (valid) {
      const int32_t g = (int32_t)(scodes[i] >> 48);
      root = first_at[goff[g]];
      end = goff[g + 1] < n ? first_at[goff[g + 1]] : N;
    }
    int32_t next = valid ? root : 0x7fffffff;
    int32_t p = wave_min(next);
    while (p < N) {
      p = __builtin_amdgcn_readfirstlane(p);
      const BHNode nd = nodes[p];
      // visit_node leaves `next` at p when the lane opens p
      const bool act = next == p;
      visit_node<STATS, CT>(nd, act, i, xt, yt, qx2i, qy2i, q, theta2, xsx, xsy,
                            nd.skip >= end ? 0x7fffffff : nd.skip, next, fx, fy, acc, pairs);
      const bool opened = act && next == p;
      if (opened) next = p + 1;
      if (__any(opened)) p = p + 1;
      else p = wave_min(next);
    }
  }
  if (valid) F[order[i]] = make_float2(fx, fy);
  if (STATS) {
    acc = wave_sum(acc);
    pairs = wave_sum(pairs);
    if (l == 0) { atomicAdd(&stats[0], acc); atomicAdd(&stats[1], pairs); }
  }
}

// ---- exact all-pairs
// Grid (target blocks) x (source slabs): a lane owns one target, the slab's
// sources are read at wave-uniform addresses (scalar loads, broadcast to the
// lanes), and each slab writes its partial sums; k_exact_sum adds the slabs
// of a target in slab order, so the result does not depend on timing.  With
// q = 0 the pair term is (dx, dy) / d^2; a bias of 1e-30 in d^2 makes the
// self pair and coincident points contribute exactly 0 (0 * 1e30) and leaves
// every d^2 above 1e-23 unchanged, as the skip of d^2 = 0 does for q != 0.
constexpr int EX_T = 256;
constexpr int EX_BLOCKS = 2048;  // target blocks x slabs to aim for (8 waves per SIMD)

template <bool Q0>
__global__ __launch_bounds__(EX_T) void k_exact(const float2* __restrict__ xy, int32_t n,
                                                int32_t L, float q, float2* __restrict__ out) {
  raise_wave_priority();
  const int32_t u = blockIdx.x * EX_T + threadIdx.x;
  const float2 xu = u < n ? xy[u] : make_float2(0.f, 0.f);
  const int32_t j0 = blockIdx.y * L;
  const int32_t j1 = min(n, j0 + L);
  float fx = 0.f, fy = 0.f;
  if (Q0) {
    int32_t j = j0;
    for (; j + 8 <= j1; j += 8) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const float2 p = xy[j + t];
        const float dx = xu.x - p.x, dy = xu.y - p.y;
        const float f = __builtin_amdgcn_rcpf(fmaf(dx, dx, fmaf(dy, dy, 1e-30f)));
        fx = fmaf(dx, f, fx);
        fy = fmaf(dy, f, fy);
      }
    }
    for (; j < j1; ++j) {
      const float2 p = xy[j];
      const float dx = xu.x - p.x, dy = xu.y - p.y;
      const float f = __builtin_amdgcn_rcpf(fmaf(dx, dx, fmaf(dy, dy, 1e-30f)));
      fx = fmaf(dx, f, fx);
      fy = fmaf(dy, f, fy);
    }
  } else {
    for (int32_t j = j0; j < j1; ++j) {
      const float2 p = xy[j];
      rq_add(xu.x - p.x, xu.y - p.y, q, 1.f, fx, fy);
    }
  }
  if (u < n) out[(size_t)blockIdx.y * n + u] = make_float2(fx, fy);
}

__global__ void k_exact_sum(const float2* __restrict__ part, int32_t n, int32_t S,
                            float2* __restrict__ F) {
  raise_wave_priority();
  const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  float fx = 0.f, fy = 0.f;
  for (int32_t s = 0; s < S; ++s) {
    const float2 v = part[(size_t)s * n + u];
    fx += v.x;
    fy += v.y;
  }
  F[u] = make_float2(fx, fy);
}

}  // namespace

hipError_t farfield_exact(BHWork* w, int32_t n, const float* xy, double q, float* F,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int32_t tb = (n + EX_T - 1) / EX_T;
  // slabs: enough blocks to fill the chip, at least 64 sources per slab
  int32_t S = std::max(1, std::min((EX_BLOCKS + tb - 1) / tb, (n + 63) / 64));
  const int32_t L = (n + S - 1) / S;
  S = (n + L - 1) / L;
  float2* out = (float2*)F;
  if (S > 1) {
    MM_TRY(ensure<float2>(w->expart, (size_t)S * n, s));
    out = w->expart.as<float2>();
  }
  const dim3 grid(tb, S);
  if (q == 0.0)
    k_exact<true><<<grid, EX_T, 0, s>>>((const float2*)xy, n, L, (float)q, out);
  else
    k_exact<false><<<grid, EX_T, 0, s>>>((const float2*)xy, n, L, (float)q, out);
  MM_TRY(hipGetLastError());
  if (S > 1) {
    k_exact_sum<<<(n + 255) / 256, 256, 0, s>>>(out, n, S, (float2*)F);
    MM_TRY(hipGetLastError());
  }
  return hipSuccess;
}

hipError_t bh_build_tree(BHWork* w, int32_t n, const float* xy, int64_t* nodes_out,
                         hipStream_t s, const BHSeg* seg) {
  const size_t N2 = 2 * (size_t)n;
  MM_TRY(ensure<uint64_t>(w->codes, n, s));
  MM_TRY(ensure<int32_t>(w->order, n, s));
  MM_TRY(ensure<float>(w->xsx, n, s));
  MM_TRY(ensure<float>(w->xsy, n, s));
  MM_TRY(ensure<uint2>(w->ix, n, s));
  MM_TRY(ensure<double>(w->px, n + 1, s));
  MM_TRY(ensure<double>(w->py, n + 1, s));
  MM_TRY(ensure<uint32_t>(w->nmask, n, s));
  MM_TRY(ensure<int4>(w->ntmp, N2, s));
  MM_TRY(ensure<int32_t>(w->first_at, (size_t)n + 1, s));
  MM_TRY(ensure<BHNode>(w->nodes, N2, s));
  MM_TRY(ensure<int32_t>(w->counter, 1, s));
  const int32_t M = seg ? seg->M : 1;
  MM_TRY(ensure<BoxInfo>(w->box, (size_t)M, s));
  MM_TRY(ensure<unsigned long long>(w->statc, 2, s));
  if (!seg && n <= BHS_MAX) {
    // small trees: one launch
    k_bh_small<<<1, BHS_T, 0, s>>>((const float2*)xy, n, w->box.as<BoxInfo>(), w->codes.as<uint64_t>(),
                                     w->order.as<int32_t>(), w->xsx.as<float>(), w->xsy.as<float>(),
                                     w->ix.as<uint2>(), w->px.as<double>(), w->py.as<double>(),
                                     w->nodes.as<BHNode>(), w->counter.as<int32_t>(), nodes_out);
    return hipGetLastError();
  }
  const int nbb = std::min(1024, std::max(1, (n + BB_T - 1) / BB_T));
  MM_TRY(ensure<float4>(w->partial, nbb, s));
  const int32_t nps = (n + PS_TILE - 1) / PS_TILE;
  MM_TRY(ensure<double>(w->pparts, 2 * ((size_t)nps + 1), s));
  MM_TRY(ensure<int32_t>(w->npart, (size_t)nps + 1, s));
  DevBuf& pparts = w->pparts;
  MM_TRY(ensure<unsigned long long>(w->statc, 2, s));

  int cbits = 48;
  if (seg) {
    k_bbox_seg<<<M, BB_T, 0, s>>>((const float2*)xy, seg->goff, w->box.as<BoxInfo>());
    while ((1ll << (cbits - 48)) < (int64_t)M) cbits++;
  } else {
    k_bbox_partial<<<nbb, BB_T, 0, s>>>((const float2*)xy, n, w->partial.as<float4>());
    k_bbox_final<<<1, 64, 0, s>>>(w->partial.as<float4>(), nbb, w->box.as<BoxInfo>());
  }
  k_morton<<<(n + 255) / 256, 256, 0, s>>>((const float2*)xy, n, w->box.as<BoxInfo>(),
                                           seg ? seg->gid : nullptr, w->codes.as<uint64_t>(),
                                           w->order.as<int32_t>(), w->nmask.as<uint32_t>());
  MM_TRY(hipGetLastError());
  MM_TRY(radix_sort_pairs(w->codes.as<uint64_t>(), w->order.as<int32_t>(), n, cbits, s, &w->sort));
  // sorted points, their tile sums, then the FP64 prefix sums of both axes
  k_gather_tiles<<<nps, PS_T, 0, s>>>((const float2*)xy, w->order.as<int32_t>(),
                                      w->codes.as<uint64_t>(), n, w->xsx.as<float>(),
                                      w->xsy.as<float>(), w->ix.as<uint2>(), pparts.as<double>(),
                                      nps + 1, w->counter.as<int32_t>());
  // node records at fixed slots and the masks of the nodes starting at each
  // point (at most n leaves and n - 1 internal nodes); the node count stays
  // on the device (cleared by k_gather_tiles: no memsets, this sequence is
  // replayed from HIP graphs)
  k_emit_nodes<<<(n + 255) / 256, 256, 0, s>>>(w->codes.as<uint64_t>(), n, w->ntmp.as<int4>(),
                                               w->nmask.as<uint32_t>(), w->counter.as<int32_t>());
  // scans: the FP64 tile sums of both axes, the node-start counts per tile,
  // then each tile's FP64 prefix sums and first-node indices in one grid
  k_fsum_parts<<<2, 1024, 0, s>>>(pparts.as<double>(), nps);
  k_node_tiles<<<nps, PS_T, 0, s>>>(w->nmask.as<uint32_t>(), n, w->npart.as<int32_t>());
  const bool fused = nps <= NODE_FUSE_MAX;
  if (!fused) k_node_parts<<<1, 1024, 0, s>>>(w->npart.as<int32_t>(), nps);
#define MM_SCANS(F)                                                                               \
  k_tile_scans<F><<<dim3(nps, 3), PS_T, 0, s>>>(                                                  \
      w->xsx.as<float>(), w->xsy.as<float>(), n, pparts.as<double>(), w->px.as<double>(),          \
      w->py.as<double>(), w->nmask.as<uint32_t>(), w->npart.as<int32_t>(), w->first_at.as<int32_t>())
  if (fused) MM_SCANS(true);
  else MM_SCANS(false);
#undef MM_SCANS
  MM_TRY(hipGetLastError());
  k_finalize_nodes<<<(unsigned)((N2 + 255) / 256), 256, 0, s>>>(
      w->ntmp.as<int4>(), w->nmask.as<uint32_t>(), n, w->first_at.as<int32_t>(),
      w->px.as<double>(), w->py.as<double>(), w->xsx.as<float>(), w->xsy.as<float>(),
      w->ix.as<uint2>(), w->nodes.as<BHNode>(), nodes_out, w->codes.as<uint64_t>());
  return hipGetLastError();
}

hipError_t farfield_bh(BHWork* w, int32_t n, const float* xy, double q, double theta, float* F,
                       uint64_t* codes_out, int32_t* order_out, int64_t* nodes_out,
                       int64_t* n_nodes_out, int count_stats, FarStats* st, hipStream_t s,
                       const BHSeg* seg) {
  MM_TRY(bh_build_tree(w, n, xy, nodes_out, s, seg));
  const uint64_t* sc = seg ? w->codes.as<uint64_t>() : nullptr;
  const int32_t* go = seg ? seg->goff : nullptr;
  const int32_t* Np = w->counter.as<int32_t>();
  if (count_stats) MM_TRY(hipMemsetAsync(w->statc.p, 0, 2 * sizeof(unsigned long long), s));
  const int32_t nw = (n + 63) / 64;
  const int32_t nblk = (nw + TR_WAVES - 1) / TR_WAVES;
  // the containment test is needed only above theta^2 = 2 (visit_node)
  const double theta2 = theta * theta;
  const bool ct = theta2 > 2.0;
#define MM_TR(ST, SG, CT)                                                                        \
  k_traverse<ST, SG, CT><<<nblk, 64 * TR_WAVES, 0, s>>>(                                           \
      w->nodes.as<BHNode>(), Np, w->xsx.as<float>(), w->xsy.as<float>(), w->ix.as<uint2>(),       \
      w->order.as<int32_t>(), n, (float)q, theta2, (float2*)F,                                     \
      ST ? w->statc.as<unsigned long long>() : nullptr, sc, go, w->first_at.as<int32_t>())
#define MM_TR2(ST, SG) { if (ct) MM_TR(ST, SG, true); else MM_TR(ST, SG, false); }
  if (count_stats) { if (seg) MM_TR2(true, true) else MM_TR2(true, false) }
  else { if (seg) MM_TR2(false, true) else MM_TR2(false, false) }
#undef MM_TR2
#undef MM_TR
  MM_TRY(hipGetLastError());
  if (codes_out) {
    // codes in id order
    DevBuf tmp;
    MM_TRY(tmp.alloc(sizeof(uint64_t) * (size_t)n, s));
    k_morton<<<(n + 255) / 256, 256, 0, s>>>((const float2*)xy, n, w->box.as<BoxInfo>(),
                                             seg ? seg->gid : nullptr, codes_out, tmp.as<int32_t>(),
                                             nullptr);
  }
  if (order_out)
    MM_TRY(hipMemcpyAsync(order_out, w->order.p, sizeof(int32_t) * (size_t)n,
                          hipMemcpyDeviceToDevice, s));
  int32_t N = 0;
  if (n_nodes_out || st) {
    MM_TRY(hipMemcpyAsync(&N, w->counter.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MM_TRY(hipStreamSynchronize(s));
  }
  if (n_nodes_out) *n_nodes_out = N;
  if (st) {
    st->nodes = N;
    st->accepted = st->leaf_pairs = st->coincident = 0;
    if (count_stats) {
      unsigned long long h[2];
      MM_TRY(hipMemcpyAsync(h, w->statc.p, sizeof(h), hipMemcpyDeviceToHost, s));
      MM_TRY(hipStreamSynchronize(s));
      st->accepted = (int64_t)h[0];
      st->leaf_pairs = (int64_t)h[1];
    }
  }
  return hipGetLastError();
}

}  // namespace mm
