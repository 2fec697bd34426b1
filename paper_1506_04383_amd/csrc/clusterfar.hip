// Cluster far field: the first two sums of Eq. 3 (Section 3.2, "Faster
// Local Improvement").  For u on level l,
//   F_u = sum over v != u in u's own cluster of the next coarser level of r(u, v)
//       + sum over vertices j != M_h(u) of the approximation level of
//         nu_j r(x_u, xp_j),
// where the approximation level is h levels beneath (or the coarsest), M_h
// maps a level-l vertex to its representative there, nu_j counts the level-l
// vertices j represents and xp_j is their node-weighted midpoint, refreshed
// from the current coordinates before every evaluation.  Vertices that share
// u's representative but not u's own cluster contribute nothing (the
// merged-vertex error the section describes for h > 1).
//
// Setup (once per level): the level's vertices sorted by cluster id for both
// maps (stable radix sort, so members are in ascending id) and the cluster
// start offsets.  Per evaluation: k_cf_mid forms (xp_j, nu_j) with one wave
// per representative (FP64 sums in a fixed order), then k_cf_far runs the
// all-pairs loop against the representatives -- read at wave-uniform
// addresses, i.e. scalar loads -- split into source slabs to fill the chip,
// plus the exact terms of u's own cluster, and k_cf_sum adds the slabs in
// slab order.  Nothing is allocated per evaluation.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

constexpr int CF_T = 256;
constexpr int CF_BLOCKS = 2048;  // target blocks x slabs to aim for

__global__ void k_cf_check(int32_t n, const int32_t* __restrict__ cl1, int32_t n1,
                           const int32_t* __restrict__ clh, int32_t nh, int32_t* __restrict__ bad) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (cl1[v] < 0 || cl1[v] >= n1 || clh[v] < 0 || clh[v] >= nh) atomicOr(bad, 1);
}

__global__ void k_cf_keys(int32_t n, const int32_t* __restrict__ cl, uint64_t* __restrict__ keys,
                          int32_t* __restrict__ vals) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  keys[v] = (uint64_t)(uint32_t)cl[v];
  vals[v] = v;
}

// off[j] = first position of cluster j in the sorted keys (j in [0, nc]);
// empty clusters get an empty range
__global__ void k_cf_bounds(int32_t n, const uint64_t* __restrict__ skeys, int32_t nc,
                            int32_t* __restrict__ off) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nc) return;
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (skeys[mid] < (uint64_t)j) lo = mid + 1; else hi = mid;
  }
  off[j] = lo;
}

__global__ void k_cf_compose(int32_t n, const int32_t* __restrict__ in,
                             const int32_t* __restrict__ cl, int32_t* __restrict__ out) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) out[v] = cl[in[v]];
}

// one wave per representative: (weighted midpoint x, y, nu, 0)
__global__ __launch_bounds__(256) void k_cf_mid(int32_t nh, const int32_t* __restrict__ offh,
                                                const int32_t* __restrict__ ordh,
                                                const float2* __restrict__ xy,
                                                const int32_t* __restrict__ c,
                                                float4* __restrict__ rep) {
  const int32_t j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = lane_id();
  if (j >= nh) return;
  const int32_t b = offh[j], e = offh[j + 1];
  double sx = 0.0, sy = 0.0, sw = 0.0;
  for (int32_t i = b + l; i < e; i += 64) {
    const int32_t v = ordh[i];
    const double w = c ? (double)c[v] : 1.0;
    const float2 p = xy[v];
    sx += w * (double)p.x;
    sy += w * (double)p.y;
    sw += w;
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sw = wave_sum(sw);
  if (l == 0)
    rep[j] = e > b ? make_float4((float)(sx / sw), (float)(sy / sw), (float)(e - b), 0.f)
                   : make_float4(0.f, 0.f, 0.f, 0.f);
}

// q = 0: (dx, dy) m / (D^2 + 1e-30): an excluded representative has m = 0 and
// a coincident point dx = dy = 0, both exactly 0; the bias leaves every
// D^2 above 1e-23 unchanged.  q != 0 goes through rq_add's D^2 > 0 test.
template <bool Q0>
__device__ inline void cf_term(float dx, float dy, float m, float q, float& fx, float& fy) {
  if (Q0) {
    const float f = m * __builtin_amdgcn_rcpf(fmaf(dx, dx, fmaf(dy, dy, 1e-30f)));
    fx = fmaf(dx, f, fx);
    fy = fmaf(dy, f, fy);
  } else {
    const float d2 = fmaf(dx, dx, dy * dy);
    if (d2 > 0.f && m != 0.f) {
      const float f = m * powf(d2, -0.5f * (q + 2.f));
      fx = fmaf(dx, f, fx);
      fy = fmaf(dy, f, fy);
    }
  }
}

template <bool Q0>
__global__ __launch_bounds__(CF_T) void k_cf_far(
    int32_t n, int32_t L, const float2* __restrict__ xy, const float4* __restrict__ rep,
    int32_t nh, const int32_t* __restrict__ clh, const int32_t* __restrict__ cl1,
    const int32_t* __restrict__ off1, const int32_t* __restrict__ ord1, float q,
    float2* __restrict__ out) {
  const int32_t u = blockIdx.x * CF_T + threadIdx.x;
  const bool valid = u < n;
  const float2 xu = valid ? xy[u] : make_float2(0.f, 0.f);
  const int32_t mh = valid ? clh[u] : -1;
  const int32_t j0 = blockIdx.y * L;
  const int32_t j1 = min(nh, j0 + L);
  float fx = 0.f, fy = 0.f;
  int32_t j = j0;
  for (; j + 4 <= j1; j += 4) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float4 r = rep[j + t];
      cf_term<Q0>(xu.x - r.x, xu.y - r.y, j + t == mh ? 0.f : r.z, q, fx, fy);
    }
  }
  for (; j < j1; ++j) {
    const float4 r = rep[j];
    cf_term<Q0>(xu.x - r.x, xu.y - r.y, j == mh ? 0.f : r.z, q, fx, fy);
  }
  if (blockIdx.y == 0 && valid) {
    // exact terms within u's own cluster of the next coarser level
    const int32_t a = cl1[u];
    for (int32_t i = off1[a]; i < off1[a + 1]; ++i) {
      const int32_t v = ord1[i];
      const float2 p = xy[v];
      cf_term<Q0>(xu.x - p.x, xu.y - p.y, v == u ? 0.f : 1.f, q, fx, fy);
    }
  }
  if (valid) out[(size_t)blockIdx.y * n + u] = make_float2(fx, fy);
}

__global__ void k_cf_sum(const float2* __restrict__ part, int32_t n, int32_t S,
                         float2* __restrict__ F) {
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

inline unsigned nb256(int64_t m) { return (unsigned)((m + 255) / 256); }

// sorted member lists and offsets of a cluster map
hipError_t members(int32_t n, const int32_t* cl, int32_t nc, DevBuf& ord, DevBuf& off,
                   hipStream_t s) {
  DevBuf keys;
  MM_TRY(keys.alloc(sizeof(uint64_t) * (size_t)std::max(n, 1), s));
  MM_TRY(ord.alloc(sizeof(int32_t) * (size_t)std::max(n, 1), s));
  MM_TRY(off.alloc(sizeof(int32_t) * ((size_t)nc + 1), s));
  if (n > 0) {
    k_cf_keys<<<nb256(n), 256, 0, s>>>(n, cl, keys.as<uint64_t>(), ord.as<int32_t>());
    MM_TRY(hipGetLastError());
    int bits = 1;
    while ((1ll << bits) < (int64_t)nc) bits++;
    MM_TRY(radix_sort_pairs(keys.as<uint64_t>(), ord.as<int32_t>(), n, bits, s));
  }
  k_cf_bounds<<<nb256((int64_t)nc + 1), 256, 0, s>>>(n, keys.as<uint64_t>(), nc, off.as<int32_t>());
  MM_TRY(hipGetLastError());
  return hipStreamSynchronize(s);  // keys is released on return
}

}  // namespace

hipError_t cluster_far_check(int32_t n, const int32_t* cl1, int32_t n1, const int32_t* clh,
                             int32_t nh, bool* ok, hipStream_t s) {
  DevBuf bad;
  MM_TRY(bad.alloc(sizeof(int32_t), s));
  MM_TRY(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
  if (n > 0) k_cf_check<<<nb256(n), 256, 0, s>>>(n, cl1, n1, clh, nh, bad.as<int32_t>());
  MM_TRY(hipGetLastError());
  int32_t h = 0;
  MM_TRY(hipMemcpyAsync(&h, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  *ok = h == 0;
  return hipSuccess;
}

hipError_t cluster_compose(int32_t n, const int32_t* in, const int32_t* cl, int32_t* out,
                           hipStream_t s) {
  if (n > 0) k_cf_compose<<<nb256(n), 256, 0, s>>>(n, in, cl, out);
  return hipGetLastError();
}

hipError_t cluster_far_setup(int32_t n, const int32_t* cl1, int32_t n1, const int32_t* clh,
                             int32_t nh, ClusterFar* cf, hipStream_t s) {
  cf->n = n;
  cf->n1 = n1;
  cf->nh = nh;
  MM_TRY(cf->cl1.alloc(sizeof(int32_t) * (size_t)std::max(n, 1), s));
  MM_TRY(cf->clh.alloc(sizeof(int32_t) * (size_t)std::max(n, 1), s));
  if (n > 0) {
    MM_TRY(hipMemcpyAsync(cf->cl1.p, cl1, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    MM_TRY(hipMemcpyAsync(cf->clh.p, clh, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
  }
  MM_TRY(members(n, cf->cl1.as<int32_t>(), n1, cf->ord1, cf->off1, s));
  MM_TRY(members(n, cf->clh.as<int32_t>(), nh, cf->ordh, cf->offh, s));
  MM_TRY(cf->rep.alloc(sizeof(float4) * (size_t)std::max(nh, 1), s));
  // source slabs over the representatives: enough blocks to fill the chip,
  // at least 64 representatives per slab
  const int32_t tb = (n + CF_T - 1) / CF_T;
  int32_t S = std::max(1, std::min((CF_BLOCKS + std::max(tb, 1) - 1) / std::max(tb, 1),
                                   (nh + 63) / 64));
  cf->L = std::max(1, (nh + S - 1) / S);
  cf->S = std::max(1, (nh + cf->L - 1) / cf->L);
  MM_TRY(cf->part.alloc(sizeof(float2) * (size_t)cf->S * (size_t)std::max(n, 1), s));
  return hipGetLastError();
}

hipError_t cluster_far(ClusterFar& cf, const float* xy, const int32_t* c, double q, float* F,
                       hipStream_t s) {
  const int32_t n = cf.n;
  if (n <= 0) return hipSuccess;
  if (cf.nh > 0)
    k_cf_mid<<<(cf.nh + 3) / 4, 256, 0, s>>>(cf.nh, cf.offh.as<int32_t>(), cf.ordh.as<int32_t>(),
                                             (const float2*)xy, c, cf.rep.as<float4>());
  MM_TRY(hipGetLastError());
  const dim3 grid((n + CF_T - 1) / CF_T, cf.S);
  if (q == 0.0)
    k_cf_far<true><<<grid, CF_T, 0, s>>>(n, cf.L, (const float2*)xy, cf.rep.as<float4>(), cf.nh,
                                         cf.clh.as<int32_t>(), cf.cl1.as<int32_t>(),
                                         cf.off1.as<int32_t>(), cf.ord1.as<int32_t>(), (float)q,
                                         cf.part.as<float2>());
  else
    k_cf_far<false><<<grid, CF_T, 0, s>>>(n, cf.L, (const float2*)xy, cf.rep.as<float4>(), cf.nh,
                                          cf.clh.as<int32_t>(), cf.cl1.as<int32_t>(),
                                          cf.off1.as<int32_t>(), cf.ord1.as<int32_t>(), (float)q,
                                          cf.part.as<float2>());
  MM_TRY(hipGetLastError());
  k_cf_sum<<<nb256(n), 256, 0, s>>>(cf.part.as<float2>(), n, cf.S, (float2*)F);
  return hipGetLastError();
}

}  // namespace mm
