// Placement: seeded initial layout of the coarsest graph and prolongation
// (Section 3.2: a fine vertex is drawn at a random polar offset around its
// coarse representative, angle uniform in [0, 2 pi), radius uniform in
// [0, sqrt(c(v'))]).  Draws come from the SplitMix64 counter generator:
// init uses tag 1, prolongation tag 2, draw index 2v + j.
#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

__global__ void k_init(int32_t n, uint64_t st, float2* __restrict__ xy) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  xy[v] = make_float2((float)unit24(sm64_at(st, 2ull * v)), (float)unit24(sm64_at(st, 2ull * v + 1)));
}

__global__ void k_prolong(int32_t n, const int32_t* __restrict__ cluster,
                          const int32_t* __restrict__ cc, const float2* __restrict__ cxy,
                          uint64_t st, float2* __restrict__ fxy) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t p = cluster[v];
  const double phi = 6.283185307179586 * unit24(sm64_at(st, 2ull * v));
  const double rad = sqrt((double)(cc ? cc[p] : 1)) * unit24(sm64_at(st, 2ull * v + 1));
  const float2 c = cxy[p];
  double sn, cs;
  sincos(phi, &sn, &cs);
  fxy[v] = make_float2((float)((double)c.x + rad * cs), (float)((double)c.y + rad * sn));
}

// Batches: draws keyed by the local vertex id v - goff[gid[v]].
// Initial layout for the vertices of graphs whose coarsest level this is.
__global__ void k_init_seg(int32_t n, uint64_t st, const int32_t* __restrict__ gid,
                           const int32_t* __restrict__ goff, const uint8_t* __restrict__ top,
                           float2* __restrict__ xy) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t g = gid[v];
  if (!top[g]) return;
  const uint64_t i = (uint64_t)(v - goff[g]);
  xy[v] = make_float2((float)unit24(sm64_at(st, 2ull * i)), (float)unit24(sm64_at(st, 2ull * i + 1)));
}

// Prolongation for vertices whose graph continues from the coarser level
// (cluster[v] >= 0: index in the coarser batch).
__global__ void k_prolong_seg(int32_t n, const int32_t* __restrict__ cluster,
                              const int32_t* __restrict__ cc, const float2* __restrict__ cxy,
                              uint64_t st, const int32_t* __restrict__ gid,
                              const int32_t* __restrict__ goff, float2* __restrict__ fxy) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t p = cluster[v];
  if (p < 0) return;
  const uint64_t i = (uint64_t)(v - goff[gid[v]]);
  const double phi = 6.283185307179586 * unit24(sm64_at(st, 2ull * i));
  const double rad = sqrt((double)(cc ? cc[p] : 1)) * unit24(sm64_at(st, 2ull * i + 1));
  const float2 c = cxy[p];
  double sn, cs;
  sincos(phi, &sn, &cs);
  fxy[v] = make_float2((float)((double)c.x + rad * cs), (float)((double)c.y + rad * sn));
}

// Two-vertex coarsest graphs: keep the drawn direction, set the distance to
// the target distance of the pair (the optimal one).
__global__ void k_place_pairs(int32_t M, const int32_t* __restrict__ goff,
                              const uint8_t* __restrict__ top, const int32_t* __restrict__ c,
                              int32_t level, double scale, float2* __restrict__ xy) {
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M || !top[g] || goff[g + 1] - goff[g] != 2) return;
  const int32_t a = goff[g];
  const double c0 = c ? c[a] : 1.0, c1 = c ? c[a + 1] : 1.0;
  const double d = level == 0 ? 1.0 : (sqrt(c0) + sqrt(c1)) * scale;
  const float2 p0 = xy[a], p1 = xy[a + 1];
  double dx = (double)p1.x - p0.x, dy = (double)p1.y - p0.y;
  double D = sqrt(dx * dx + dy * dy);
  if (D == 0.0) { dx = 1.0; dy = 0.0; D = 1.0; }
  xy[a + 1] = make_float2((float)(p0.x + d * dx / D), (float)(p0.y + d * dy / D));
}

__global__ void k_sqrtw(int32_t n, const int32_t* __restrict__ c, float* __restrict__ out) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) out[v] = (float)sqrt((double)(c ? c[v] : 1));
}

}  // namespace

hipError_t init_layout(int32_t n, uint64_t seed, int32_t level, float* xy, hipStream_t s) {
  k_init<<<(n + 255) / 256, 256, 0, s>>>(n, rng_stream(seed, (uint32_t)level, TAG_INIT), (float2*)xy);
  return hipGetLastError();
}

hipError_t prolong(int32_t n_fine, const int32_t* cluster, const int32_t* coarse_c,
                   const float* coarse_xy, uint64_t seed, int32_t level, float* fine_xy,
                   hipStream_t s) {
  k_prolong<<<(n_fine + 255) / 256, 256, 0, s>>>(n_fine, cluster, coarse_c, (const float2*)coarse_xy,
                                                 rng_stream(seed, (uint32_t)level, TAG_PROLONG),
                                                 (float2*)fine_xy);
  return hipGetLastError();
}

hipError_t init_layout_seg(int32_t n, uint64_t seed, int32_t level, const int32_t* gid,
                           const int32_t* goff, const uint8_t* top, float* xy, hipStream_t s) {
  k_init_seg<<<(n + 255) / 256, 256, 0, s>>>(n, rng_stream(seed, (uint32_t)level, TAG_INIT), gid,
                                             goff, top, (float2*)xy);
  return hipGetLastError();
}

hipError_t prolong_seg(int32_t n_fine, const int32_t* cluster, const int32_t* coarse_c,
                       const float* coarse_xy, uint64_t seed, int32_t level, const int32_t* gid,
                       const int32_t* goff, float* fine_xy, hipStream_t s) {
  k_prolong_seg<<<(n_fine + 255) / 256, 256, 0, s>>>(
      n_fine, cluster, coarse_c, (const float2*)coarse_xy,
      rng_stream(seed, (uint32_t)level, TAG_PROLONG), gid, goff, (float2*)fine_xy);
  return hipGetLastError();
}

hipError_t place_pairs_seg(int32_t M, const int32_t* goff, const uint8_t* top, const int32_t* c,
                           int32_t level, double scale, float* xy, hipStream_t s) {
  k_place_pairs<<<(M + 255) / 256, 256, 0, s>>>(M, goff, top, c, level, scale, (float2*)xy);
  return hipGetLastError();
}

hipError_t sqrt_weights(int32_t n, const int32_t* c, float* out, hipStream_t s) {
  k_sqrtw<<<(n + 255) / 256, 256, 0, s>>>(n, c, out);
  return hipGetLastError();
}

}  // namespace mm
