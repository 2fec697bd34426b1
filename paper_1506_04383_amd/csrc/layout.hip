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

hipError_t sqrt_weights(int32_t n, const int32_t* c, float* out, hipStream_t s) {
  k_sqrtw<<<(n + 255) / 256, 256, 0, s>>>(n, c, out);
  return hipGetLastError();
}

}  // namespace mm
