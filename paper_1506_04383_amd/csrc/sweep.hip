// One Jacobi iteration of the local update, Eq. 2, over the k-hop sets:
//   A_u = sum_{v in S(u)} w_uv (x_v + d_uv (x_u - x_v)/|x_u - x_v|)
//   C_u = sum_{v in S(u)} r_q(u, v)
//   x'_u = (A_u + alpha (F_u - C_u)) / rho_u,   rho_u = sum_{v in S(u)} w_uv
// F is the far field over all v != u, so F - C is the entropy term over the
// pairs outside S (the subtraction Eq. 3 uses for its last sum).  Target
// distances: d = hop on the finest level, hop (sqrt c_u + sqrt c_v) scale on
// coarse levels; w = d^-2.  A coincident pair contributes w x_v to A only.
//
// A group of G lanes owns one row and streams its ids (coalesced) while
// gathering x_v; the row's hop boundaries sit in registers.  The relative
// change |x'-x|^2, |x|^2 is reduced in FP64 per block in fixed order and the
// block partials are summed in order by a second kernel (deterministic).
#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

constexpr int SW_T = 256;
constexpr int KMAX = 8;

template <int G, bool COARSE, bool Q0>
__global__ __launch_bounds__(SW_T) void k_sweep(
    int32_t n, int32_t k, const int64_t* __restrict__ off, const int32_t* __restrict__ hend,
    const int32_t* __restrict__ nbr, const float* __restrict__ sqrtc, float scale,
    const float2* __restrict__ xy, const float2* __restrict__ F, float alpha, float q,
    float2* __restrict__ out, double2* __restrict__ part, const int32_t* __restrict__ gid,
    const float* __restrict__ galpha, const float* __restrict__ alpha_dev) {
  constexpr int RPB = SW_T / G;  // rows per block
  __shared__ double2 red[RPB];
  const int gl = threadIdx.x % G, gi = threadIdx.x / G;
  const int32_t u = blockIdx.x * RPB + gi;
  double2 dd = make_double2(0.0, 0.0);
  // batches: each graph has its own alpha; a negative one marks a finished
  // graph, whose coordinates are carried over unchanged
  if (alpha_dev) alpha = *alpha_dev;
  if (galpha && u < n) alpha = galpha[gid[u]];
  if (u < n && alpha < 0.f) {
    if (gl == 0) out[u] = xy[u];
  } else if (u < n) {
    const int64_t beg = off[u], end = off[u + 1];
    int32_t he[KMAX];
#pragma unroll
    for (int h = 0; h < KMAX; ++h) he[h] = h < k ? hend[(int64_t)u * k + h] : 0x7fffffff;
    const float2 xu = xy[u];
    const float scu = COARSE ? sqrtc[u] : 0.f;
    float ax = 0.f, ay = 0.f, cx = 0.f, cy = 0.f, rho = 0.f;
    // U independent entries per lane per step: their id and coordinate loads
    // are issued before any is consumed, so U gathers are in flight per lane.
    constexpr int U = 8;
    for (int64_t e0 = beg + gl; e0 < end; e0 += (int64_t)U * G) {
      int32_t vv[U];
      float2 xv[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const int64_t e = e0 + (int64_t)j * G;
        vv[j] = e < end ? nbr[e] : -1;
      }
#pragma unroll
      for (int j = 0; j < U; ++j) xv[j] = vv[j] >= 0 ? xy[vv[j]] : make_float2(0.f, 0.f);
#pragma unroll
      for (int j = 0; j < U; ++j) {
        if (vv[j] < 0) continue;
        const int32_t rel = (int32_t)(e0 + (int64_t)j * G - beg);
        int h = 1;
#pragma unroll
        for (int q2 = 0; q2 < KMAX - 1; ++q2) h += (rel >= he[q2]) ? 1 : 0;
        float d;
        if (COARSE) d = (float)h * (scu + sqrtc[vv[j]]) * scale;
        else d = (float)h;
        const float w = 1.f / (d * d);
        const float dx = xu.x - xv[j].x, dy = xu.y - xv[j].y;
        const float D2 = dx * dx + dy * dy;
        rho += w;
        if (D2 > 0.f) {
          const float inv = rsqrtf(D2);
          ax += w * (xv[j].x + d * dx * inv);
          ay += w * (xv[j].y + d * dy * inv);
          float f;
          if (Q0) f = inv * inv;
          else f = powf(D2, -0.5f * (q + 2.f));
          cx += dx * f;
          cy += dy * f;
        } else {
          ax += w * xv[j].x;
          ay += w * xv[j].y;
        }
      }
    }
    ax = group_sum(ax, G); ay = group_sum(ay, G);
    cx = group_sum(cx, G); cy = group_sum(cy, G);
    rho = group_sum(rho, G);
    if (gl == 0) {
      const float2 fu = F[u];
      float2 xn;
      xn.x = (ax + alpha * (fu.x - cx)) / rho;
      xn.y = (ay + alpha * (fu.y - cy)) / rho;
      out[u] = xn;
      const double ex = (double)xn.x - (double)xu.x, ey = (double)xn.y - (double)xu.y;
      dd.x = ex * ex + ey * ey;
      dd.y = (double)xu.x * (double)xu.x + (double)xu.y * (double)xu.y;
    }
  }
  if (gl == 0) red[gi] = dd;
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 s = make_double2(0.0, 0.0);
    for (int i = 0; i < RPB; ++i) { s.x += red[i].x; s.y += red[i].y; }
    part[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(1024) void k_sum_parts(const double2* __restrict__ part, int32_t m,
                                                    double* __restrict__ out) {
  __shared__ double shx[1024], shy[1024];
  double sx = 0.0, sy = 0.0;
  // fixed assignment: thread t sums parts t, t+1024, ... in order
  for (int32_t i = threadIdx.x; i < m; i += 1024) { sx += part[i].x; sy += part[i].y; }
  shx[threadIdx.x] = sx;
  shy[threadIdx.x] = sy;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      shx[threadIdx.x] += shx[threadIdx.x + s];
      shy[threadIdx.x] += shy[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[0] = shx[0]; out[1] = shy[0]; }
}

template <int G>
hipError_t launch(const KhopDev& kh, bool coarse, bool q0, const float* sqrtc, float scale,
                  const float* xy, const float* F, float alpha, float q, float* out, double2* part,
                  int32_t nb, hipStream_t s, const int32_t* gid, const float* galpha,
                  const float* alpha_dev) {
  const float2* x2 = (const float2*)xy;
  const float2* F2 = (const float2*)F;
  float2* o2 = (float2*)out;
#define MM_SW(C, Q)                                                                          \
  k_sweep<G, C, Q><<<nb, SW_T, 0, s>>>(kh.n, kh.k, kh.off, kh.hend, kh.nbr, sqrtc, scale, x2, \
                                       F2, alpha, q, o2, part, gid, galpha, alpha_dev)
  if (coarse) { if (q0) MM_SW(true, true); else MM_SW(true, false); }
  else { if (q0) MM_SW(false, true); else MM_SW(false, false); }
#undef MM_SW
  return hipGetLastError();
}

}  // namespace

hipError_t sweep_into(const KhopDev& kh, int32_t level, const float* sqrtc, double scale,
                      const float* xy, const float* F, double alpha, double q, float* xy_out,
                      double* delta2_dev, double2* part, size_t part_bytes, hipStream_t s,
                      const int32_t* gid, const float* galpha, const float* alpha_dev,
                      int32_t group) {
  if (kh.k > KMAX) return hipErrorInvalidValue;
  const int G = group > 0 ? group : row_group(kh);
  if (G != 8 && G != 16 && G != 32 && G != 64) return hipErrorInvalidValue;
  const int32_t nb = sweep_blocks(kh.n, G);
  if (!part || part_bytes < sizeof(double2) * (size_t)nb) return hipErrorInvalidValue;
  const bool coarse = (level > 0) && sqrtc != nullptr;
  const bool q0 = (q == 0.0);
  hipError_t e;
  switch (G) {
    case 64: e = launch<64>(kh, coarse, q0, sqrtc, (float)scale, xy, F, (float)alpha, (float)q, xy_out, part, nb, s, gid, galpha, alpha_dev); break;
    case 32: e = launch<32>(kh, coarse, q0, sqrtc, (float)scale, xy, F, (float)alpha, (float)q, xy_out, part, nb, s, gid, galpha, alpha_dev); break;
    case 16: e = launch<16>(kh, coarse, q0, sqrtc, (float)scale, xy, F, (float)alpha, (float)q, xy_out, part, nb, s, gid, galpha, alpha_dev); break;
    default: e = launch<8>(kh, coarse, q0, sqrtc, (float)scale, xy, F, (float)alpha, (float)q, xy_out, part, nb, s, gid, galpha, alpha_dev); break;
  }
  MM_TRY(e);
  k_sum_parts<<<1, 1024, 0, s>>>(part, nb, delta2_dev);
  return hipGetLastError();
}

hipError_t sweep(const KhopDev& kh, int32_t level, const float* sqrtc, double scale,
                 const float* xy, const float* F, double alpha, double q, float* xy_out,
                 double* delta2_dev, hipStream_t s, const int32_t* gid, const float* galpha,
                 const float* alpha_dev, DevBuf* part_ws, int32_t group) {
  if (kh.k > KMAX) return hipErrorInvalidValue;
  const int G = group > 0 ? group : row_group(kh);
  const int32_t nb = sweep_blocks(kh.n, G);
  DevBuf local;
  DevBuf& part = part_ws ? *part_ws : local;
  if (part.bytes < sizeof(double2) * (size_t)nb) MM_TRY(part.alloc(sizeof(double2) * (size_t)nb, s));
  return sweep_into(kh, level, sqrtc, scale, xy, F, alpha, q, xy_out, delta2_dev,
                    part.as<double2>(), part.bytes, s, gid, galpha, alpha_dev, G);
}

}  // namespace mm
