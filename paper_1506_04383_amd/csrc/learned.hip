// Learned far-field correction (q = 0): Barnes-Hut at a coarse opening
// angle plus a small MLP that predicts what the accepted cell's centre-of-
// mass term misses.
//
// For target u and accepted cell C (mass m, centre of mass com, tight-cell
// side s) let d = |x_u - com|, e = (x_u - com)/d, p = e rotated by +90
// degrees, t = s/d, kappa = m t^2 / d.  The cell adds
//     m r(x_u - com) + kappa (h0 e + h1 p),   h = MLP(f),
// f = [t, offset of com from the cell centre along e, p (units of s),
//      central second moments per unit mass rotated into (e, p)
//      (ee, pp, ep; units of s^2), log2(m)/16, 0].
// With this scaling h is the cell's dimensionless multipole coefficient: as
// t -> 0 it tends to (mu_ee - mu_pp, -2 mu_ep), the quadrupole term of the
// expansion of sum_v 1/conj(z - w_v).
//
// MLP 8 -> 64 -> 64 -> 2, ReLU, weights rounded to BF16, FP32 accumulation
// on the matrix cores.  Rows are evaluated 16 at a time in transposed form:
// layer l computes H_l^T = W_l H_{l-1}^T, so the accumulator layout of one
// layer (lane: unit 4(l/16)+j of a 16-unit block, row l%16) is the B-operand
// layout of the next and activations never leave registers.  Inference (the
// traversal, mlp_forward) uses gfx950's 16x16x32 BF16 product on pairs of
// such blocks (mlp_blocks32); training keeps the 16x16x16 form, whose
// operand layouts its backward products share.
//
// Parameters (FP32, packed): W1[64][8], b1[64], W2[64][64], b2[64], W3[2][64],
// b3[2] -- 4866 values.
#include <algorithm>

#include "bh.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int NIN = 8, NH = 64, NOUT = 2;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH,
              OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NOUT * NH,
              NPARAM = OFF_B3 + NOUT;
static_assert(NPARAM == kMlpParams, "parameter count");

// FP32 -> BF16, round to nearest even (inputs are finite): gfx950's
// v_cvt_pk_bf16_f32, two values per instruction in the packed form.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ inline uint32_t f2bf2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
// four values as one BF16 operand fragment
__device__ inline v4s f2bf4(float a, float b, float c, float d) {
  return __builtin_bit_cast(v4s, (uint2){f2bf2(a, b), f2bf2(c, d)});
}

__device__ inline v4f mfma(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Orders a wave's LDS writes before its later LDS reads of other lanes' data.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// BF16 weights staged in LDS in A-operand order.
struct MlpLds {
  uint16_t w1[NH * 16];  // [unit][feature], features 8..15 zero
  uint16_t w2[NH * NH];  // [out][in]
  uint16_t w3[16 * NH];  // [out][in], rows 2..15 zero
  float b1[NH], b2[NH], b3[4];
};

__device__ void stage_weights(const float* __restrict__ w, MlpLds& L) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < NH * 16; i += nt) {
    const int u = i >> 4, k = i & 15;
    L.w1[i] = k < NIN ? f2bf(w[OFF_W1 + u * NIN + k]) : (uint16_t)0;
  }
  for (int i = tid; i < NH * NH; i += nt) L.w2[i] = f2bf(w[OFF_W2 + i]);
  for (int i = tid; i < 16 * NH; i += nt) L.w3[i] = (i >> 6) < NOUT ? f2bf(w[OFF_W3 + i]) : (uint16_t)0;
  for (int i = tid; i < NH; i += nt) {
    L.b1[i] = w[OFF_B1 + i];
    L.b2[i] = w[OFF_B2 + i];
  }
  if (tid < 4) L.b3[tid] = tid < NOUT ? w[OFF_B3 + tid] : 0.f;
}

__device__ inline v4s ld4(const uint16_t* p) { return *reinterpret_cast<const v4s*>(p); }

// gfx950's 16x16x32 BF16 product: A lane l = row l%16, K 8(l/16)..+7; B lane
// l = column l%16, the same K; C/D as in the 16x16x16 form.  Used for
// inference.  K is taken in a permuted order: K slot 8g+j (j < 4) is input
// unit 32p + 4g + j and slot 8g+4+j is unit 32p + 16 + 4g + j, so a pair of
// accumulator blocks of the previous layer (lane: units 4g..4g+3 of each) is
// the B fragment as it is, and the A fragment is two 4-value loads of the
// weight row.
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ inline v4f mfma32(v8s a, v8s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
__device__ inline v8s cat8(v4s lo, v4s hi) {
  return v8s{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}
// writes the low (hi = 0) or high half of a fragment
__device__ inline void set_half(v8s& v, int hi, v4s h) {
  if (hi) { v[4] = h[0]; v[5] = h[1]; v[6] = h[2]; v[7] = h[3]; }
  else { v[0] = h[0]; v[1] = h[1]; v[2] = h[2]; v[3] = h[3]; }
}

// Forward pass of up to four 16-row blocks on the 16x16x32 product,
// interleaved layer by layer (their matrix-core chains are independent).
// x[b]: lane l < 16 holds the 8 features of row l of block b (others zero).
// Lanes 0-15 return h of row l of block b in o[b] (.x, .y).
__device__ inline void mlp_blocks32(const MlpLds& L, const v8s* x, int nb, v4f* o) {
  const int l = lane_id(), r = l & 15, g = l >> 4;
  // activations held directly as B fragments: a1[b][p] = blocks 2p, 2p+1
  v8s a1[4][2], a2[4][2];
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    // layer 1: K = the 8 features (slots of lane group 0), zero elsewhere
    const v8s w = g == 0 ? *reinterpret_cast<const v8s*>(&L.w1[(ob * 16 + r) * 16])
                         : v8s{0, 0, 0, 0, 0, 0, 0, 0};
    float bias[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bias[j] = L.b1[ob * 16 + 4 * g + j];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (b < nb) {
        const v4f c = mfma32(w, x[b], v4f{0.f, 0.f, 0.f, 0.f});
        const v4s h = f2bf4(fmaxf(c[0] + bias[0], 0.f), fmaxf(c[1] + bias[1], 0.f),
                            fmaxf(c[2] + bias[2], 0.f), fmaxf(c[3] + bias[3], 0.f));
        set_half(a1[b][ob >> 1], ob & 1, h);
      }
    }
  }
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    v4f c[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) c[b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kp = 0; kp < 2; ++kp) {
      const uint16_t* wr = &L.w2[(ob * 16 + r) * NH + kp * 32 + 4 * g];
      const v8s w = cat8(ld4(wr), ld4(wr + 16));
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (b < nb) c[b] = mfma32(w, a1[b][kp], c[b]);
    }
    float bias[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bias[j] = L.b2[ob * 16 + 4 * g + j];
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (b < nb)
        set_half(a2[b][ob >> 1], ob & 1,
                 f2bf4(fmaxf(c[b][0] + bias[0], 0.f), fmaxf(c[b][1] + bias[1], 0.f),
                       fmaxf(c[b][2] + bias[2], 0.f), fmaxf(c[b][3] + bias[3], 0.f)));
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) o[b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kp = 0; kp < 2; ++kp) {
    const uint16_t* wr = &L.w3[r * NH + kp * 32 + 4 * g];
    const v8s w = cat8(ld4(wr), ld4(wr + 16));
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (b < nb) o[b] = mfma32(w, a2[b][kp], o[b]);
  }
  const float b30 = L.b3[0], b31 = L.b3[1];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    o[b][0] += b30;
    o[b][1] += b31;
  }
}

// Forward pass of 16 rows.  x: B operand of the features (lane l < 32: row
// l%16, features 4(l/16)..+3; other lanes zero).  Lanes 0-15 return h of row
// l in (.x, .y).  KEEP stores the pre-activations and BF16 activations in
// accumulator layout for the backward pass.
template <bool KEEP>
__device__ inline v4f mlp16(const MlpLds& L, v4s x, v4f* z1, v4s* h1, v4f* z2, v4s* h2) {
  const int l = lane_id(), r = l & 15, g = l >> 4;
  v4s a1[4], a2[4];
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    v4f c = {0.f, 0.f, 0.f, 0.f};
    c = mfma(ld4(&L.w1[(ob * 16 + r) * 16 + 4 * g]), x, c);
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] += L.b1[ob * 16 + 4 * g + j];
    const v4s hb = f2bf4(fmaxf(c[0], 0.f), fmaxf(c[1], 0.f), fmaxf(c[2], 0.f), fmaxf(c[3], 0.f));
    a1[ob] = hb;
    if (KEEP) { z1[ob] = c; h1[ob] = hb; }
  }
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    v4f c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) c = mfma(ld4(&L.w2[(ob * 16 + r) * NH + kb * 16 + 4 * g]), a1[kb], c);
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] += L.b2[ob * 16 + 4 * g + j];
    const v4s hb = f2bf4(fmaxf(c[0], 0.f), fmaxf(c[1], 0.f), fmaxf(c[2], 0.f), fmaxf(c[3], 0.f));
    a2[ob] = hb;
    if (KEEP) { z2[ob] = c; h2[ob] = hb; }
  }
  v4f o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) o = mfma(ld4(&L.w3[r * NH + kb * 16 + 4 * g]), a2[kb], o);
  o[0] += L.b3[0];
  o[1] += L.b3[1];
  return o;
}

// ---------------------------------------------------------------- moments
// Depth code of every node (leaves 24, internal nodes their tight depth).
__global__ void k_node_depth(const BHNode* __restrict__ nodes, const int32_t* __restrict__ Np,
                             uint8_t* __restrict__ depth) {
  const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < *Np) depth[p] = (uint8_t)(nodes[p].meta & 0xff);
}

// Per-node cell record for the features (FP32): {s, log2(m)/16, offset of
// the centre of mass from the cell centre / s (x, y)}, {central second
// moments per unit mass / s^2 (xx, yy, xy), 0}.
struct Cell {
  float4 a, b;
};

// Central second moments per unit mass (FP64) of the nodes of depth D:
// leaves (D = 24) sum their points, internal nodes merge their children
// (parallel-axis rule, children in order) computed by earlier launches.
__global__ void k_node_moments(const BHNode* __restrict__ nodes, const int32_t* __restrict__ Np,
                               const uint8_t* __restrict__ depth, int32_t D,
                               const BoxInfo* __restrict__ box, const float* __restrict__ xsx,
                               const float* __restrict__ xsy, double* __restrict__ mom,
                               Cell* __restrict__ cell) {
  const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *Np || depth[p] != D) return;
  const BHNode nd = nodes[p];
  double sxx = 0.0, syy = 0.0, sxy = 0.0;
  if (nd.meta >> 8) {
    const int32_t cnt = (int32_t)nd.mass;
    for (int32_t j = nd.first; j < nd.first + cnt; ++j) {
      const double dx = (double)xsx[j] - nd.cx, dy = (double)xsy[j] - nd.cy;
      sxx += dx * dx;
      syy += dy * dy;
      sxy += dx * dy;
    }
  } else {
    for (int32_t ch = p + 1; ch < nd.skip; ch = nodes[ch].skip) {
      const BHNode cn = nodes[ch];
      const double mc = cn.mass, dx = cn.cx - nd.cx, dy = cn.cy - nd.cy;
      const double* cm = mom + 3 * (int64_t)ch;
      sxx += mc * (cm[0] + dx * dx);
      syy += mc * (cm[1] + dy * dy);
      sxy += mc * (cm[2] + dx * dy);
    }
  }
  const double m = nd.mass;
  sxx /= m;
  syy /= m;
  sxy /= m;
  double* o = mom + 3 * (int64_t)p;
  o[0] = sxx;
  o[1] = syy;
  o[2] = sxy;
  // cell geometry; the box scale is a power of two, so these are exact
  const BoxInfo bx = *box;
  const double inv_scale = 1.0 / bx.scale;
  const double S = (double)(1u << (24 - D));
  const double s = S * inv_scale, is = 1.0 / s;
  const double gx = bx.xmin + ((double)nd.ox + 0.5 * S) * inv_scale;
  const double gy = bx.ymin + ((double)nd.oy + 0.5 * S) * inv_scale;
  Cell c;
  c.a = make_float4((float)s, log2f(nd.mass) * 0.0625f, (float)((nd.cx - gx) * is),
                    (float)((nd.cy - gy) * is));
  c.b = make_float4((float)(sxx * is * is), (float)(syy * is * is), (float)(sxy * is * is), 0.f);
  cell[p] = c;
}

// ---------------------------------------------------------------- features
struct Feat {
  float f[8];
  float kex, key;  // kappa e
};

// Features of (target at (xt, yt), cell nd with record c).  False when
// x_u == com.
__device__ inline bool cell_features(const BHNode& nd, const Cell& c, float xt, float yt,
                                     Feat& o) {
  const float dx = (float)((double)xt - nd.cx), dy = (float)((double)yt - nd.cy);
  const float d2 = dx * dx + dy * dy;
  if (!(d2 > 0.f)) return false;
  const float inv = __builtin_amdgcn_rsqf(d2);
  const float ex = dx * inv, ey = dy * inv, px = -ey, py = ex;
  const float mxx = c.b.x, myy = c.b.y, mxy = c.b.z;
  const float t = c.a.x * inv;
  o.f[0] = t;
  o.f[1] = c.a.z * ex + c.a.w * ey;
  o.f[2] = c.a.z * px + c.a.w * py;
  o.f[3] = ex * ex * mxx + 2.f * ex * ey * mxy + ey * ey * myy;
  o.f[4] = px * px * mxx + 2.f * px * py * mxy + py * py * myy;
  o.f[5] = ex * px * mxx + (ex * py + ey * px) * mxy + ey * py * myy;
  o.f[6] = c.a.y;
  o.f[7] = 0.f;
  const float kappa = nd.mass * t * t * inv;
  o.kex = kappa * ex;
  o.key = kappa * ey;
  return true;
}

// Opening test of the plain traversal in exact integers (qx2i = 2 i_u + 1):
// accept iff u is outside C and theta^2 |d|^2 > 4 S^2 (exact doubles).
__device__ inline bool open_test(const BHNode& nd, int32_t qx2i, int32_t qy2i, double theta2) {
  const int sh = 24 - (nd.meta & 0xff);
  const int32_t S = 1 << sh;
  const int32_t dxi = qx2i - (int32_t)(2u * nd.ox + (uint32_t)S);
  const int32_t dyi = qy2i - (int32_t)(2u * nd.oy + (uint32_t)S);
  if (abs(dxi) < S && abs(dyi) < S) return false;
  const double dxd = (double)dxi, dyd = (double)dyi;
  // 4 S^2 = 2^(2 sh + 2) from its exponent bits (exact)
  return theta2 * fma(dxd, dxd, dyd * dyd) > __hiloint2double((1023 + 2 * sh + 2) << 20, 0);
}

// ---------------------------------------------------------------- traversal
constexpr int TL_WAVES = 4;
constexpr int QCAP = 128;  // ring of queued (lane, cell) rows per wave
struct QRow {
  float f[8];
  float kex, key;
  int32_t lane, pad;
};

// Runs the MLP on rows [qh, qh + rows) of the ring (rows <= 64, wave-
// uniform) as up to four 16-row blocks interleaved layer by layer (their
// matrix-core chains are independent), then adds each row's correction to
// its lane, in queue order.
__device__ inline void flush_rows(const MlpLds& L, const QRow* ring, int qh, int rows,
                                  float& cfx, float& cfy) {
  // the weights are read from LDS here rather than held in registers across
  // the traversal (occupancy)
  asm volatile("" ::: "memory");
  const int l = lane_id(), r = l & 15, g = l >> 4;
  const int nb = (rows + 15) >> 4;
  v8s x[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    x[b] = v8s{0, 0, 0, 0, 0, 0, 0, 0};
    if (b < nb && g == 0 && 16 * b + r < rows) {
      const QRow& e = ring[(qh + 16 * b + r) & (QCAP - 1)];
      x[b] = cat8(f2bf4(e.f[0], e.f[1], e.f[2], e.f[3]), f2bf4(e.f[4], e.f[5], e.f[6], e.f[7]));
    }
  }
  v4f o[4];
  mlp_blocks32(L, x, nb, o);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (b >= nb) break;
    float ax = 0.f, ay = 0.f;
    int32_t tl = -1;
    if (g == 0 && 16 * b + r < rows) {
      const QRow& e = ring[(qh + 16 * b + r) & (QCAP - 1)];
      const float h0 = o[b][0], h1 = o[b][1];
      ax = h0 * e.kex - h1 * e.key;
      ay = h0 * e.key + h1 * e.kex;
      tl = e.lane;
    }
    const int m = min(16, rows - 16 * b);
    for (int j = 0; j < m; ++j) {
      const int32_t t = __builtin_amdgcn_readlane(tl, j);
      const float bx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ax), j));
      const float by = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ay), j));
      if (l == t) { cfx += bx; cfy += by; }
    }
  }
}

__global__ __launch_bounds__(64 * TL_WAVES) __attribute__((amdgpu_waves_per_eu(3))) void k_traverse_learned(
    const BHNode* __restrict__ nodes, const int32_t* __restrict__ Np,
    const Cell* __restrict__ cell, const float* __restrict__ xsx, const float* __restrict__ xsy,
    const uint2* __restrict__ ixy, const int32_t* __restrict__ order, int32_t n, double theta2,
    const float* __restrict__ wts, float2* __restrict__ F) {
  __shared__ __align__(16) MlpLds L;
  __shared__ __align__(16) QRow ring_all[TL_WAVES][QCAP];
  stage_weights(wts, L);
  __syncthreads();
  const int wv = threadIdx.x >> 6, l = lane_id();
  const int32_t wbase = (blockIdx.x * TL_WAVES + wv) * 64;
  if (wbase >= n) return;
  QRow* ring = ring_all[wv];
  const int32_t i = wbase + l;
  const int32_t N = *Np;
  const bool valid = i < n;
  const float xt = valid ? xsx[i] : 0.f, yt = valid ? xsy[i] : 0.f;
  const uint2 qt = valid ? ixy[i] : make_uint2(0, 0);
  const int32_t qx2i = 2 * (int32_t)qt.x + 1, qy2i = 2 * (int32_t)qt.y + 1;
  float fx = 0.f, fy = 0.f, cfx = 0.f, cfy = 0.f;
  int32_t next = valid ? 0 : 0x7fffffff;
  int qh = 0, qt_ = 0;  // ring head / tail (wave-uniform, monotonic)
  int32_t p = 0;
  while (p < N) {
    p = __builtin_amdgcn_readfirstlane(p);
    const BHNode nd = nodes[p];
    const bool act = (next == p);
    if (nd.meta >> 8) {
      const int32_t cnt = (int32_t)nd.mass;
      if (cnt == 1) {
        if (act && nd.first != i) rq_add(xt - (float)nd.cx, yt - (float)nd.cy, 0.f, 1.f, fx, fy);
      } else {
        for (int32_t j = nd.first; j < nd.first + cnt; ++j) {
          const float sx = xsx[j], sy = xsy[j];
          if (act && j != i) rq_add(xt - sx, yt - sy, 0.f, 1.f, fx, fy);
        }
      }
      if (act) next = nd.skip;
      p = wave_min(next);
    } else {
      bool opened = false, push = false;
      Feat ft;
      if (act) {
        if (open_test(nd, qx2i, qy2i, theta2)) {
          rq_add((float)((double)xt - nd.cx), (float)((double)yt - nd.cy), 0.f, nd.mass, fx, fy);
          push = cell_features(nd, cell[p], xt, yt, ft);
          next = nd.skip;
        } else {
          next = p + 1;
          opened = true;
        }
      }
      const uint64_t bal = __ballot(push);
      if (bal) {
        if (push) {
          QRow& e = ring[(qt_ + __popcll(bal & lanemask_lt())) & (QCAP - 1)];
#pragma unroll
          for (int j = 0; j < 8; ++j) e.f[j] = ft.f[j];
          e.kex = ft.kex;
          e.key = ft.key;
          e.lane = l;
        }
        qt_ += __popcll(bal);
        wave_lds_sync();
        if (qt_ - qh >= 64) {
          flush_rows(L, ring, qh, 64, cfx, cfy);
          qh += 64;
        }
        wave_lds_sync();
      }
      if (__any(opened)) p = p + 1;
      else p = wave_min(next);
    }
  }
  while (qt_ > qh) {
    flush_rows(L, ring, qh, min(64, qt_ - qh), cfx, cfy);
    qh += 64;
  }
  if (valid) F[order[i]] = make_float2(fx + cfx, fy + cfy);
}

// Training samples: the (target, cell) pairs the traversal accepts, with
// features, kappa e, and the exact residual of the cell in h units (FP64).
// COUNT: cnt[i] = accepted cells of sorted target i.  Otherwise rows are
// written from off[i] on (at most cap in total).
template <bool COUNT>
__global__ __launch_bounds__(64 * TL_WAVES) void k_far_samples(
    const BHNode* __restrict__ nodes, const int32_t* __restrict__ Np,
    const Cell* __restrict__ cell, const float* __restrict__ xsx, const float* __restrict__ xsy,
    const uint2* __restrict__ ixy, const int32_t* __restrict__ order, int32_t n, double theta2,
    int32_t* __restrict__ cnt,
    const int64_t* __restrict__ off, int64_t cap, int32_t* __restrict__ u_out,
    int32_t* __restrict__ node_out, float* __restrict__ feat, float* __restrict__ tgt,
    float* __restrict__ coef) {
  const int l = lane_id();
  const int32_t wbase = (blockIdx.x * TL_WAVES + (threadIdx.x >> 6)) * 64;
  if (wbase >= n) return;
  const int32_t i = wbase + l;
  const int32_t N = *Np;
  const bool valid = i < n;
  const float xt = valid ? xsx[i] : 0.f, yt = valid ? xsy[i] : 0.f;
  const uint2 qt = valid ? ixy[i] : make_uint2(0, 0);
  const int32_t qx2i = 2 * (int32_t)qt.x + 1, qy2i = 2 * (int32_t)qt.y + 1;
  int32_t next = valid ? 0 : 0x7fffffff;
  int32_t k = 0;
  const int64_t base = (!COUNT && valid) ? off[i] : 0;
  const int32_t u = valid ? order[i] : -1;
  int32_t p = 0;
  while (p < N) {
    p = __builtin_amdgcn_readfirstlane(p);
    const BHNode nd = nodes[p];
    const bool act = (next == p);
    if (nd.meta >> 8) {
      if (act) next = nd.skip;
      p = wave_min(next);
      continue;
    }
    bool opened = false, take = false;
    Feat ft;
    if (act) {
      if (open_test(nd, qx2i, qy2i, theta2)) {
        take = cell_features(nd, cell[p], xt, yt, ft);
        next = nd.skip;
      } else {
        next = p + 1;
        opened = true;
      }
    }
    if (!COUNT && __any(take)) {
      // exact sum over the cell's points (wave-uniform loop), FP64
      const double ux = xt, uy = yt;
      double sx = 0.0, sy = 0.0;
      const int32_t c = (int32_t)nd.mass;
      for (int32_t j = nd.first; j < nd.first + c; ++j) {
        const double ddx = ux - (double)xsx[j], ddy = uy - (double)xsy[j];
        const double d2 = ddx * ddx + ddy * ddy;
        if (take && d2 > 0.0) { sx += ddx / d2; sy += ddy / d2; }
      }
      if (take) {
        const int64_t row = base + k;
        if (row < cap) {
          const double dx = ux - nd.cx, dy = uy - nd.cy, d2 = dx * dx + dy * dy;
          const double d = sqrt(d2), ex = dx / d, ey = dy / d;
          const double t = (double)cell[p].a.x / d, kappa = (double)nd.mass * t * t / d;
          const double Rx = sx - (double)nd.mass * dx / d2, Ry = sy - (double)nd.mass * dy / d2;
          u_out[row] = u;
          node_out[row] = p;
#pragma unroll
          for (int j = 0; j < 8; ++j) feat[8 * row + j] = ft.f[j];
          tgt[2 * row] = (float)((Rx * ex + Ry * ey) / kappa);
          tgt[2 * row + 1] = (float)((-Rx * ey + Ry * ex) / kappa);
          coef[2 * row] = ft.kex;
          coef[2 * row + 1] = ft.key;
        }
      }
    }
    if (take) ++k;
    if (__any(opened)) p = p + 1;
    else p = wave_min(next);
  }
  if (COUNT && valid) cnt[i] = k;
}

// ---------------------------------------------------------------- MLP batches
constexpr int MW = 4;  // waves per block in the batch kernels

__device__ inline v4s feat_frag(const float* __restrict__ feat, int64_t row, bool ok) {
  const int g = lane_id() >> 4;
  v4s x = {0, 0, 0, 0};
  if (ok && g < 2) {
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = (short)f2bf(feat[8 * row + 4 * g + j]);
  }
  return x;
}

__global__ __launch_bounds__(64 * MW) void k_mlp_forward(const float* __restrict__ feat,
                                                          int64_t count,
                                                          const float* __restrict__ wts,
                                                          float* __restrict__ out) {
  __shared__ __align__(16) MlpLds L;
  stage_weights(wts, L);
  __syncthreads();
  const int l = lane_id(), r = l & 15;
  const int64_t nblk = (count + 15) / 16;
  for (int64_t b = (int64_t)blockIdx.x * MW + (threadIdx.x >> 6); b < nblk;
       b += (int64_t)gridDim.x * MW) {
    const int64_t row = b * 16 + r;
    v8s x = v8s{0, 0, 0, 0, 0, 0, 0, 0};
    if (l < 16 && row < count) {
      const float* f = feat + 8 * row;
      x = cat8(f2bf4(f[0], f[1], f[2], f[3]), f2bf4(f[4], f[5], f[6], f[7]));
    }
    v4f o[4];
    mlp_blocks32(L, &x, 1, o);
    if (l < 16 && row < count) {
      out[2 * row] = o[0][0];
      out[2 * row + 1] = o[0][1];
    }
  }
}

// Per-wave LDS scratch of the backward pass (rows x units, BF16).
struct BwdLds {
  uint16_t h1[16 * NH], h2[16 * NH], dz1[16 * NH], dz2[16 * NH];
  uint16_t x[16 * 16];
  float dh[16 * 2];
};

// Writes an accumulator-layout block (unit 4g+j of block ob, row r) as rows x units.
__device__ inline void put_rows(uint16_t* s, int ob, v4s v) {
  const int l = lane_id(), r = l & 15, g = l >> 4;
  *reinterpret_cast<v4s*>(&s[r * NH + ob * 16 + 4 * g]) = v;
}
// Fragment (row 4g+j, unit ob*16 + r) of a rows x units matrix: the A operand
// of X^T (units x rows) or the B operand of X (rows x units).
__device__ inline v4s get_cols(const uint16_t* s, int ld, int ob) {
  const int l = lane_id(), r = l & 15, g = l >> 4;
  v4s v;
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = (short)s[(4 * g + j) * ld + ob * 16 + r];
  return v;
}

// Loss L = 1/(2B) sum |h - y|^2 and its gradient for rows [b0, b0+B) (or
// rows drawn with SplitMix64 when state != 0).  Each wave handles RB blocks
// of 16 rows and writes its partial gradient (and partial loss) to
// part[wave * (NPARAM + 1) ...].
constexpr int RB = 4;
__global__ __launch_bounds__(64 * MW) void k_mlp_grad(
    const float* __restrict__ feat, const float* __restrict__ tgt, int64_t N, int64_t B,
    uint64_t state, const float* __restrict__ wts, float* __restrict__ part) {
  __shared__ __align__(16) MlpLds L;
  __shared__ __align__(16) BwdLds S_all[MW];
  stage_weights(wts, L);
  __syncthreads();
  const int wv = threadIdx.x >> 6, l = lane_id(), r = l & 15, g = l >> 4;
  BwdLds& S = S_all[wv];
  const int64_t gw = (int64_t)blockIdx.x * MW + wv;
  const float invB = 1.f / (float)B;
  v4f acc2[16], acc1[4], acc3[4];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc2[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) { acc1[t] = v4f{0.f, 0.f, 0.f, 0.f}; acc3[t] = acc1[t]; }
  float db1[16], db2[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) { db1[t] = 0.f; db2[t] = 0.f; }
  float db3a = 0.f, db3b = 0.f, loss = 0.f;

  for (int rb = 0; rb < RB; ++rb) {
    const int64_t b = (gw * RB + rb) * 16 + r;  // batch position of this lane's row
    const bool ok = b < B;
    int64_t row = 0;
    if (ok) row = state ? (int64_t)(sm64_at(state, (uint64_t)b) % (uint64_t)N) : b;
    const v4s x = feat_frag(feat, row, ok);
    v4f z1[4], z2[4];
    v4s h1[4], h2[4];
    const v4f o = mlp16<true>(L, x, z1, h1, z2, h2);
    // output gradient dh = (h - y) / B on lanes 0-15
    float dh0 = 0.f, dh1 = 0.f;
    if (g == 0 && ok) {
      const float e0 = o[0] - tgt[2 * row], e1 = o[1] - tgt[2 * row + 1];
      loss += 0.5f * (e0 * e0 + e1 * e1);
      dh0 = e0 * invB;
      dh1 = e1 * invB;
    }
    db3a += dh0;
    db3b += dh1;
    // dH2^T = W3^T dh^T (K = output units, padded to 16)
    v4s bdh = {0, 0, 0, 0};
    if (g == 0) { bdh[0] = (short)f2bf(dh0); bdh[1] = (short)f2bf(dh1); }
    v4s dz2b[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      v4s a = {0, 0, 0, 0};
      if (g == 0) {
        a[0] = (short)L.w3[0 * NH + ob * 16 + r];
        a[1] = (short)L.w3[1 * NH + ob * 16 + r];
      }
      v4f c = {0.f, 0.f, 0.f, 0.f};
      c = mfma(a, bdh, c);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float dz = z2[ob][j] > 0.f ? c[j] : 0.f;
        db2[ob * 4 + j] += dz;
        dz2b[ob][j] = (short)f2bf(dz);
      }
    }
    // dH1^T = W2^T dZ2^T (K = layer-2 units)
    v4s dz1b[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      v4f c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        v4s a;
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = (short)L.w2[(kb * 16 + 4 * g + j) * NH + ob * 16 + r];
        c = mfma(a, dz2b[kb], c);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float dz = z1[ob][j] > 0.f ? c[j] : 0.f;
        db1[ob * 4 + j] += dz;
        dz1b[ob][j] = (short)f2bf(dz);
      }
    }
    // stage rows x units copies for the weight-gradient products (K = rows)
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      put_rows(S.h1, ob, h1[ob]);
      put_rows(S.h2, ob, h2[ob]);
      put_rows(S.dz1, ob, dz1b[ob]);
      put_rows(S.dz2, ob, dz2b[ob]);
    }
    if (g < 2) {
      // features as rows x 16
      *reinterpret_cast<v4s*>(&S.x[r * 16 + 4 * g]) = x;
    } else {
      *reinterpret_cast<v4s*>(&S.x[r * 16 + 4 * g]) = v4s{0, 0, 0, 0};
    }
    if (g == 0) { S.dh[2 * r] = dh0; S.dh[2 * r + 1] = dh1; }
    wave_lds_sync();
    // dW2 = dZ2^T H1, dW1 = dZ1^T X, dW3 = dh^T H2
    v4s bh1[4], bh2[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) { bh1[nb] = get_cols(S.h1, NH, nb); bh2[nb] = get_cols(S.h2, NH, nb); }
    const v4s bx = get_cols(S.x, 16, 0);
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      const v4s a2 = get_cols(S.dz2, NH, ob);
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc2[ob * 4 + nb] = mfma(a2, bh1[nb], acc2[ob * 4 + nb]);
      acc1[ob] = mfma(get_cols(S.dz1, NH, ob), bx, acc1[ob]);
    }
    v4s adh = {0, 0, 0, 0};
    if (r < 2) {
#pragma unroll
      for (int j = 0; j < 4; ++j) adh[j] = (short)f2bf(S.dh[2 * (4 * g + j) + r]);
    }
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc3[nb] = mfma(adh, bh2[nb], acc3[nb]);
    wave_lds_sync();
  }
  // bias sums over the 16 rows held by lanes with the same g
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    db1[t] = group_sum(db1[t], 16);
    db2[t] = group_sum(db2[t], 16);
  }
  db3a = group_sum(db3a, 16);
  db3b = group_sum(db3b, 16);
  loss = wave_sum(loss);
  float* P = part + gw * (NPARAM + 1);
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        P[OFF_W2 + (ob * 16 + 4 * g + j) * NH + nb * 16 + r] = acc2[ob * 4 + nb][j];
    if (r < NIN) {
#pragma unroll
      for (int j = 0; j < 4; ++j) P[OFF_W1 + (ob * 16 + 4 * g + j) * NIN + r] = acc1[ob][j];
    }
    if (g == 0) {
#pragma unroll
      for (int j = 0; j < NOUT; ++j) P[OFF_W3 + j * NH + ob * 16 + r] = acc3[ob][j];
    }
    if (r == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        P[OFF_B1 + ob * 16 + 4 * g + j] = db1[ob * 4 + j];
        P[OFF_B2 + ob * 16 + 4 * g + j] = db2[ob * 4 + j];
      }
    }
  }
  if (l == 0) {
    P[OFF_B3] = db3a;
    P[OFF_B3 + 1] = db3b;
    P[NPARAM] = loss;
  }
}

// Sums the per-wave partials in wave order; optionally applies one Adam step
// (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) to the FP32 weights.
// The step is evaluated in FP64 (0.999 has no FP32 value: 0.999f would make
// the second moment's weight 1 - beta2 off by 1.3e-5 relative) and the
// moments and weights are stored in FP32.
__global__ void k_mlp_reduce(const float* __restrict__ part, int32_t nw, float* __restrict__ grad,
                             float* __restrict__ loss_out, float* __restrict__ w,
                             float* __restrict__ am, float* __restrict__ av, int32_t t, double lr,
                             float invB) {
  const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > NPARAM) return;
  double s = 0.0;
  for (int32_t k = 0; k < nw; ++k) s += part[(int64_t)k * (NPARAM + 1) + p];
  if (p == NPARAM) {
    if (loss_out) *loss_out = (float)(s * invB);
    return;
  }
  const float gp = (float)s;
  if (grad) grad[p] = gp;
  if (w) {
    const double b1 = 0.9, b2 = 0.999, g = (double)gp;
    const double m = b1 * (double)am[p] + (1.0 - b1) * g;
    const double v = b2 * (double)av[p] + (1.0 - b2) * g * g;
    am[p] = (float)m;
    av[p] = (float)v;
    const double mh = m / (1.0 - pow(b1, (double)t)), vh = v / (1.0 - pow(b2, (double)t));
    w[p] = (float)((double)w[p] - lr * mh / (sqrt(vh) + 1e-8));
  }
}

// Initial weights (one thread per parameter), as mlp_init describes.
__global__ void k_mlp_init(uint64_t state, float out_scale, float* __restrict__ w) {
  const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  float sd = 0.f;  // biases stay 0
  if (p >= OFF_W1 && p < OFF_B1) sd = sqrtf(2.f / (float)NIN);
  else if (p >= OFF_W2 && p < OFF_B2) sd = sqrtf(2.f / (float)NH);
  else if (p >= OFF_W3 && p < OFF_B3) sd = out_scale / sqrtf((float)NH);
  // Box-Muller: u1 in (0, 1] from the top 24 bits, u2 in [0, 1)
  const float u1 = (float)((sm64_at(state, 2 * (uint64_t)p) >> 40) + 1) * 0x1p-24f;
  const float u2 = (float)(sm64_at(state, 2 * (uint64_t)p + 1) >> 40) * 0x1p-24f;
  const float z = sqrtf(-2.f * logf(u1)) * cospif(2.f * u2);
  w[p] = sd * z;
}

inline int32_t grad_waves(int64_t B) { return (int32_t)((B + 16 * RB - 1) / (16 * RB)); }

hipError_t tree_moments(BHWork* w, int32_t n, hipStream_t s) {
  const size_t NMAX = 2 * (size_t)n;
  MM_TRY(ensure<double>(w->mom, 3 * NMAX, s));
  MM_TRY(ensure<Cell>(w->cell, NMAX, s));
  MM_TRY(ensure<uint8_t>(w->ndepth, NMAX, s));
  const int32_t* Np = w->counter.as<int32_t>();
  const int nb = (int)((NMAX + 255) / 256);
  k_node_depth<<<nb, 256, 0, s>>>(w->nodes.as<BHNode>(), Np, w->ndepth.as<uint8_t>());
  for (int32_t D = 24; D >= 0; --D)
    k_node_moments<<<nb, 256, 0, s>>>(w->nodes.as<BHNode>(), Np, w->ndepth.as<uint8_t>(), D,
                                      w->box.as<BoxInfo>(), w->xsx.as<float>(), w->xsy.as<float>(),
                                      w->mom.as<double>(), w->cell.as<Cell>());
  return hipGetLastError();
}

}  // namespace

hipError_t farfield_learned(BHWork* w, int32_t n, const float* xy, double theta, const float* wts,
                            float* F, hipStream_t s) {
  MM_TRY(bh_build_tree(w, n, xy, nullptr, s));
  MM_TRY(tree_moments(w, n, s));
  const int32_t nw = (n + 63) / 64;
  k_traverse_learned<<<(nw + TL_WAVES - 1) / TL_WAVES, 64 * TL_WAVES, 0, s>>>(
      w->nodes.as<BHNode>(), w->counter.as<int32_t>(), w->cell.as<Cell>(), w->xsx.as<float>(),
      w->xsy.as<float>(), w->ix.as<uint2>(), w->order.as<int32_t>(), n, theta * theta, wts,
      (float2*)F);
  return hipGetLastError();
}

hipError_t far_samples(BHWork* w, int32_t n, const float* xy, double theta, int64_t cap,
                       int32_t* u_out, int32_t* node_out, float* feat, float* tgt, float* coef,
                       int64_t* count_host, hipStream_t s) {
  MM_TRY(bh_build_tree(w, n, xy, nullptr, s));
  MM_TRY(tree_moments(w, n, s));
  MM_TRY(ensure<int32_t>(w->scount, n, s));
  MM_TRY(ensure<int64_t>(w->soff, (size_t)n + 1, s));
  const int32_t nw = (n + 63) / 64, nb = (nw + TL_WAVES - 1) / TL_WAVES;
  const BHNode* nodes = w->nodes.as<BHNode>();
  const int32_t* Np = w->counter.as<int32_t>();
  k_far_samples<true><<<nb, 64 * TL_WAVES, 0, s>>>(
      nodes, Np, w->cell.as<Cell>(), w->xsx.as<float>(), w->xsy.as<float>(), w->ix.as<uint2>(),
      w->order.as<int32_t>(), n, theta * theta, w->scount.as<int32_t>(), nullptr, 0, nullptr,
      nullptr, nullptr, nullptr, nullptr);
  MM_TRY(hipGetLastError());
  MM_TRY(scan_excl_i32(w->scount.as<int32_t>(), w->soff.as<int64_t>(), n, s));
  int64_t total = 0;
  MM_TRY(hipMemcpyAsync(&total, w->soff.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  *count_host = total;
  if (cap > 0 && total > 0) {
    k_far_samples<false><<<nb, 64 * TL_WAVES, 0, s>>>(
        nodes, Np, w->cell.as<Cell>(), w->xsx.as<float>(), w->xsy.as<float>(), w->ix.as<uint2>(),
        w->order.as<int32_t>(), n, theta * theta, nullptr, w->soff.as<int64_t>(), cap, u_out,
        node_out, feat, tgt, coef);
    MM_TRY(hipGetLastError());
  }
  return hipSuccess;
}

hipError_t mlp_forward(int64_t count, const float* feat, const float* wts, float* out,
                       hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t nblk = (count + 15) / 16;
  const int64_t grid = std::min<int64_t>((nblk + MW - 1) / MW, 4096);
  k_mlp_forward<<<(int)grid, 64 * MW, 0, s>>>(feat, count, wts, out);
  return hipGetLastError();
}

hipError_t mlp_grad(int64_t count, const float* feat, const float* tgt, const float* wts,
                    float* grad, float* loss_dev, hipStream_t s) {
  const int32_t nw = grad_waves(count);
  const int32_t nwp = (nw + MW - 1) / MW * MW;
  DevBuf part;
  MM_TRY(part.alloc(sizeof(float) * (size_t)nwp * (NPARAM + 1), s));
  k_mlp_grad<<<nwp / MW, 64 * MW, 0, s>>>(feat, tgt, count, count, 0, wts, part.as<float>());
  MM_TRY(hipGetLastError());
  k_mlp_reduce<<<(NPARAM + 256) / 256, 256, 0, s>>>(part.as<float>(), nwp, grad, loss_dev,
                                                    nullptr, nullptr, nullptr, 0, 0.0,
                                                    1.f / (float)count);
  return hipGetLastError();
}

hipError_t mlp_init(uint64_t seed, double out_scale, float* wts, hipStream_t s) {
  k_mlp_init<<<(NPARAM + 255) / 256, 256, 0, s>>>(rng_stream(seed, 0, 65), (float)out_scale, wts);
  return hipGetLastError();
}

hipError_t mlp_train(int64_t N, const float* feat, const float* tgt, float* wts, float* adam,
                     int32_t steps, int32_t batch, double lr, uint64_t seed, int32_t step0,
                     float* losses, hipStream_t s) {
  const int32_t nw = grad_waves(batch);
  const int32_t nwp = (nw + MW - 1) / MW * MW;
  DevBuf part;
  MM_TRY(part.alloc(sizeof(float) * (size_t)nwp * (NPARAM + 1), s));
  for (int32_t it = 0; it < steps; ++it) {
    const int32_t t = step0 + it + 1;
    uint64_t state = rng_stream(seed, (uint32_t)t, 64);
    if (state == 0) state = 1;  // 0 would mean "rows in order"
    k_mlp_grad<<<nwp / MW, 64 * MW, 0, s>>>(feat, tgt, N, batch, state, wts, part.as<float>());
    k_mlp_reduce<<<(NPARAM + 256) / 256, 256, 0, s>>>(part.as<float>(), nwp, nullptr,
                                                      losses ? losses + it : nullptr, wts, adam,
                                                      adam + NPARAM, t, lr,
                                                      1.f / (float)batch);
  }
  return hipGetLastError();
}

}  // namespace mm
