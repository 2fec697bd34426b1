// Tile-major stress sets and the LDS-tiled Jacobi sweep (Eq. 2).
//
// The k-hop sets are a sparse n x n pattern whose columns are gathered
// (x_v) for every entry.  When rows are long, a row-at-a-time sweep is bound
// by the L2 traffic of those random 8-byte gathers.  Here the columns are cut
// into tiles of T = 2^tbits vertices; the coordinates (and sqrt c) of one
// tile are staged in LDS and every (row, tile) chunk of the sets is swept
// against them.  Entries are stored tile-major, 16 bits each:
// ((v - tile * T) << 3) | hop, so hop <= 7 and T <= 2^13; the local id
// indexes the staged tile, and the hop a small table of 1/hop and the bias
// added to D^2 (hop 0 marks padding: bias +inf makes 1/D = 0, so all of a
// padding entry's terms are exactly 0).
//
// Per chunk the partial sum  P = sum w (x_v + d (x_u - x_v)/D) - alpha sum r_q(u,v)
// is written to a row-major slot; the combine kernel adds a row's slots in
// tile order and forms x'_u = (P + alpha F_u) / rho_u (fixed order: the
// result is run-to-run identical).  rho_u = sum_{S(u)} w_uv is computed once
// per level from the canonical sets.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

constexpr int TB_WAVES = 4;          // waves per block of the conversion kernels
constexpr int TB_MAXTILES = 4096;    // conversion keeps per-tile counters in LDS
constexpr int TB_MAXW = TB_MAXTILES / 32;
constexpr int TS_T = 512;            // sweep block
constexpr int32_t UNIT_CH = 768;      // chunks per work unit (metadata staged in LDS)

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// wave inclusive max-scan
__device__ inline int32_t wave_incl_max(int32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int32_t w = __shfl_up(v, o, 64);
    if (l >= o) v = max(v, w);
  }
  return v;
}

// K1: number of distinct tiles per row
// Distinct tiles per row (the row's chunk count); with RHO also
// rho_u = sum over S(u) of w_uv in exactly k_rho's order (per hop segment,
// lane-strided, then a wave sum), so both give the same bits.
template <bool RHO>
__global__ __launch_bounds__(64 * TB_WAVES) void k_row_tiles(
    int32_t n, int32_t k, int32_t tbits, int32_t ntw, const int64_t* __restrict__ off,
    const int32_t* __restrict__ hend, const int32_t* __restrict__ nbr,
    const float* __restrict__ sqrtc, float scale, int32_t* __restrict__ nch,
    float* __restrict__ rho) {
  __shared__ uint32_t tbm[TB_WAVES][TB_MAXW];
  const int w = threadIdx.x >> 6, l = lane_id();
  const int32_t u = blockIdx.x * TB_WAVES + w;
  if (u >= n) return;
  uint32_t* bm = tbm[w];
  for (int i = l; i < ntw; i += 64) bm[i] = 0u;
  wave_sync();
  const int64_t beg = off[u];
  const float su = (RHO && sqrtc) ? sqrtc[u] : 0.f;
  float r = 0.f;
  int32_t seg0 = 0;
  for (int h = 1; h <= k; ++h) {
    const int32_t seg1 = hend[(int64_t)u * k + h - 1];
    for (int32_t i = seg0 + l; i < seg1; i += 64) {
      const int32_t v = nbr[beg + i];
      const int32_t t = v >> tbits;
      const uint32_t bit = 1u << (t & 31);
      if (!(bm[t >> 5] & bit)) atomicOr(&bm[t >> 5], bit);
      if (RHO && sqrtc) {
        const float d = (float)h * (su + sqrtc[v]) * scale;
        r += 1.f / (d * d);
      }
    }
    seg0 = seg1;
  }
  wave_sync();
  int32_t c = 0;
  for (int i = l; i < ntw; i += 64) c += __popc(bm[i]);
  c = wave_sum(c);
  if (l == 0) nch[u] = c;
  if (RHO) {
    if (sqrtc) {
      r = wave_sum(r);
      if (l == 0) rho[u] = r;
    } else if (l == 0) {
      int32_t prev = 0;
      float rr = 0.f;
      for (int h = 1; h <= k; ++h) {
        const int32_t e = hend[(int64_t)u * k + h - 1];
        rr += (float)(e - prev) / (float)(h * h);
        prev = e;
      }
      rho[u] = rr;
    }
  }
}

// K3 / K6: per row, per tile runs.  FILL=false: chunk sizes (row-major
// slots).  FILL=true: write the 16-bit entries; with BASE the start of every
// touched tile's chunk is looked up once per row (an LDS table of int64) so
// that the entry loop has no dependent global loads.  The row's entries are
// loaded one 64-entry step ahead.
template <bool FILL, bool BASE>
__global__ __launch_bounds__(64 * TB_WAVES) void k_row_chunks(
    int32_t n, int32_t k, int32_t tbits, int32_t ntiles, int32_t ntw,
    const int64_t* __restrict__ off, const int32_t* __restrict__ hend,
    const int32_t* __restrict__ nbr, const int64_t* __restrict__ rc_ptr,
    int32_t* __restrict__ cm_tile, int32_t* __restrict__ cm_size, int32_t* __restrict__ cm_row,
    const int32_t* __restrict__ pos_of_slot, const int64_t* __restrict__ chunk_off,
    uint16_t* __restrict__ ent) {
  // per wave, sized by the tile count: tile bitmap (ntw words), its popcount
  // prefix (ntw), per-tile counters (ntiles), with BASE the chunk starts
  // (ntiles int64, 8-byte aligned)
  extern __shared__ uint32_t tb_dyn[];
  const int w = threadIdx.x >> 6, l = lane_id();
  const int32_t u = blockIdx.x * TB_WAVES + w;
  if (u >= n) return;
  const size_t per = ((2 * (size_t)ntw + (size_t)ntiles + 1) & ~(size_t)1) +
                     (BASE ? 2 * (size_t)ntiles : 0);
  uint32_t* bm = tb_dyn + (size_t)w * per;
  int32_t* pf = reinterpret_cast<int32_t*>(bm + ntw);
  int32_t* ct = pf + ntw;
  int64_t* base = BASE ? reinterpret_cast<int64_t*>(bm + ((2 * (size_t)ntw + (size_t)ntiles + 1) &
                                                          ~(size_t)1))
                       : nullptr;
  const int64_t beg = off[u], endr = off[u + 1];
  for (int i = l; i < ntw; i += 64) bm[i] = 0u;
  wave_sync();
  {
    int32_t vn = beg + l < endr ? nbr[beg + l] : 0;
    for (int64_t e = beg + l; e < endr; e += 64) {
      const int32_t v = vn;
      if (e + 64 < endr) vn = nbr[e + 64];
      const int32_t t = v >> tbits;
      const uint32_t bit = 1u << (t & 31);
      if (!(bm[t >> 5] & bit)) atomicOr(&bm[t >> 5], bit);
    }
  }
  wave_sync();
  // zero the counters of touched tiles; popcount prefix over words
  for (int i = l; i < ntw; i += 64) {
    uint32_t b = bm[i];
    while (b) { int j = __ffs(b) - 1; b &= b - 1; ct[(i << 5) + j] = 0; }
  }
  if (l == 0) {
    int32_t run = 0;
    for (int i = 0; i < ntw; ++i) { pf[i] = run; run += __popc(bm[i]); }
  }
  wave_sync();
  const int64_t rbase = rc_ptr[u];
  if (FILL && BASE) {
    for (int i = l; i < ntw; i += 64) {
      uint32_t b = bm[i];
      int32_t rank = pf[i];
      while (b) {
        const int j = __ffs(b) - 1;
        b &= b - 1;
        base[(i << 5) + j] = chunk_off[pos_of_slot[rbase + rank]];
        rank++;
      }
    }
    wave_sync();
  }
  int32_t seg0 = 0;
  for (int h = 1; h <= k; ++h) {
    const int32_t seg1 = hend[(int64_t)u * k + h - 1];
    int32_t vn = seg0 + l < seg1 ? nbr[beg + seg0 + l] : 0;
    for (int32_t b = seg0; b < seg1; b += 64) {
      const int32_t i = b + l;
      const bool valid = i < seg1;
      const int32_t v = vn;
      if (i + 64 < seg1) vn = nbr[beg + i + 64];
      const int32_t t = valid ? (v >> tbits) : 0x7fffffff;
      const int32_t tprev = __shfl_up(t, 1, 64);
      const bool start = valid && (l == 0 || tprev != t);
      const int32_t rs = wave_incl_max(start ? l : -1);
      const int32_t tnext = __shfl_down(t, 1, 64);
      const bool end = valid && (l == 63 || i + 1 >= seg1 || tnext != t);
      if (FILL && valid) {
        int64_t cbase;
        if (BASE) {
          cbase = base[t];
        } else {
          const int32_t rank = pf[t >> 5] + __popc(bm[t >> 5] & ((1u << (t & 31)) - 1u));
          cbase = chunk_off[pos_of_slot[rbase + rank]];
        }
        const int64_t dst = cbase + ct[t] + (l - rs);
        ent[dst] = (uint16_t)(((v & ((1 << tbits) - 1)) << 3) | h);
      }
      wave_sync();
      if (end) ct[t] += l - rs + 1;
      wave_sync();
    }
    seg0 = seg1;
  }
  if (!FILL) {
    for (int i = l; i < ntw; i += 64) {
      uint32_t bb = bm[i];
      int32_t r = pf[i];
      while (bb) {
        int j = __ffs(bb) - 1;
        bb &= bb - 1;
        const int32_t t = (i << 5) + j;
        cm_tile[rbase + r] = t;
        cm_size[rbase + r] = ct[t];
        cm_row[rbase + r] = u;
        r++;
      }
    }
  }
}

__global__ void k_gather_sorted_chunks(int64_t m, const int32_t* __restrict__ svals,
                                       const int32_t* __restrict__ cm_size,
                                       const int32_t* __restrict__ cm_row,
                                       int32_t* __restrict__ ssize, int32_t* __restrict__ chunk_row,
                                       int32_t* __restrict__ pos_of_slot) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  const int32_t s = svals[c];
  ssize[c] = (cm_size[s] + 7) & ~7;  // chunks padded to 16-byte blocks (hop 0 = padding)
  chunk_row[c] = cm_row[s];
  pos_of_slot[s] = (int32_t)c;
}

__global__ void k_chunk_keys(int64_t m, const int32_t* __restrict__ cm_tile,
                             const int32_t* __restrict__ cm_size, uint64_t* __restrict__ keys) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  keys[c] = ((uint64_t)(uint32_t)cm_tile[c] << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)cm_size[c]);
}
__global__ void k_tile_first(int64_t m, const uint64_t* __restrict__ skey,
                             int32_t* __restrict__ tile_first) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  const uint32_t t = (uint32_t)(skey[c] >> 32);
  if (c == 0 || (uint32_t)(skey[c - 1] >> 32) != t) tile_first[t] = (int32_t)c;
}
// unit starts: the first chunk of a tile, every UNIT_CH-th chunk after it,
// and every chunk that begins a new span of emax entries (so that levels with
// few, long chunks still give enough work units to fill the chip)
__global__ void k_unit_flags(int64_t m, const uint64_t* __restrict__ skey,
                             const int32_t* __restrict__ tile_first,
                             const int64_t* __restrict__ chunk_off, int64_t emax,
                             int32_t* __restrict__ flag) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  const int64_t tf = tile_first[skey[c] >> 32];
  flag[c] = ((c - tf) % UNIT_CH == 0 || (c > tf && chunk_off[c] / emax != chunk_off[c - 1] / emax))
                ? 1 : 0;
}
__global__ void k_unit_fill(int64_t m, const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
                           const uint64_t* __restrict__ skey, int32_t* __restrict__ unit_c0,
                           int32_t* __restrict__ unit_tile) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m || !flag[c]) return;
  unit_c0[pos[c]] = (int32_t)c;
  unit_tile[pos[c]] = (int32_t)(skey[c] >> 32);
}
__global__ void k_set_i32(int32_t* p, int32_t v) { *p = v; }

// rho_u = sum over S(u) of w_uv (canonical sets)
__global__ void k_rho(int32_t n, int32_t k, const int64_t* __restrict__ off,
                      const int32_t* __restrict__ hend, const int32_t* __restrict__ nbr,
                      const float* __restrict__ sqrtc, float scale, float* __restrict__ rho) {
  const int w = threadIdx.x >> 6, l = lane_id();
  const int32_t u = blockIdx.x * (blockDim.x >> 6) + w;
  if (u >= n) return;
  float r = 0.f;
  if (!sqrtc) {
    if (l == 0) {
      int32_t prev = 0;
      for (int h = 1; h <= k; ++h) {
        const int32_t e = hend[(int64_t)u * k + h - 1];
        r += (float)(e - prev) / (float)(h * h);
        prev = e;
      }
      rho[u] = r;
    }
    return;
  }
  const int64_t beg = off[u];
  const float su = sqrtc[u];
  int32_t seg0 = 0;
  for (int h = 1; h <= k; ++h) {
    const int32_t seg1 = hend[(int64_t)u * k + h - 1];
    for (int32_t i = seg0 + l; i < seg1; i += 64) {
      const float d = (float)h * (su + sqrtc[nbr[beg + i]]) * scale;
      r += 1.f / (d * d);
    }
    seg0 = seg1;
  }
  r = wave_sum(r);
  if (l == 0) rho[u] = r;
}

// ---- the tiled sweep
//
// One workgroup per work unit (<= UNIT_CH chunks of one tile).  Prologue:
// the tile's coordinates (and sqrt c) and the unit's chunk metadata (first
// block, slot, x_u) are staged in LDS.  Then each group of G lanes streams
// chunks gi, gi + NG, ...: per step a lane takes NB 16-byte blocks (8
// entries each) G blocks apart, so the group covers NB * G consecutive
// blocks of its chunk.  The only global loads in the loop are the entry
// blocks of the lane's next step, issued unconditionally (clamped address)
// before the current blocks are computed, so their latency overlaps one step
// of work.  A lane visits its blocks in the same order for every NB, so NB
// changes only how many bytes are in flight, not the result.
template <int G, int NB, bool COARSE, bool Q0>
__global__ __launch_bounds__(TS_T) void k_sweep_tiled(
    int32_t n, int32_t tbits, const int32_t* __restrict__ unit_c0,
    const int32_t* __restrict__ unit_tile, const int64_t* __restrict__ chunk_off,
    const int32_t* __restrict__ chunk_row, const int32_t* __restrict__ chunk_slot,
    const uint16_t* __restrict__ ent, const float2* __restrict__ xy,
    const float* __restrict__ sqrtc, float scale, float alpha, float q,
    float2* __restrict__ partial, const float* __restrict__ alpha_dev) {
  extern __shared__ float2 sx[];
  // per hop h: (1/h, bias added to D^2); h = 0 marks padding: (0, +inf), so a
  // padding entry gets 1/D = 0 and every one of its terms is exactly 0
  __shared__ float2 lut[16];
  __shared__ int32_t mblk[UNIT_CH + 1];   // first block of each chunk (absolute)
  __shared__ int32_t mslot[UNIT_CH];
  __shared__ float2 mxu[UNIT_CH];
  __shared__ float mscu[COARSE ? UNIT_CH : 1];
  const int32_t T = 1 << tbits;
  float* ssc = reinterpret_cast<float*>(sx + T);
  const int32_t tile = unit_tile[blockIdx.x];
  const int32_t c0 = unit_c0[blockIdx.x], c1 = unit_c0[blockIdx.x + 1];
  const int32_t nch = c1 - c0;
  const int32_t v0 = tile * T;
  const int32_t nv = min(T, n - v0);
  for (int32_t i = threadIdx.x; i < nv; i += TS_T) {
    sx[i] = xy[v0 + i];
    if (COARSE) ssc[i] = sqrtc[v0 + i] * scale;
  }
  for (int32_t i = threadIdx.x; i <= nch; i += TS_T) {
    mblk[i] = (int32_t)(chunk_off[c0 + i] >> 3);
    if (i < nch) {
      const int32_t u = chunk_row[c0 + i];
      mslot[i] = chunk_slot[c0 + i];
      mxu[i] = xy[u];
      if (COARSE) mscu[i] = sqrtc[u] * scale;
    }
  }
  if (alpha_dev) alpha = *alpha_dev;
  if (threadIdx.x < 16) {
    // q = 0: a 1e-30 bias keeps 1/D finite for a coincident pair, whose
    // r-terms then vanish through dx = dy = 0; q != 0 tests D^2 > 0 instead
    const float h = (float)threadIdx.x;
    lut[threadIdx.x] = threadIdx.x ? make_float2(1.f / h, Q0 ? 1e-30f : 0.f)
                                   : make_float2(0.f, INFINITY);
  }
  __syncthreads();
  const int gl = threadIdx.x % G, gi = threadIdx.x / G;
  constexpr int NG = TS_T / G;
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const u32x4* __restrict__ ent4 = reinterpret_cast<const u32x4*>(ent);
  int32_t ci = gi;                      // chunk (relative to the unit)
  int32_t ae = ci < nch ? mblk[ci + 1] : 0;
  int32_t a = ci < nch ? mblk[ci] + gl : 0;
  u32x4 blk[NB];
  bool vb[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    vb[b] = ci < nch && a + b * G < ae;
    blk[b] = ent4[vb[b] ? a + b * G : 0];
  }
  float2 xu = ci < nch ? mxu[ci] : make_float2(0.f, 0.f);
  float scu = (COARSE && ci < nch) ? mscu[ci] : 0.f;
  float px = 0.f, py = 0.f;
  // one 16-byte block: decode the 8 entries, issue their LDS reads, then
  // compute (branch-free)
  auto run = [&](const u32x4 bk) {
    const uint32_t wv[4] = {bk.x, bk.y, bk.z, bk.w};
    float2 xv[8];
    float2 lw[8];
    float sc[8];
#pragma unroll
    for (int q2 = 0; q2 < 8; ++q2) {
      const uint32_t pk = (wv[q2 >> 1] >> (16 * (q2 & 1))) & 0xFFFFu;
      const uint32_t vl = pk >> 3;
      xv[q2] = sx[vl];
      lw[q2] = lut[pk & 7u];
      if (COARSE) sc[q2] = ssc[vl];
    }
#pragma unroll
    for (int q2 = 0; q2 < 8; ++q2) {
      const float dx = xu.x - xv[q2].x, dy = xu.y - xv[q2].y;
      const float D2 = fmaf(dx, dx, fmaf(dy, dy, lw[q2].y));
      // w d = 1/d with d = hop (finest level) or hop (sqrt c_u + sqrt c_v)
      // scale (coarse levels; the staged roots are pre-scaled), w = (w d)^2
      float wd = lw[q2].x;
      if (COARSE) wd *= __builtin_amdgcn_rcpf(scu + sc[q2]);
      const float w = wd * wd;
      float inv = __builtin_amdgcn_rsqf(D2);
      if (!Q0) inv = D2 > 0.f ? inv : 0.f;
      const float rq = Q0 ? 0.f : (D2 > 0.f ? powf(D2, -0.5f * (q + 2.f)) : 0.f);
      // w d / D - alpha / D^(q+2); zero for padding and coincident pairs
      const float coef = Q0 ? inv * fmaf(-alpha, inv, wd) : fmaf(wd, inv, -alpha * rq);
      px = fmaf(w, xv[q2].x, px);
      py = fmaf(w, xv[q2].y, py);
      px = fmaf(coef, dx, px);
      py = fmaf(coef, dy, py);
    }
  };
  for (;;) {
    const bool active = ci < nch;
    if (!__any(active)) break;
    // the group's next position: same chunk, or its next chunk if this step
    // finishes the current one (same decision for all lanes of the group)
    const bool sw = active && (a - gl + NB * G >= ae);
    int32_t a_nx = a + NB * G;
    int32_t ae_nx = ae;
    bool act_nx = active;
    if (sw) {
      const int32_t cn = ci + NG;
      if (cn < nch) {
        a_nx = mblk[cn] + gl;
        ae_nx = mblk[cn + 1];
      } else {
        act_nx = false;
      }
    }
    u32x4 nblk[NB];
    bool nvb[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      nvb[b] = act_nx && a_nx + b * G < ae_nx;
      nblk[b] = __builtin_nontemporal_load(&ent4[nvb[b] ? a_nx + b * G : 0]);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
      if (vb[b]) run(blk[b]);
    if (__any(sw)) {
      const float rx = group_sum(px, G), ry = group_sum(py, G);
      if (sw) {
        if (gl == 0) partial[mslot[ci]] = make_float2(rx, ry);
        px = 0.f;
        py = 0.f;
        ci += NG;
        if (ci < nch) {
          xu = mxu[ci];
          if (COARSE) scu = mscu[ci];
        }
      }
    }
    a = a_nx;
    ae = ae_nx;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      vb[b] = nvb[b];
      blk[b] = nblk[b];
    }
  }
}

constexpr int CB_T = 256;
constexpr int CB_G = 16;  // lanes per row in the combine
__global__ __launch_bounds__(CB_T) void k_combine(int32_t n, const int64_t* __restrict__ rc_ptr,
                                                  const float2* __restrict__ partial,
                                                  const float* __restrict__ rho,
                                                  const float2* __restrict__ xy,
                                                  const float2* __restrict__ F, float alpha,
                                                  float2* __restrict__ out,
                                                  double2* __restrict__ dpart,
                                                  const float* __restrict__ alpha_dev) {
  if (alpha_dev) alpha = *alpha_dev;
  constexpr int RPB = CB_T / CB_G;
  __shared__ double2 red[RPB];
  const int gl = threadIdx.x % CB_G, gi = threadIdx.x / CB_G;
  const int32_t u = blockIdx.x * RPB + gi;
  double2 dd = make_double2(0.0, 0.0);
  if (u < n) {
    float px = 0.f, py = 0.f;
    for (int64_t s = rc_ptr[u] + gl; s < rc_ptr[u + 1]; s += CB_G) {
      const float2 p = partial[s];
      px += p.x;
      py += p.y;
    }
    px = group_sum(px, CB_G);
    py = group_sum(py, CB_G);
    if (gl == 0) {
      const float2 fu = F[u], xu = xy[u];
      const float r = rho[u];
      float2 xn;
      xn.x = (px + alpha * fu.x) / r;
      xn.y = (py + alpha * fu.y) / r;
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
    dpart[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(1024) void k_sum_parts2(const double2* __restrict__ part, int32_t m,
                                                     double* __restrict__ out) {
  __shared__ double shx[1024], shy[1024];
  double sx = 0.0, sy = 0.0;
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

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

bool tiled_eligible(const KhopDev& kh, int32_t tbits) {
  const int64_t ntiles = ((int64_t)kh.n + (1 << tbits) - 1) >> tbits;
  // entries are (local id << 3) | hop: 3 hop bits, tbits + 3 <= 16
  return kh.k <= 7 && tbits <= 13 && ntiles <= TB_MAXTILES && kh.total > 0;
}

hipError_t compute_rho(const KhopDev& kh, const float* sqrtc, double scale, float* rho,
                       hipStream_t s) {
  k_rho<<<nblk(kh.n, 4), 256, 0, s>>>(kh.n, kh.k, kh.off, kh.hend, kh.nbr, sqrtc, (float)scale, rho);
  return hipGetLastError();
}

hipError_t tiled_build(const KhopDev& kh, int32_t tbits, double min_avg_chunk, TiledSet* ts,
                       hipStream_t s, const float* sqrtc, double scale, float* rho) {
  const int32_t n = kh.n;
  const int32_t ntiles = (int32_t)(((int64_t)n + (1 << tbits) - 1) >> tbits);
  const int32_t ntw = (ntiles + 31) >> 5;
  ts->n = n;
  ts->tbits = tbits;
  ts->ntiles = ntiles;
  DevBuf nch, cm_tile, cm_size, cm_row, skeys, svals, ssize, flag, upos;
  MM_TRY(nch.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(ts->b_rc_ptr.alloc(sizeof(int64_t) * (size_t)(n + 1), s));
  ts->rc_ptr = ts->b_rc_ptr.as<int64_t>();
  if (rho)
    k_row_tiles<true><<<nblk(n, TB_WAVES), 64 * TB_WAVES, 0, s>>>(
        n, kh.k, tbits, ntw, kh.off, kh.hend, kh.nbr, sqrtc, (float)scale, nch.as<int32_t>(), rho);
  else
    k_row_tiles<false><<<nblk(n, TB_WAVES), 64 * TB_WAVES, 0, s>>>(
        n, kh.k, tbits, ntw, kh.off, kh.hend, kh.nbr, nullptr, 1.f, nch.as<int32_t>(), nullptr);
  MM_TRY(hipGetLastError());
  MM_TRY(scan_excl_i32(nch.as<int32_t>(), ts->rc_ptr, n, s));
  int64_t m = 0;
  MM_TRY(hipMemcpyAsync(&m, ts->rc_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  if (m >= (1ll << 31)) return hipErrorInvalidValue;
  ts->nchunks = m;
  ts->avg_chunk = (double)kh.total / (double)std::max<int64_t>(m, 1);
  ts->built = false;
  if (ts->avg_chunk < min_avg_chunk) return hipSuccess;  // chunks too short to pay off
  MM_TRY(cm_tile.alloc(sizeof(int32_t) * (size_t)m, s));
  MM_TRY(cm_size.alloc(sizeof(int32_t) * (size_t)m, s));
  MM_TRY(cm_row.alloc(sizeof(int32_t) * (size_t)m, s));
  const size_t per_wave = (2 * (size_t)ntw + (size_t)ntiles + 1) & ~(size_t)1;
  const size_t tb_shm = sizeof(uint32_t) * (size_t)TB_WAVES * per_wave;
  // the fill pass keeps the chunk starts of a row's tiles in LDS when they fit
  const size_t tb_shm_base = sizeof(uint32_t) * (size_t)TB_WAVES * (per_wave + 2 * (size_t)ntiles);
  const bool use_base = tb_shm_base <= 65536;
  if (tb_shm > 65536) {
    MM_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_row_chunks<false, false>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)tb_shm));
    MM_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_row_chunks<true, false>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)tb_shm));
  }
  k_row_chunks<false, false><<<nblk(n, TB_WAVES), 64 * TB_WAVES, tb_shm, s>>>(
      n, kh.k, tbits, ntiles, ntw, kh.off, kh.hend, kh.nbr, ts->rc_ptr, cm_tile.as<int32_t>(),
      cm_size.as<int32_t>(), cm_row.as<int32_t>(), nullptr, nullptr, nullptr);
  MM_TRY(hipGetLastError());
  // order chunks by (tile, row): stable sort of row-major slots by tile
  MM_TRY(skeys.alloc(sizeof(uint64_t) * (size_t)m, s));
  MM_TRY(svals.alloc(sizeof(int32_t) * (size_t)m, s));
  MM_TRY(iota_i32(svals.as<int32_t>(), m, s));
  // chunks of a tile in descending size (stable: ties keep row order), so the
  // chunks of a work unit have similar sizes and its lane groups stay balanced
  k_chunk_keys<<<nblk(m), 256, 0, s>>>(m, cm_tile.as<int32_t>(), cm_size.as<int32_t>(),
                                       skeys.as<uint64_t>());
  int kbits = 1;
  while ((1 << kbits) < ntiles) kbits++;
  MM_TRY(radix_sort_pairs(skeys.as<uint64_t>(), svals.as<int32_t>(), m, 32 + kbits, s));
  MM_TRY(ssize.alloc(sizeof(int32_t) * (size_t)m, s));
  MM_TRY(ts->b_chunk_row.alloc(sizeof(int32_t) * (size_t)m, s));
  MM_TRY(ts->b_chunk_off.alloc(sizeof(int64_t) * (size_t)(m + 1), s));
  ts->chunk_row = ts->b_chunk_row.as<int32_t>();
  ts->chunk_off = ts->b_chunk_off.as<int64_t>();
  // pos_of_slot reuses cm_tile's storage after the sort
  int32_t* pos_of_slot = cm_tile.as<int32_t>();
  k_gather_sorted_chunks<<<nblk(m), 256, 0, s>>>(m, svals.as<int32_t>(), cm_size.as<int32_t>(),
                                                 cm_row.as<int32_t>(), ssize.as<int32_t>(),
                                                 ts->chunk_row, pos_of_slot);
  MM_TRY(scan_excl_i32(ssize.as<int32_t>(), ts->chunk_off, m, s));
  // chunk -> row-major slot
  MM_TRY(ts->b_chunk_slot.alloc(sizeof(int32_t) * (size_t)m, s));
  ts->chunk_slot = ts->b_chunk_slot.as<int32_t>();
  MM_TRY(hipMemcpyAsync(ts->chunk_slot, svals.p, sizeof(int32_t) * (size_t)m,
                        hipMemcpyDeviceToDevice, s));
  int64_t padded = 0;
  MM_TRY(hipMemcpyAsync(&padded, ts->chunk_off + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  if ((padded >> 3) >= (1ll << 31)) return hipSuccess;  // block ids are int32 in the sweep
  MM_TRY(ts->b_ent.alloc(sizeof(uint16_t) * (size_t)std::max<int64_t>(padded, 8), s));
  ts->ent = ts->b_ent.as<uint16_t>();
  MM_TRY(hipMemsetAsync(ts->ent, 0, sizeof(uint16_t) * (size_t)padded, s));
  ts->total = kh.total;
  ts->padded = padded;
  if (use_base)
    k_row_chunks<true, true><<<nblk(n, TB_WAVES), 64 * TB_WAVES, tb_shm_base, s>>>(
        n, kh.k, tbits, ntiles, ntw, kh.off, kh.hend, kh.nbr, ts->rc_ptr, nullptr, nullptr,
        nullptr, pos_of_slot, ts->chunk_off, ts->ent);
  else
    k_row_chunks<true, false><<<nblk(n, TB_WAVES), 64 * TB_WAVES, tb_shm, s>>>(
        n, kh.k, tbits, ntiles, ntw, kh.off, kh.hend, kh.nbr, ts->rc_ptr, nullptr, nullptr,
        nullptr, pos_of_slot, ts->chunk_off, ts->ent);
  MM_TRY(hipGetLastError());
  // work units
  MM_TRY(flag.alloc(sizeof(int32_t) * (size_t)m, s));
  MM_TRY(upos.alloc(sizeof(int64_t) * (size_t)(m + 1), s));
  {
    DevBuf tfirst;
    MM_TRY(tfirst.alloc(sizeof(int32_t) * (size_t)ntiles, s));
    k_tile_first<<<nblk(m), 256, 0, s>>>(m, skeys.as<uint64_t>(), tfirst.as<int32_t>());
    // at least ~8 work units per CU when the level is small; never fewer
    // than 64K entries per unit (the tile staging is amortised over them)
    const int64_t emax = std::max<int64_t>(65536, padded / 2048);
    k_unit_flags<<<nblk(m), 256, 0, s>>>(m, skeys.as<uint64_t>(), tfirst.as<int32_t>(),
                                         ts->chunk_off, emax, flag.as<int32_t>());
  }
  MM_TRY(scan_excl_i32(flag.as<int32_t>(), upos.as<int64_t>(), m, s));
  int64_t nu = 0;
  MM_TRY(hipMemcpyAsync(&nu, upos.as<int64_t>() + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  ts->nunits = (int32_t)nu;
  MM_TRY(ts->b_unit_c0.alloc(sizeof(int32_t) * (size_t)(nu + 1), s));
  MM_TRY(ts->b_unit_tile.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nu, 1), s));
  ts->unit_c0 = ts->b_unit_c0.as<int32_t>();
  ts->unit_tile = ts->b_unit_tile.as<int32_t>();
  k_unit_fill<<<nblk(m), 256, 0, s>>>(m, flag.as<int32_t>(), upos.as<int64_t>(), skeys.as<uint64_t>(),
                                      ts->unit_c0, ts->unit_tile);
  k_set_i32<<<1, 1, 0, s>>>(ts->unit_c0 + nu, (int32_t)m);
  MM_TRY(ts->b_partial.alloc(sizeof(float2) * (size_t)m, s));
  ts->built = true;
  return hipGetLastError();
}

hipError_t sweep_tiled(const TiledSet& ts, int32_t level, const float* sqrtc, double scale,
                       const float* rho, const float* xy, const float* F, double alpha, double q,
                       float* xy_out, double* delta2_dev, hipStream_t s, const float* alpha_dev,
                       int32_t group, int32_t nb) {
  const bool coarse = level > 0 && sqrtc != nullptr;
  const bool q0 = q == 0.0;
  const int32_t T = 1 << ts.tbits;
  const size_t shm = (size_t)T * (sizeof(float2) + (coarse ? sizeof(float) : 0));
  // a group of G lanes (one 8-entry block each per step) per chunk
  const int G = group > 0 ? group : tiled_group(ts);
  const int NB = nb > 0 ? nb : tiled_blocks(ts);
  float2* part = ts.b_partial.as<float2>();
#define MM_TS(GG, NBV, C, Q)                                                                     \
  do {                                                                                           \
    static bool attr_set = false; /* once per instantiation (not during a capture) */           \
    if (!attr_set) {                                                                             \
      MM_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_tiled<GG, NBV, C, Q>), \
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));         \
      attr_set = true;                                                                           \
    }                                                                                            \
    k_sweep_tiled<GG, NBV, C, Q><<<ts.nunits, TS_T, shm, s>>>(                                   \
        ts.n, ts.tbits, ts.unit_c0, ts.unit_tile, ts.chunk_off, ts.chunk_row, ts.chunk_slot,     \
        ts.ent, (const float2*)xy, sqrtc, (float)scale, (float)alpha, (float)q, part, alpha_dev); \
  } while (0)
#define MM_TSN(GG, NBV)                                                                  \
  do {                                                                                   \
    if (coarse) { if (q0) MM_TS(GG, NBV, true, true); else MM_TS(GG, NBV, true, false); } \
    else { if (q0) MM_TS(GG, NBV, false, true); else MM_TS(GG, NBV, false, false); }      \
  } while (0)
#define MM_TSG(GG)                                   \
  do {                                               \
    if (NB == 4) MM_TSN(GG, 4); else MM_TSN(GG, 2);  \
  } while (0)
  switch (G) {
    case 16: MM_TSG(16); break;
    case 8: MM_TSG(8); break;
    default: MM_TSG(4); break;
  }
#undef MM_TSG
#undef MM_TSN
#undef MM_TS
  MM_TRY(hipGetLastError());
  const int32_t ncb = (ts.n + CB_T / CB_G - 1) / (CB_T / CB_G);
  DevBuf& dpart = const_cast<TiledSet&>(ts).b_dpart;
  if (dpart.bytes < sizeof(double2) * (size_t)ncb) MM_TRY(dpart.alloc(sizeof(double2) * (size_t)ncb, s));
  k_combine<<<ncb, CB_T, 0, s>>>(ts.n, ts.rc_ptr, part, rho, (const float2*)xy, (const float2*)F,
                                (float)alpha, (float2*)xy_out, dpart.as<double2>(), alpha_dev);
  k_sum_parts2<<<1, 1024, 0, s>>>(dpart.as<double2>(), ncb, delta2_dev);
  return hipGetLastError();
}

}  // namespace mm
