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
// per level, with the tile-major copy itself, in tilemajor.hip.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

constexpr int TS_T = 512;            // sweep block
constexpr int32_t UNIT_CH = kUnitChunks;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte block of 8 entries of one chunk (row u, one tile): decode the
// entries, issue their LDS reads, then accumulate (branch-free) into (px, py)
// the sum over the entries of c (x_u - x_v) with
//   c = w d / D - alpha / D^(q+2) - w,   w = d^-2,
// i.e. Eq. 2's numerator minus rho_u x_u (the combine adds rho_u x_u back).
// sx: the tile's coordinates; ssc: sqrt c of the tile's vertices times the
// distance scale (coarse levels); lut: the per-hop table (hop_entry).
template <bool COARSE, bool Q0>
__device__ __forceinline__ void sweep_block(const u32x4 bk, const float2* __restrict__ sx,
                                            const float2* __restrict__ ssc,
                                            const float2* __restrict__ lut, const float2 xu,
                                            const float scu, const float alpha, const float q,
                                            float& px, float& py) {
  const uint32_t wv[4] = {bk.x, bk.y, bk.z, bk.w};
  float2 xv[8];
  float2 lw[8];
  float sc[8];
#pragma unroll
  for (int q2 = 0; q2 < 8; ++q2) {
    const uint32_t pk = (wv[q2 >> 1] >> (16 * (q2 & 1))) & 0xFFFFu;
    // byte offsets: id * 8 is the entry with its hop bits cleared, and
    // id * 4 half of that
    const uint32_t xo = pk & 0xFFF8u;
    xv[q2] = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(sx) + xo);
    lw[q2] = lut[pk & 7u];
    // sqrt c sits at the same 8-byte stride as the coordinates, so one
    // address register serves both reads (different immediate offsets)
    if (COARSE) sc[q2] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(ssc) + xo);
  }
  if (COARSE && Q0) {
    // coarse levels, q = 0: with g = h (sqrt c_u + sqrt c_v) scale = 1/wd and
    // r = 1/(g D) = wd/D, the coefficient is  r - r^2 (alpha g^2 + D^2)
    // (= wd/D - alpha/D^2 - wd^2): one reciprocal square root per entry.
    // The table holds (h, bias added to g^2 D^2): a tiny bias keeps r finite
    // for a coincident pair (whose offset is 0); +inf for padding gives
    // r = 0 and a zero coefficient.
#pragma unroll
    for (int q2 = 0; q2 < 8; ++q2) {
      const float dx = xu.x - xv[q2].x, dy = xu.y - xv[q2].y;
      const float D2 = fmaf(dx, dx, dy * dy);
      const float g = lw[q2].x * (scu + sc[q2]);
      const float g2 = g * g;
      const float r = __builtin_amdgcn_rsqf(fmaf(D2, g2, lw[q2].y));
      const float coef = fmaf(-(r * r), fmaf(alpha, g2, D2), r);
      px = fmaf(coef, dx, px);
      py = fmaf(coef, dy, py);
    }
    return;
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
    // w x_v = w x_u - w (x_u - x_v): the sums are taken relative to x_u, so
    // one coefficient multiplies the offset.  It is 0 for padding; for a
    // coincident pair it is finite and the offset is 0.
    const float coef = Q0 ? fmaf(inv, fmaf(-alpha, inv, wd), -w) : fmaf(wd, inv, fmaf(-alpha, rq, -w));
    px = fmaf(coef, dx, px);
    py = fmaf(coef, dy, py);
  }
}

// The per-hop table of the sweeps (index = hop; hop 0 marks padding).
// Finest level, or q != 0: (1/h, bias added to D^2), padding (0, +inf) so that
// 1/D = 0 and every term of a padding entry is exactly 0; at q = 0 a 1e-30
// bias keeps 1/D finite for a coincident pair, whose r-terms then vanish
// through dx = dy = 0 (q != 0 tests D^2 > 0 instead).  Coarse levels at
// q = 0: (h, bias added to g^2 D^2) as sweep_block describes.
template <bool COARSE, bool Q0>
__device__ inline float2 hop_entry(uint32_t h) {
  if (COARSE && Q0) return h ? make_float2((float)h, 1e-20f) : make_float2(1.f, INFINITY);
  return h ? make_float2(1.f / (float)h, Q0 ? 1e-30f : 0.f) : make_float2(0.f, INFINITY);
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
template <int G, int NB, int TB, bool COARSE, bool Q0>
__global__ __launch_bounds__(TS_T) void k_sweep_tiled(
    int32_t n, const int32_t* __restrict__ unit_c0,
    const int32_t* __restrict__ unit_tile, const int64_t* __restrict__ chunk_off,
    const int32_t* __restrict__ chunk_row, const int32_t* __restrict__ chunk_slot,
    const uint16_t* __restrict__ ent, const float2* __restrict__ xy,
    const float* __restrict__ sqrtc, float scale, float alpha, float q,
    float2* __restrict__ partial, const float* __restrict__ alpha_dev,
    const int32_t* __restrict__ gid, const float* __restrict__ galpha) {
  // the tile's coordinates (and pre-scaled roots on coarse levels) in static
  // LDS at a fixed address, so an entry's high 13 bits address them directly
  // the per-hop table (hop_entry) sits at the start of the coordinate array
  // so that both lookups of an entry use the instruction's immediate offset
  constexpr int32_t T = 1 << TB;
  __shared__ float2 slx[16 + T];
  float2* const lut = slx;
  float2* const sx = slx + 16;
  __shared__ float2 ssc[COARSE ? T : 1];  // (sqrt c * scale, unused)
  __shared__ int32_t mblk[UNIT_CH + 1];   // first block of each chunk (absolute)
  __shared__ int32_t mslot[UNIT_CH];
  __shared__ float2 mxu[UNIT_CH];
  __shared__ float mscu[COARSE ? UNIT_CH : 1];
  __shared__ float malpha[UNIT_CH];       // per-graph alpha of each chunk's row (batches)
  const int32_t tile = unit_tile[blockIdx.x];
  const int32_t c0 = unit_c0[blockIdx.x], c1 = unit_c0[blockIdx.x + 1];
  const int32_t nch = c1 - c0;
  const int32_t v0 = tile * T;
  const int32_t nv = min(T, n - v0);
  for (int32_t i = threadIdx.x; i < nv; i += TS_T) {
    sx[i] = xy[v0 + i];
    if (COARSE) ssc[i] = make_float2(sqrtc[v0 + i] * scale, 0.f);
  }
  for (int32_t i = threadIdx.x; i <= nch; i += TS_T) {
    mblk[i] = (int32_t)(chunk_off[c0 + i] >> 3);
    if (i < nch) {
      const int32_t u = chunk_row[c0 + i];
      mslot[i] = chunk_slot[c0 + i];
      mxu[i] = xy[u];
      if (COARSE) mscu[i] = sqrtc[u] * scale;
      if (galpha) malpha[i] = galpha[gid[u]];
    }
  }
  if (alpha_dev) alpha = *alpha_dev;
  if (threadIdx.x < 16) {
    lut[threadIdx.x] = hop_entry<COARSE, Q0>(threadIdx.x);
  }
  __syncthreads();
  const float alpha0 = alpha;
  const int gl = threadIdx.x % G, gi = threadIdx.x / G;
  constexpr int NG = TS_T / G;
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
  if (galpha) alpha = ci < nch ? malpha[ci] : alpha0;
  float px = 0.f, py = 0.f;
  auto run = [&](const u32x4 bk) {
    sweep_block<COARSE, Q0>(bk, sx, ssc, lut, xu, scu, alpha, q, px, py);
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
          if (galpha) alpha = malpha[ci];
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

// ---- the sliced sweep
//
// Sliced layout: the chunks of a tile (sorted by decreasing length) are cut
// into slices of 64; block j of the slice's chunk i is stored at
// slice_base + 64 j + i (chunks shorter than the slice's first are padded
// with zero entries, which contribute 0).  One wave sweeps one slice with
// one lane per chunk: every load of the wave reads 64 consecutive blocks, a
// lane's partial sum is its chunk's, and no lane is idle except on padding
// (the chunks of a slice have nearly equal lengths).  One workgroup per work
// unit (up to kUnitSlices slices of one tile) stages the tile's coordinates once;
// its waves take the unit's slices in turn.  Blocks are loaded NB at a time,
// one step ahead.
template <int NB, int TB, bool COARSE, bool Q0>
__global__ __launch_bounds__(TS_T) void k_sweep_sliced(
    int32_t n, const int32_t* __restrict__ unit_s0, const int32_t* __restrict__ unit_tile,
    const int64_t* __restrict__ slice_base, const int32_t* __restrict__ slice_h,
    const int32_t* __restrict__ slice_c0, const int32_t* __restrict__ chunk_row,
    const int32_t* __restrict__ chunk_slot, const uint16_t* __restrict__ ent,
    const float2* __restrict__ xy, const float* __restrict__ sqrtc, float scale, float alpha,
    float q, float2* __restrict__ partial, const float* __restrict__ alpha_dev,
    const int32_t* __restrict__ gid, const float* __restrict__ galpha, int32_t nunits) {
  constexpr int32_t T = 1 << TB;
  __shared__ float2 slx[16 + T];  // hop table, then the tile's coordinates
  float2* const lut = slx;
  float2* const sx = slx + 16;
  __shared__ float2 ssc[COARSE ? T : 1];  // (sqrt c * scale, unused)
  if (alpha_dev) alpha = *alpha_dev;
  if (threadIdx.x < 16) {
    lut[threadIdx.x] = hop_entry<COARSE, Q0>(threadIdx.x);
  }
  const int l = lane_id();
  const int32_t wv = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
  // work units blockIdx.x, + gridDim.x, ... (one per work-group unless the
  // grid is capped to leave room for kernels running beside the sweep)
  for (int32_t ub = blockIdx.x; ub < nunits; ub += gridDim.x) {
  const int32_t tile = unit_tile[ub];
  const int32_t s0 = unit_s0[ub], s1 = unit_s0[ub + 1];
  const int32_t v0 = tile * T;
  const int32_t nv = min(T, n - v0);
  if (ub != (int32_t)blockIdx.x) __syncthreads();  // the previous unit's reads are done
  for (int32_t i = threadIdx.x; i < nv; i += TS_T) {
    sx[i] = xy[v0 + i];
    if (COARSE) ssc[i] = make_float2(sqrtc[v0 + i] * scale, 0.f);
  }
  __syncthreads();
  for (int32_t sl = s0 + wv; sl < s1; sl += TS_T / 64) {
    // slice parameters are wave-uniform (scalar registers, scalar branches)
    const int32_t c0 = __builtin_amdgcn_readfirstlane(slice_c0[sl]);
    const int32_t nc = __builtin_amdgcn_readfirstlane(slice_c0[sl + 1]) - c0;
    const int32_t h = __builtin_amdgcn_readfirstlane(slice_h[sl]);
    const int64_t sb = slice_base[sl];
    const bool lv = l < nc;
    const int32_t c = c0 + (lv ? l : 0);
    const int32_t row = chunk_row[c];
    const float2 xu = xy[row];
    const float scu = COARSE ? sqrtc[row] * scale : 0.f;
    // batches: the alpha of the row's graph (a lane-varying value)
    const float al = galpha ? galpha[gid[row]] : alpha;
    // the slice's blocks from a wave-uniform base; a lane's block j sits
    // 64 j + l blocks beyond it (32-bit byte offsets within the slice).  Loads
    // past the slice's last row re-read that row (in bounds, never used), so
    // every load is unconditional.
    const char* __restrict__ eb = reinterpret_cast<const char*>(ent) + sb * 16;
    auto ld = [&](int32_t j) {
      const uint32_t jj = (uint32_t)min(j, h - 1);
      return __builtin_nontemporal_load(
          reinterpret_cast<const u32x4*>(eb + (jj * 64u + (uint32_t)l) * 16u));
    };
    float px = 0.f, py = 0.f;
    u32x4 ba[NB], bb[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) ba[b] = ld(b);
    for (int32_t j = 0; j < h; j += 2 * NB) {
#pragma unroll
      for (int b = 0; b < NB; ++b) bb[b] = ld(j + NB + b);
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (j + b < h) sweep_block<COARSE, Q0>(ba[b], sx, ssc, lut, xu, scu, al, q, px, py);
      if (j + NB >= h) break;
#pragma unroll
      for (int b = 0; b < NB; ++b) ba[b] = ld(j + 2 * NB + b);
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (j + NB + b < h) sweep_block<COARSE, Q0>(bb[b], sx, ssc, lut, xu, scu, al, q, px, py);
    }
    if (lv) partial[chunk_slot[c]] = make_float2(px, py);
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
                                                  const float* __restrict__ alpha_dev,
                                                  const int32_t* __restrict__ gid,
                                                  const float* __restrict__ galpha) {
  if (alpha_dev) alpha = *alpha_dev;
  constexpr int RPB = CB_T / CB_G;
  __shared__ double2 red[RPB];
  const int gl = threadIdx.x % CB_G, gi = threadIdx.x / CB_G;
  const int32_t u = blockIdx.x * RPB + gi;
  double2 dd = make_double2(0.0, 0.0);
  // batches: each graph has its own alpha; a negative one marks a finished
  // graph, whose coordinates are carried over unchanged
  const float al = (galpha && u < n) ? galpha[gid[u]] : alpha;
  if (u < n && al < 0.f) {
    if (gl == 0) out[u] = xy[u];
  } else if (u < n) {
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
      // the partial sums are relative to x_u (see the sweep)
      float2 xn;
      xn.x = xu.x + (px + al * fu.x) / r;
      xn.y = xu.y + (py + al * fu.y) / r;
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

hipError_t sweep_tiled_partial(const TiledSet& ts, int32_t level, const float* sqrtc, double scale,
                               const float* xy, double alpha, double q, hipStream_t s,
                               const float* alpha_dev, int32_t group, int32_t nb,
                               const int32_t* gid, const float* galpha, int32_t max_groups) {
  const bool coarse = level > 0 && sqrtc != nullptr;
  const int32_t sl_grid = max_groups > 0 ? std::min(ts.nunits, max_groups) : ts.nunits;
  const bool q0 = q == 0.0;
  if (ts.tbits < 11 || ts.tbits > 13) return hipErrorInvalidValue;
  // a group of G lanes (one 8-entry block each per step) per chunk
  const int G = group > 0 ? group : tiled_group(ts);
  const int NB = nb > 0 ? nb : tiled_blocks(ts);
  float2* part = ts.b_partial.as<float2>();
#define MM_TS(GG, NBV, TBV, C, Q)                                                               \
  k_sweep_tiled<GG, NBV, TBV, C, Q><<<ts.nunits, TS_T, 0, s>>>(                                 \
      ts.n, ts.unit_c0, ts.unit_tile, ts.chunk_off, ts.chunk_row, ts.chunk_slot, ts.ent,         \
      (const float2*)xy, sqrtc, (float)scale, (float)alpha, (float)q, part, alpha_dev, gid, galpha)
#define MM_TST(GG, NBV, TBV)                                                                   \
  do {                                                                                         \
    if (coarse) { if (q0) MM_TS(GG, NBV, TBV, true, true); else MM_TS(GG, NBV, TBV, true, false); } \
    else { if (q0) MM_TS(GG, NBV, TBV, false, true); else MM_TS(GG, NBV, TBV, false, false); }      \
  } while (0)
#define MM_TSN(GG, NBV)                                            \
  do {                                                             \
    if (ts.tbits == 13) MM_TST(GG, NBV, 13);                       \
    else if (ts.tbits == 12) MM_TST(GG, NBV, 12);                  \
    else MM_TST(GG, NBV, 11);                                      \
  } while (0)
#define MM_TSG(GG)                                   \
  do {                                               \
    if (NB == 4) MM_TSN(GG, 4); else MM_TSN(GG, 2);  \
  } while (0)
#define MM_SL(NBV, TBV, C, Q)                                                                   \
  k_sweep_sliced<NBV, TBV, C, Q><<<sl_grid, TS_T, 0, s>>>(                                       \
      ts.n, ts.unit_c0, ts.unit_tile, ts.slice_base, ts.slice_h, ts.slice_c0, ts.chunk_row,      \
      ts.chunk_slot, ts.ent, (const float2*)xy, sqrtc, (float)scale, (float)alpha, (float)q, part, \
      alpha_dev, gid, galpha, ts.nunits)
#define MM_SLT(NBV, TBV)                                                                       \
  do {                                                                                         \
    if (coarse) { if (q0) MM_SL(NBV, TBV, true, true); else MM_SL(NBV, TBV, true, false); }    \
    else { if (q0) MM_SL(NBV, TBV, false, true); else MM_SL(NBV, TBV, false, false); }         \
  } while (0)
#define MM_SLN(NBV)                                                \
  do {                                                             \
    if (ts.tbits == 13) MM_SLT(NBV, 13);                           \
    else if (ts.tbits == 12) MM_SLT(NBV, 12);                      \
    else MM_SLT(NBV, 11);                                          \
  } while (0)
  if (ts.sliced) {
    if (NB == 4) MM_SLN(4); else MM_SLN(2);
  } else {
    switch (G) {
      case 16: MM_TSG(16); break;
      case 8: MM_TSG(8); break;
      case 4: MM_TSG(4); break;
      case 2: MM_TSG(2); break;
      case 1: MM_TSG(1); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef MM_SLN
#undef MM_SLT
#undef MM_SL
#undef MM_TSG
#undef MM_TSN
#undef MM_TST
#undef MM_TS
  return hipGetLastError();
}

hipError_t sweep_tiled_combine(const TiledSet& ts, const float* rho, const float* xy,
                               const float* F, double alpha, float* xy_out, double* delta2_dev,
                               hipStream_t s, const float* alpha_dev, const int32_t* gid,
                               const float* galpha) {
  const int32_t ncb = (ts.n + CB_T / CB_G - 1) / (CB_T / CB_G);
  DevBuf& dpart = const_cast<TiledSet&>(ts).b_dpart;
  if (dpart.bytes < sizeof(double2) * (size_t)ncb) MM_TRY(dpart.alloc(sizeof(double2) * (size_t)ncb, s));
  k_combine<<<ncb, CB_T, 0, s>>>(ts.n, ts.rc_ptr, ts.b_partial.as<float2>(), rho,
                                (const float2*)xy, (const float2*)F, (float)alpha,
                                (float2*)xy_out, dpart.as<double2>(), alpha_dev, gid, galpha);
  // batches take their per-graph relative change elsewhere (delta2_dev null)
  if (delta2_dev) k_sum_parts2<<<1, 1024, 0, s>>>(dpart.as<double2>(), ncb, delta2_dev);
  return hipGetLastError();
}

hipError_t sweep_tiled(const TiledSet& ts, int32_t level, const float* sqrtc, double scale,
                       const float* rho, const float* xy, const float* F, double alpha, double q,
                       float* xy_out, double* delta2_dev, hipStream_t s, const float* alpha_dev,
                       int32_t group, int32_t nb) {
  MM_TRY(sweep_tiled_partial(ts, level, sqrtc, scale, xy, alpha, q, s, alpha_dev, group, nb));
  return sweep_tiled_combine(ts, rho, xy, F, alpha, xy_out, delta2_dev, s, alpha_dev);
}

}  // namespace mm
