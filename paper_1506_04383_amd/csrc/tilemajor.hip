// Tile-major copy of the stress sets for the LDS-tiled sweep (tiled.hip):
// the k-hop sets (sorted by (hop, v) per row; canonical ids, or for k = 2
// the bitmaps the search kept for its long rows) are re-laid per
// (row, tile) chunk, 16 bits per entry ((v - tile * T) << 3 | hop), chunks
// ordered by tile and, within a tile, by decreasing length; either
// consecutively (work units of <= kUnitChunks chunks) or in the sliced
// layout (slices of 64 chunks, block j of chunk i at slice_base + 64 j + i;
// work units of <= kUnitSlices slices).  Also rho_u = sum over S(u) of w_uv.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

constexpr int TB_WAVES = 4;          // waves per block of the conversion kernels
constexpr int TB_MAXW = kTiledMaxTiles / 32;
constexpr int RU = 4;                // 64-entry steps loaded at once per wave (conversion)
constexpr int32_t UNIT_CH = kUnitChunks;
constexpr int32_t UNIT_S = kUnitSlices;

// the value of lane l - 1 (lane 0: its own) and of lane l + 1 (lane 63:
// its own), by DPP wave shifts
__device__ inline int32_t lane_prev(int32_t v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false);  // wave_shr:1
}
__device__ inline int32_t lane_next(int32_t v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false);  // wave_shl:1
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
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
    float* __restrict__ rho, const int32_t* __restrict__ skip) {
  __shared__ uint32_t tbm[TB_WAVES][TB_MAXW];
  const int w = threadIdx.x >> 6, l = lane_id();
  const int32_t u = blockIdx.x * TB_WAVES + w;
  if (u >= n || (skip && skip[u])) return;
  uint32_t* bm = tbm[w];
  for (int i = l; i < ntw; i += 64) bm[i] = 0u;
  wave_sync();
  const int64_t beg = off[u];
  const float su = (RHO && sqrtc) ? sqrtc[u] : 0.f;
  float r = 0.f;
  int32_t seg0 = 0;
  for (int h = 1; h <= k; ++h) {
    const int32_t seg1 = hend[(int64_t)u * k + h - 1];
    // RU 64-entry steps per pass, their loads (and sqrt c gathers) issued
    // before any is used; each lane still takes its entries in order
    for (int32_t i0 = seg0; i0 < seg1; i0 += 64 * RU) {
      int32_t vv[RU];
      float sv[RU];
#pragma unroll
      for (int uu = 0; uu < RU; ++uu) {
        const int32_t i = i0 + 64 * uu + l;
        vv[uu] = i < seg1 ? nbr[beg + i] : 0;
      }
#pragma unroll
      for (int uu = 0; uu < RU; ++uu)
        sv[uu] = (RHO && sqrtc && i0 + 64 * uu + l < seg1) ? sqrtc[vv[uu]] : 0.f;
#pragma unroll
      for (int uu = 0; uu < RU; ++uu) {
        if (i0 + 64 * uu + l >= seg1) break;
        const int32_t v = vv[uu];
        const int32_t t = v >> tbits;
        const uint32_t bit = 1u << (t & 31);
        if (!(bm[t >> 5] & bit)) atomicOr(&bm[t >> 5], bit);
        if (RHO && sqrtc) {
          const float d = (float)h * (su + sv[uu]) * scale;
          r += 1.f / (d * d);
        }
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
// loaded RU 64-entry steps at a time.
template <bool FILL, bool BASE>
__global__ __launch_bounds__(64 * TB_WAVES) void k_row_chunks(
    int32_t n, int32_t k, int32_t tbits, int32_t ntiles, int32_t ntw,
    const int64_t* __restrict__ off, const int32_t* __restrict__ hend,
    const int32_t* __restrict__ nbr, const int64_t* __restrict__ rc_ptr,
    int32_t* __restrict__ cm_tile, int32_t* __restrict__ cm_size, int32_t* __restrict__ cm_row,
    const int32_t* __restrict__ pos_of_slot, const int64_t* __restrict__ chunk_off,
    uint16_t* __restrict__ ent, const int32_t* __restrict__ skip) {
  // per wave, sized by the tile count: tile bitmap (ntw words), its popcount
  // prefix (ntw), per-tile counters (ntiles), with BASE the chunk starts
  // (ntiles int64, 8-byte aligned)
  extern __shared__ uint32_t tb_dyn[];
  const int w = threadIdx.x >> 6, l = lane_id();
  const int32_t u = blockIdx.x * TB_WAVES + w;
  if (u >= n || (skip && skip[u])) return;
  const size_t per = ((2 * (size_t)ntw + (size_t)ntiles + 1) & ~(size_t)1) +
                     (BASE ? 2 * (size_t)ntiles : 0);
  uint32_t* bm = tb_dyn + (size_t)w * per;
  int32_t* pf = reinterpret_cast<int32_t*>(bm + ntw);
  int32_t* ct = pf + ntw;
  int64_t* base = BASE ? reinterpret_cast<int64_t*>(bm + ((2 * (size_t)ntw + (size_t)ntiles + 1) &
                                                          ~(size_t)1))
                       : nullptr;
  const int64_t beg = off[u], endr = beg + hend[(int64_t)u * k + k - 1];
  for (int i = l; i < ntw; i += 64) bm[i] = 0u;
  wave_sync();
  for (int64_t e0 = beg; e0 < endr; e0 += 64 * RU) {
    int32_t vv[RU];
#pragma unroll
    for (int uu = 0; uu < RU; ++uu) {
      const int64_t e = e0 + 64 * uu + l;
      vv[uu] = e < endr ? nbr[e] : 0;
    }
#pragma unroll
    for (int uu = 0; uu < RU; ++uu) {
      if (e0 + 64 * uu + l >= endr) break;
      const int32_t t = vv[uu] >> tbits;
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
    for (int32_t b0 = seg0; b0 < seg1; b0 += 64 * RU) {
      int32_t vv[RU];
#pragma unroll
      for (int uu = 0; uu < RU; ++uu) {
        const int32_t i = b0 + 64 * uu + l;
        vv[uu] = i < seg1 ? nbr[beg + i] : 0;
      }
#pragma unroll
      for (int uu = 0; uu < RU; ++uu) {
        const int32_t b = b0 + 64 * uu;
        if (b >= seg1) break;  // wave-uniform
        const int32_t i = b + l;
        const bool valid = i < seg1;
        const int32_t v = vv[uu];
        const int32_t t = valid ? (v >> tbits) : 0x7fffffff;
        const int32_t tprev = lane_prev(t);
        const bool start = valid && (l == 0 || tprev != t);
        const int32_t rs = wave_incl_max(start ? l : -1);
        const int32_t tnext = lane_next(t);
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
    }
    seg0 = seg1;
  }
  if (FILL) {
    // each chunk's padding to a whole 8-entry block: hop 0
    wave_sync();
    for (int i = l; i < ntw; i += 64) {
      uint32_t bb = bm[i];
      int32_t rank = pf[i];
      while (bb) {
        const int j = __ffs(bb) - 1;
        bb &= bb - 1;
        const int32_t t = (i << 5) + j;
        const int64_t cb = BASE ? base[t] : chunk_off[pos_of_slot[rbase + rank]];
        for (int32_t p = ct[t]; p & 7; ++p) ent[cb + p] = 0;
        rank++;
      }
    }
  } else {
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

// ---- rows read straight from the breadth-first search (direct build, k = 2)
// A big row u = rows[r] has hop 1 = its CSR row (ascending) and hop 2 = the
// set bits of its kept bitmap (bm + r * W, ascending), which is exactly its
// canonical set; these kernels produce what the three passes above produce
// for it from the canonical set, with the same results.

constexpr int32_t kDirectMaxTiles = 1024;  // LDS per wave: 12 B per tile

// words wb .. wb + 3 of a kept bitmap row (16-byte aligned; wb a multiple of
// 4); words at or past W (the row's padding) read as 0
__device__ __forceinline__ uint4 load_words4(const uint4* __restrict__ row, int32_t wb, int32_t W) {
  if (wb >= W) return make_uint4(0u, 0u, 0u, 0u);
  uint4 q = row[wb >> 2];
  if (wb + 3 >= W) {
    if (wb + 1 >= W) q.y = 0u;
    if (wb + 2 >= W) q.z = 0u;
    q.w = 0u;
  }
  return q;
}

// K1 for big rows: the row's entries per tile (dense, tcnt[r * ntiles + t])
// and its tile count; with RHO (finest level) also rho_u from the hop counts
// (k_row_tiles' formula).
template <bool RHO>
__global__ __launch_bounds__(64 * TB_WAVES) void k_big_tiles(
    int64_t nbig, const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ col, const uint32_t* __restrict__ bm, int32_t W, int32_t Wp,
    const int32_t* __restrict__ hend, int32_t tbits, int32_t ntiles, int32_t* __restrict__ tcnt,
    int32_t* __restrict__ nch, float* __restrict__ rho) {
  extern __shared__ int32_t bt_dyn[];
  const int w = threadIdx.x >> 6, l = lane_id();
  const int64_t r = (int64_t)blockIdx.x * TB_WAVES + w;
  if (r >= nbig) return;
  int32_t* ct = bt_dyn + (size_t)w * (size_t)ntiles;
  const int32_t u = rows[r];
  for (int32_t t = l; t < ntiles; t += 64) ct[t] = 0;
  wave_sync();
  const int32_t b = rp[u], d = rp[u + 1] - b;
  // hop 1: in a 64-entry step of the ascending row a tile's entries are one run
  for (int32_t i0 = 0; i0 < d; i0 += 64) {
    const int32_t i = i0 + l;
    const bool valid = i < d;
    const int32_t v = valid ? col[b + i] : 0;
    const int32_t t = valid ? (v >> tbits) : 0x7fffffff;
    const int32_t tprev = lane_prev(t);
    const bool start = valid && (l == 0 || tprev != t);
    const int32_t rs = wave_incl_max(start ? l : -1);
    const int32_t tnext = lane_next(t);
    const bool end = valid && (l == 63 || i + 1 >= d || tnext != t);
    if (end) ct[t] += l - rs + 1;
    wave_sync();
  }
  // hop 2: 256-word steps, four words per lane (a tile's words are a run of
  // G >= 16 lanes), two steps loaded at a time; per tile a group sum
  const uint4* __restrict__ brow = reinterpret_cast<const uint4*>(bm + (size_t)r * (size_t)Wp);
  const int32_t tsh = tbits - 5;
  const int32_t G = min(64, (1 << tsh) >> 2);
  for (int32_t w0 = 0; w0 < W; w0 += 512) {
    uint4 x[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) x[j] = load_words4(brow, w0 + 256 * j + 4 * l, W);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int32_t wb = w0 + 256 * j + 4 * l;
      int32_t c = __popc(x[j].x) + __popc(x[j].y) + __popc(x[j].z) + __popc(x[j].w);
      c = group_sum(c, G);
      if ((l & (G - 1)) == 0 && wb < W) ct[wb >> tsh] += c;
    }
  }
  wave_sync();
  int32_t nt = 0;
  int32_t* __restrict__ trow = tcnt + (size_t)r * (size_t)ntiles;
  for (int32_t t = l; t < ntiles; t += 64) {
    const int32_t c = ct[t];
    trow[t] = c;
    nt += c > 0 ? 1 : 0;
  }
  nt = wave_sum(nt);
  if (l == 0) nch[u] = nt;
  if (RHO && l == 0) {
    int32_t prev = 0;
    float rr = 0.f;
    for (int h = 1; h <= 2; ++h) {
      const int32_t e = hend[(int64_t)u * 2 + h - 1];
      rr += (float)(e - prev) / (float)(h * h);
      prev = e;
    }
    rho[u] = rr;
  }
}

// K3 for big rows: the row-major chunk slots (tile, size, row) in tile order
__global__ __launch_bounds__(64 * TB_WAVES) void k_big_slots(
    int64_t nbig, const int32_t* __restrict__ rows, int32_t ntiles,
    const int32_t* __restrict__ tcnt, const int64_t* __restrict__ rc_ptr,
    int32_t* __restrict__ cm_tile, int32_t* __restrict__ cm_size, int32_t* __restrict__ cm_row) {
  const int w = threadIdx.x >> 6, l = lane_id();
  const int64_t r = (int64_t)blockIdx.x * TB_WAVES + w;
  if (r >= nbig) return;
  const int32_t u = rows[r];
  const int64_t rbase = rc_ptr[u];
  const int32_t* __restrict__ trow = tcnt + (size_t)r * (size_t)ntiles;
  int32_t run = 0;
  for (int32_t t0 = 0; t0 < ntiles; t0 += 64) {
    const int32_t t = t0 + l;
    const int32_t c = t < ntiles ? trow[t] : 0;
    const uint64_t m = __ballot(c > 0);
    const int32_t rank = run + __popcll(m & lanemask_lt());
    if (c > 0) {
      cm_tile[rbase + rank] = t;
      cm_size[rbase + rank] = c;
      cm_row[rbase + rank] = u;
    }
    run += __popcll(m);
  }
}

// K6 for big rows: the 16-bit entries, per chunk hop 1 then hop 2, each
// ascending (the canonical order restricted to the tile).  Per wave in LDS:
// the start of each touched tile's chunk (int64) and its fill count.
__global__ __launch_bounds__(64 * TB_WAVES) void k_big_fill(
    int64_t nbig, const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ col, const uint32_t* __restrict__ bm, int32_t W, int32_t Wp,
    int32_t tbits, int32_t ntiles, const int32_t* __restrict__ tcnt,
    const int64_t* __restrict__ rc_ptr, const int32_t* __restrict__ pos_of_slot,
    const int64_t* __restrict__ chunk_off, uint16_t* __restrict__ ent) {
  extern __shared__ int64_t bf_dyn[];
  const int w = threadIdx.x >> 6, l = lane_id();
  const int64_t r = (int64_t)blockIdx.x * TB_WAVES + w;
  if (r >= nbig) return;
  const size_t per = (size_t)ntiles + (((size_t)ntiles + 1) >> 1);  // int64 units
  int64_t* base = bf_dyn + (size_t)w * per;
  int32_t* ct = reinterpret_cast<int32_t*>(base + ntiles);
  const int32_t u = rows[r];
  const int64_t rbase = rc_ptr[u];
  const int32_t* __restrict__ trow = tcnt + (size_t)r * (size_t)ntiles;
  int32_t run = 0;
  for (int32_t t0 = 0; t0 < ntiles; t0 += 64) {
    const int32_t t = t0 + l;
    const int32_t c = t < ntiles ? trow[t] : 0;
    const uint64_t m = __ballot(c > 0);
    const int32_t rank = run + __popcll(m & lanemask_lt());
    if (t < ntiles) {
      ct[t] = 0;
      if (c > 0) {
        const int64_t cb = chunk_off[pos_of_slot[rbase + rank]];
        base[t] = cb;
        // the chunk's padding to a whole 8-entry block: hop 0
        for (int32_t p = c; p & 7; ++p) ent[cb + p] = 0;
      }
    }
    run += __popcll(m);
  }
  wave_sync();
  const int32_t lo = (1 << tbits) - 1;
  const int32_t b = rp[u], d = rp[u + 1] - b;
  for (int32_t i0 = 0; i0 < d; i0 += 64) {
    const int32_t i = i0 + l;
    const bool valid = i < d;
    const int32_t v = valid ? col[b + i] : 0;
    const int32_t t = valid ? (v >> tbits) : 0x7fffffff;
    const int32_t tprev = lane_prev(t);
    const bool start = valid && (l == 0 || tprev != t);
    const int32_t rs = wave_incl_max(start ? l : -1);
    const int32_t tnext = lane_next(t);
    const bool end = valid && (l == 63 || i + 1 >= d || tnext != t);
    if (valid) ent[base[t] + ct[t] + (l - rs)] = (uint16_t)(((v & lo) << 3) | 1);
    wave_sync();
    if (end) ct[t] += l - rs + 1;
    wave_sync();
  }
  // hop 2: 64-word steps, one word per lane (consecutive lanes then write
  // consecutive entries: four words per lane spread each store over four
  // times the addresses and ran slower), four steps loaded at a time; a
  // 64-word step lies inside one tile
  const uint32_t* __restrict__ brow = bm + (size_t)r * (size_t)Wp;
  const int32_t tsh = tbits - 5;
  for (int32_t w0 = 0; w0 < W; w0 += 256) {
    uint32_t x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int32_t wi = w0 + 64 * j + l;
      x[j] = wi < W ? brow[wi] : 0u;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int32_t wj = w0 + 64 * j;
      if (wj >= W) break;
      const int32_t pc = __popc(x[j]);
      const int32_t inc = wave_incl_scan(pc);
      const int32_t tot = __builtin_amdgcn_readlane(inc, 63);
      if (tot == 0) continue;
      const int32_t t = wj >> tsh;
      int64_t pos = base[t] + ct[t] + (inc - pc);
      uint32_t xx = x[j];
      while (xx) {
        const int bit = __ffs(xx) - 1;
        xx &= xx - 1;
        const int32_t v = ((wj + l) << 5) + bit;
        ent[pos++] = (uint16_t)(((v & lo) << 3) | 2);
      }
      wave_sync();
      if (l == 0) ct[t] += tot;
      wave_sync();
    }
  }
}

// rho_u on coarse levels (w_uv = 1 / (hop (sqrt c_u + sqrt c_v) scale)^2)
// from the consecutive tile-major chunks: a wave sums one chunk at a time
// (16-byte blocks of 8 entries, padding entries have hop 0) into the chunk's
// row-major slot, with sqrt c of the block's first chunk's tile staged in LDS
// (chunks are sorted by tile, so a block rarely straddles two tiles; other
// tiles' values are read from memory); k_rho_rows adds a row's slots in slot
// order.  Per entry this reads 2 bytes and one LDS word instead of
// gathering sqrt c_v from memory for every entry of every row.
constexpr int32_t RH_CH = 256;  // chunks per workgroup
template <int TB>
__global__ __launch_bounds__(256) void k_rho_chunks(
    int64_t m, const uint64_t* __restrict__ skey, const int64_t* __restrict__ chunk_off,
    const int32_t* __restrict__ chunk_row, const int32_t* __restrict__ chunk_slot,
    const uint4* __restrict__ ent, int32_t n, const float* __restrict__ sqrtc, float scale,
    float* __restrict__ part) {
  constexpr int32_t T = 1 << TB;
  __shared__ float ssc[T];
  const int64_t c0 = (int64_t)blockIdx.x * RH_CH;
  const int32_t t0 = (int32_t)(skey[c0] >> 32);
  const int32_t v0 = t0 * T, nv = min(T, n - v0);
  for (int32_t i = threadIdx.x; i < nv; i += 256) ssc[i] = sqrtc[v0 + i];
  __syncthreads();
  const int l = lane_id();
  const int32_t wv = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
  const int64_t c1 = min<int64_t>(c0 + RH_CH, m);
  for (int64_t c = c0 + wv; c < c1; c += 4) {
    const int32_t t = __builtin_amdgcn_readfirstlane((int32_t)(skey[c] >> 32));
    const int64_t b0 = chunk_off[c] >> 3, b1 = chunk_off[c + 1] >> 3;
    const float su = sqrtc[chunk_row[c]];
    const float* __restrict__ sv = t == t0 ? ssc : sqrtc + (size_t)t * T;
    float r = 0.f;
    for (int64_t b = b0 + l; b < b1; b += 64) {
      const uint4 q = ent[b];
      const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t e = (w4[k >> 1] >> (16 * (k & 1))) & 0xffffu;
        const uint32_t h = e & 7u;
        // hardware reciprocal (within 1 ulp); padding (hop 0) adds 0
        const float d = (float)h * (su + sv[e >> 3]) * scale;
        r += h ? __builtin_amdgcn_rcpf(d * d) : 0.f;
      }
    }
    r = wave_sum(r);
    if (l == 0) part[chunk_slot[c]] = r;
  }
}
__global__ void k_rho_rows(int32_t n, const int64_t* __restrict__ rc_ptr,
                           const float* __restrict__ part, float* __restrict__ rho) {
  const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  float r = 0.f;
  for (int64_t s = rc_ptr[u]; s < rc_ptr[u + 1]; ++s) r += part[s];
  rho[u] = r;
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

// Sliced layout.  Sorted chunk c has rank r = c - tile_first[tile] within its
// tile; slices are the runs of 64 ranks.  flag[c] = 1 where a slice starts.
__global__ void k_slice_flags(int64_t m, const uint64_t* __restrict__ skey,
                              const int32_t* __restrict__ tile_first, int32_t* __restrict__ flag) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  const int64_t r = c - tile_first[skey[c] >> 32];
  flag[c] = (r & 63) == 0 ? 1 : 0;
}
// slice s (= spos[c] at its first chunk): first chunk, height in blocks (its
// first chunk is its longest) and the 64 h blocks it occupies
__global__ void k_slice_fill(int64_t m, const int32_t* __restrict__ flag,
                             const int64_t* __restrict__ spos, const int32_t* __restrict__ ssize,
                             int32_t* __restrict__ slice_c0, int32_t* __restrict__ slice_h,
                             int32_t* __restrict__ slice_blocks) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m || !flag[c]) return;
  const int64_t sl = spos[c];
  slice_c0[sl] = (int32_t)c;
  slice_h[sl] = ssize[c] >> 3;
  slice_blocks[sl] = (ssize[c] >> 3) * 64;
}
// Consecutive layout -> sliced layout through LDS, a workgroup per slice
// (grid-stride over slices), in windows of TJ block rows: the waves read
// runs of TJ consecutive blocks of a chunk (half a wave per chunk, so each
// read instruction covers two chunks' contiguous runs) into an LDS tile
// [chunk][row], then write block rows, lane i taking chunk i (1 KB per
// row).  Blocks past a chunk's end, and the rows of lanes without a chunk,
// are written as zero blocks, so every block of the slice is written.  The
// tile's row stride (TJ + 1 blocks) keeps both phases free of bank conflicts.
constexpr int TJ = 32;
__global__ __launch_bounds__(256) void k_slice_transpose(
    int64_t nsl, const int32_t* __restrict__ slice_c0, const int32_t* __restrict__ slice_h,
    const int64_t* __restrict__ slice_base, const int64_t* __restrict__ chunk_off,
    const uint4* __restrict__ src, uint4* __restrict__ dst) {
  __shared__ uint4 tl[64][TJ + 1];
  __shared__ int64_t cb[64];
  __shared__ int32_t cn[64];
  const int t = threadIdx.x, w = t >> 6, l = lane_id();
  const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t sl = blockIdx.x; sl < nsl; sl += gridDim.x) {
    const int32_t c0 = slice_c0[sl], nc = slice_c0[sl + 1] - c0, h = slice_h[sl];
    if (t < 64) {
      const bool v = t < nc;
      const int64_t b0 = v ? chunk_off[c0 + t] >> 3 : 0;
      cb[t] = b0;
      cn[t] = v ? (int32_t)((chunk_off[c0 + t + 1] >> 3) - b0) : 0;
    }
    __syncthreads();
    uint4* __restrict__ d = dst + slice_base[sl];
    for (int32_t j0 = 0; j0 < h; j0 += TJ) {
      // chunks 2p and 2p + 1 per wave instruction, p = w, w + 4, ...
      const int32_t jj = l & (TJ - 1);
      for (int32_t p = w; p < 32; p += 4) {
        const int32_t i = 2 * p + (l >> 5);
        const int32_t b = j0 + jj;
        tl[i][jj] = b < cn[i] ? src[cb[i] + b] : zero;
      }
      __syncthreads();
      const int32_t rows = min(TJ, h - j0);
      for (int32_t j = w; j < rows; j += 4) d[(int64_t)(j0 + j) * 64 + l] = tl[l][j];
      __syncthreads();
    }
  }
}
// unit starts over slices: the first slice of a tile, every UNIT_S-th slice
// after it, and every slice that begins a new span of emax blocks
__global__ void k_slice_unit_flags(int32_t S, const int32_t* __restrict__ slice_c0,
                                   const uint64_t* __restrict__ skey,
                                   const int32_t* __restrict__ tile_first,
                                   const int64_t* __restrict__ slice_base, int64_t emax,
                                   int32_t* __restrict__ flag) {
  const int32_t sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= S) return;
  const int32_t c = slice_c0[sl];
  const int32_t rs = (c - tile_first[skey[c] >> 32]) >> 6;  // slice rank within the tile
  flag[sl] = (rs % UNIT_S == 0 || (rs > 0 && slice_base[sl] / emax != slice_base[sl - 1] / emax))
                 ? 1 : 0;
}
__global__ void k_slice_unit_fill(int32_t S, const int32_t* __restrict__ flag,
                                  const int64_t* __restrict__ pos,
                                  const int32_t* __restrict__ slice_c0,
                                  const uint64_t* __restrict__ skey, int32_t* __restrict__ unit_s0,
                                  int32_t* __restrict__ unit_tile) {
  const int32_t sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= S || !flag[sl]) return;
  unit_s0[pos[sl]] = sl;
  unit_tile[pos[sl]] = (int32_t)(skey[slice_c0[sl]] >> 32);
}

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

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

bool tiled_eligible(const KhopDev& kh, int32_t tbits) {
  const int64_t ntiles = ((int64_t)kh.n + (1 << tbits) - 1) >> tbits;
  // entries are (local id << 3) | hop: 3 hop bits, tbits + 3 <= 16
  return kh.k <= 7 && tbits <= 13 && ntiles <= kTiledMaxTiles && kh.total > 0;
}

hipError_t compute_rho(const KhopDev& kh, const float* sqrtc, double scale, float* rho,
                       hipStream_t s) {
  k_rho<<<nblk(kh.n, 4), 256, 0, s>>>(kh.n, kh.k, kh.off, kh.hend, kh.nbr, sqrtc, (float)scale, rho);
  return hipGetLastError();
}

namespace {

// Where the rows' entries come from: the canonical lists (off, nbr) for
// every row not flagged in skip; the flagged ("big") rows, listed in rows,
// from their CSR row (hop 1) and kept hop-2 bitmap (bm + r * W).
struct TileSrc {
  int32_t n = 0, k = 0;
  int64_t total = 0;
  const int64_t* off = nullptr;
  const int32_t* hend = nullptr;
  const int32_t* nbr = nullptr;
  const int32_t* skip = nullptr;
  int64_t nbig = 0;
  const int32_t* rows = nullptr;
  const uint32_t* bm = nullptr;
  int32_t W = 0, Wp = 0;
  const int32_t* rp = nullptr;
  const int32_t* col = nullptr;
};

hipError_t tiled_build_src(const TileSrc& src, int32_t tbits, double min_avg_chunk, TiledSet* ts,
                           hipStream_t s, const float* sqrtc, double scale, float* rho, bool sliced) {
  const int32_t n = src.n;
  const int32_t ntiles = (int32_t)(((int64_t)n + (1 << tbits) - 1) >> tbits);
  const int32_t ntw = (ntiles + 31) >> 5;
  ts->n = n;
  ts->tbits = tbits;
  ts->ntiles = ntiles;
  DevBuf nch, cm_tile, cm_size, cm_row, skeys, svals, ssize, flag, upos;
  MM_TRY(nch.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(ts->b_rc_ptr.alloc(sizeof(int64_t) * (size_t)(n + 1), s));
  ts->rc_ptr = ts->b_rc_ptr.as<int64_t>();
  // coarse levels: rho from the built chunks (below); finest level: from
  // the hop counts in the first pass
  const bool rho_first = rho && !sqrtc;
  if (rho_first)
    k_row_tiles<true><<<nblk(n, TB_WAVES), 64 * TB_WAVES, 0, s>>>(
        n, src.k, tbits, ntw, src.off, src.hend, src.nbr, nullptr, 1.f, nch.as<int32_t>(), rho,
        src.skip);
  else
    k_row_tiles<false><<<nblk(n, TB_WAVES), 64 * TB_WAVES, 0, s>>>(
        n, src.k, tbits, ntw, src.off, src.hend, src.nbr, nullptr, 1.f, nch.as<int32_t>(), nullptr,
        src.skip);
  MM_TRY(hipGetLastError());
  // big rows: entries per tile (dense, kept for the slot and fill passes)
  DevBuf tcnt;
  const unsigned gbig = (unsigned)((src.nbig + TB_WAVES - 1) / TB_WAVES);
  if (src.nbig > 0) {
    MM_TRY(tcnt.alloc(sizeof(int32_t) * (size_t)src.nbig * (size_t)ntiles, s));
    const size_t shm = sizeof(int32_t) * TB_WAVES * (size_t)ntiles;
    if (rho_first)
      k_big_tiles<true><<<gbig, 64 * TB_WAVES, shm, s>>>(
          src.nbig, src.rows, src.rp, src.col, src.bm, src.W, src.Wp, src.hend, tbits, ntiles,
          tcnt.as<int32_t>(), nch.as<int32_t>(), rho);
    else
      k_big_tiles<false><<<gbig, 64 * TB_WAVES, shm, s>>>(
          src.nbig, src.rows, src.rp, src.col, src.bm, src.W, src.Wp, src.hend, tbits, ntiles,
          tcnt.as<int32_t>(), nch.as<int32_t>(), nullptr);
    MM_TRY(hipGetLastError());
  }
  MM_TRY(scan_excl_i32(nch.as<int32_t>(), ts->rc_ptr, n, s));
  int64_t m = 0;
  MM_TRY(hipMemcpyAsync(&m, ts->rc_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  if (m >= (1ll << 31)) return hipErrorInvalidValue;
  ts->nchunks = m;
  ts->avg_chunk = (double)src.total / (double)std::max<int64_t>(m, 1);
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
      n, src.k, tbits, ntiles, ntw, src.off, src.hend, src.nbr, ts->rc_ptr, cm_tile.as<int32_t>(),
      cm_size.as<int32_t>(), cm_row.as<int32_t>(), nullptr, nullptr, nullptr, src.skip);
  MM_TRY(hipGetLastError());
  if (src.nbig > 0) {
    k_big_slots<<<gbig, 64 * TB_WAVES, 0, s>>>(src.nbig, src.rows, ntiles, tcnt.as<int32_t>(),
                                               ts->rc_ptr, cm_tile.as<int32_t>(),
                                               cm_size.as<int32_t>(), cm_row.as<int32_t>());
    MM_TRY(hipGetLastError());
  }
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
  DevBuf tfirst;
  MM_TRY(tfirst.alloc(sizeof(int32_t) * (size_t)ntiles, s));
  k_tile_first<<<nblk(m), 256, 0, s>>>(m, skeys.as<uint64_t>(), tfirst.as<int32_t>());
  int64_t nsl = 0;
  DevBuf sflag, spos;
  // consecutive chunks (the sliced layout is built from them)
  MM_TRY(scan_excl_i32(ssize.as<int32_t>(), ts->chunk_off, m, s));
  if (sliced) {
    // slices of 64 chunks of one tile; block j of the slice's chunk i at
    // slice_base + 64 j + i
    MM_TRY(sflag.alloc(sizeof(int32_t) * (size_t)m, s));
    MM_TRY(spos.alloc(sizeof(int64_t) * (size_t)(m + 1), s));
    k_slice_flags<<<nblk(m), 256, 0, s>>>(m, skeys.as<uint64_t>(), tfirst.as<int32_t>(),
                                          sflag.as<int32_t>());
    MM_TRY(scan_excl_i32(sflag.as<int32_t>(), spos.as<int64_t>(), m, s));
    MM_TRY(hipMemcpyAsync(&nsl, spos.as<int64_t>() + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MM_TRY(hipStreamSynchronize(s));
    DevBuf sblocks;
    MM_TRY(ts->b_slice_c0.alloc(sizeof(int32_t) * (size_t)(nsl + 1), s));
    MM_TRY(ts->b_slice_h.alloc(sizeof(int32_t) * (size_t)nsl, s));
    MM_TRY(ts->b_slice_base.alloc(sizeof(int64_t) * (size_t)(nsl + 1), s));
    MM_TRY(sblocks.alloc(sizeof(int32_t) * (size_t)nsl, s));
    ts->slice_c0 = ts->b_slice_c0.as<int32_t>();
    ts->slice_h = ts->b_slice_h.as<int32_t>();
    ts->slice_base = ts->b_slice_base.as<int64_t>();
    k_slice_fill<<<nblk(m), 256, 0, s>>>(m, sflag.as<int32_t>(), spos.as<int64_t>(),
                                         ssize.as<int32_t>(), ts->slice_c0, ts->slice_h,
                                         sblocks.as<int32_t>());
    k_set_i32<<<1, 1, 0, s>>>(ts->slice_c0 + nsl, (int32_t)m);
    MM_TRY(scan_excl_i32(sblocks.as<int32_t>(), ts->slice_base, nsl, s));
  }
  // chunk -> row-major slot
  MM_TRY(ts->b_chunk_slot.alloc(sizeof(int32_t) * (size_t)m, s));
  ts->chunk_slot = ts->b_chunk_slot.as<int32_t>();
  MM_TRY(hipMemcpyAsync(ts->chunk_slot, svals.p, sizeof(int32_t) * (size_t)m,
                        hipMemcpyDeviceToDevice, s));
  int64_t padded = 0;
  MM_TRY(hipMemcpyAsync(&padded, ts->chunk_off + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  int64_t sl_blocks = 0;
  if (sliced)
    MM_TRY(hipMemcpyAsync(&sl_blocks, ts->slice_base + nsl, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  if ((padded >> 3) >= (1ll << 31) || sl_blocks >= (1ll << 31)) return hipSuccess;  // int32 block ids
  // the consecutive layout: the sets themselves, or the staging copy of the
  // sliced layout
  DevBuf stage;
  DevBuf& cons = sliced ? stage : ts->b_ent;
  MM_TRY(cons.alloc(sizeof(uint16_t) * (size_t)std::max<int64_t>(padded, 8), s));
  // (every chunk's padding is written by the filling kernels)
  if (use_base)
    k_row_chunks<true, true><<<nblk(n, TB_WAVES), 64 * TB_WAVES, tb_shm_base, s>>>(
        n, src.k, tbits, ntiles, ntw, src.off, src.hend, src.nbr, ts->rc_ptr, nullptr, nullptr,
        nullptr, pos_of_slot, ts->chunk_off, cons.as<uint16_t>(), src.skip);
  else
    k_row_chunks<true, false><<<nblk(n, TB_WAVES), 64 * TB_WAVES, tb_shm, s>>>(
        n, src.k, tbits, ntiles, ntw, src.off, src.hend, src.nbr, ts->rc_ptr, nullptr, nullptr,
        nullptr, pos_of_slot, ts->chunk_off, cons.as<uint16_t>(), src.skip);
  MM_TRY(hipGetLastError());
  if (src.nbig > 0) {
    const size_t shm = sizeof(int64_t) * TB_WAVES * ((size_t)ntiles + (((size_t)ntiles + 1) >> 1));
    k_big_fill<<<gbig, 64 * TB_WAVES, shm, s>>>(src.nbig, src.rows, src.rp, src.col, src.bm, src.W,
                                               src.Wp, tbits, ntiles, tcnt.as<int32_t>(), ts->rc_ptr,
                                               pos_of_slot, ts->chunk_off, cons.as<uint16_t>());
    MM_TRY(hipGetLastError());
  }
  if (rho && sqrtc) {
    DevBuf part;
    MM_TRY(part.alloc(sizeof(float) * (size_t)m, s));
    const unsigned gr = (unsigned)((m + RH_CH - 1) / RH_CH);
#define MM_RH(TBV)                                                                             \
  k_rho_chunks<TBV><<<gr, 256, 0, s>>>(m, skeys.as<uint64_t>(), ts->chunk_off, ts->chunk_row,   \
                                       svals.as<int32_t>(), cons.as<uint4>(), n, sqrtc,         \
                                       (float)scale, part.as<float>())
    if (tbits == 13) MM_RH(13);
    else if (tbits == 12) MM_RH(12);
    else MM_RH(11);
#undef MM_RH
    MM_TRY(hipGetLastError());
    k_rho_rows<<<nblk(n), 256, 0, s>>>(n, ts->rc_ptr, part.as<float>(), rho);
    MM_TRY(hipGetLastError());
  }
  if (sliced) {
    padded = sl_blocks * 8;
    MM_TRY(ts->b_ent.alloc(sizeof(uint16_t) * (size_t)std::max<int64_t>(padded, 8), s));
    k_slice_transpose<<<(unsigned)std::min<int64_t>(nsl, 16384), 256, 0, s>>>(
        nsl, ts->slice_c0, ts->slice_h, ts->slice_base, ts->chunk_off, cons.as<uint4>(),
        ts->b_ent.as<uint4>());
    MM_TRY(hipGetLastError());
  }  // the staging copy is freed (stream-ordered) on return
  ts->ent = ts->b_ent.as<uint16_t>();
  ts->total = src.total;
  ts->padded = padded;
  // work units: chunks (tiled) or slices (sliced) of one tile
  const int64_t mu = sliced ? nsl : m;
  MM_TRY(flag.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(mu, 1), s));
  MM_TRY(upos.alloc(sizeof(int64_t) * (size_t)(mu + 1), s));
  // at least ~8 work units per CU when the level is small; never fewer
  // than 64K entries per unit (the tile staging is amortised over them)
  const int64_t emax = std::max<int64_t>(65536, padded / 2048);
  if (sliced)
    k_slice_unit_flags<<<nblk(mu), 256, 0, s>>>((int32_t)mu, ts->slice_c0, skeys.as<uint64_t>(),
                                                tfirst.as<int32_t>(), ts->slice_base, emax / 8,
                                                flag.as<int32_t>());
  else
    k_unit_flags<<<nblk(m), 256, 0, s>>>(m, skeys.as<uint64_t>(), tfirst.as<int32_t>(),
                                         ts->chunk_off, emax, flag.as<int32_t>());
  MM_TRY(scan_excl_i32(flag.as<int32_t>(), upos.as<int64_t>(), mu, s));
  int64_t nu = 0;
  MM_TRY(hipMemcpyAsync(&nu, upos.as<int64_t>() + mu, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  ts->nunits = (int32_t)nu;
  MM_TRY(ts->b_unit_c0.alloc(sizeof(int32_t) * (size_t)(nu + 1), s));
  MM_TRY(ts->b_unit_tile.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nu, 1), s));
  ts->unit_c0 = ts->b_unit_c0.as<int32_t>();
  ts->unit_tile = ts->b_unit_tile.as<int32_t>();
  if (sliced)
    k_slice_unit_fill<<<nblk(mu), 256, 0, s>>>((int32_t)mu, flag.as<int32_t>(), upos.as<int64_t>(),
                                               ts->slice_c0, skeys.as<uint64_t>(), ts->unit_c0,
                                               ts->unit_tile);
  else
    k_unit_fill<<<nblk(m), 256, 0, s>>>(m, flag.as<int32_t>(), upos.as<int64_t>(),
                                        skeys.as<uint64_t>(), ts->unit_c0, ts->unit_tile);
  k_set_i32<<<1, 1, 0, s>>>(ts->unit_c0 + nu, (int32_t)mu);
  ts->sliced = sliced;
  ts->nslices = nsl;
  MM_TRY(ts->b_partial.alloc(sizeof(float2) * (size_t)m, s));
  ts->built = true;
  return hipGetLastError();
}

}  // namespace

hipError_t tiled_build(const KhopDev& kh, int32_t tbits, double min_avg_chunk, TiledSet* ts,
                       hipStream_t s, const float* sqrtc, double scale, float* rho, bool sliced) {
  TileSrc src;
  src.n = kh.n;
  src.k = kh.k;
  src.total = kh.total;
  src.off = kh.off;
  src.hend = kh.hend;
  src.nbr = kh.nbr;
  return tiled_build_src(src, tbits, min_avg_chunk, ts, s, sqrtc, scale, rho, sliced);
}

bool tiled_direct_ok(const KhopDev& kh, const KhopCount& st, int32_t tbits) {
  const int64_t ntiles = ((int64_t)kh.n + (1 << tbits) - 1) >> tbits;
  // dense per-tile counts of the big rows: at most 2 GB
  return kh.k == 2 && st.k == 2 && st.keep && st.nbig > 0 && tiled_eligible(kh, tbits) &&
         ntiles <= kDirectMaxTiles && st.nbig * ntiles * 4 <= (int64_t)2 << 30;
}

hipError_t tiled_build_direct(const KhopDev& kh, const KhopCount& st, const int32_t* row_ptr,
                              const int32_t* col, const int64_t* off_small,
                              const int32_t* nbr_small, int32_t tbits, double min_avg_chunk,
                              TiledSet* ts, hipStream_t s, const float* sqrtc, double scale,
                              float* rho, bool sliced) {
  if (!tiled_direct_ok(kh, st, tbits)) return hipErrorInvalidValue;
  TileSrc src;
  src.n = kh.n;
  src.k = kh.k;
  src.total = kh.total;
  src.off = off_small;
  src.hend = kh.hend;
  src.nbr = nbr_small;
  src.skip = st.big.as<int32_t>();
  src.nbig = st.nbig;
  src.rows = st.rows.as<int32_t>();
  src.bm = st.bmk.as<uint32_t>();
  src.W = st.W;
  src.Wp = st.Wp;
  src.rp = row_ptr;
  src.col = col;
  return tiled_build_src(src, tbits, min_avg_chunk, ts, s, sqrtc, scale, rho, sliced);
}

}  // namespace mm
