// k-hop distance sets S_k(u) = { v != u : hop(u,v) <= k }, sorted by (hop, v):
// the stress superset of the general maxent-stress model (footnote to Eq. 1),
// found by a frontier BFS per source vertex.
//
// Two kernels, each with a counting pass (row lengths and per-hop ends) and
// a filling pass (after an int64 scan of the counts gives the row offsets):
//  * small rows: one wavefront per source; the hop-h frontier lives in LDS;
//    candidates (neighbours of the hop-(h-1) frontier) are bitonic-sorted in
//    LDS, deduplicated, and filtered against hops h-1 and h-2 (a neighbour of
//    a hop-(h-1) vertex has hop h-2, h-1 or h).  Rows whose candidates exceed
//    the LDS capacity are flagged for the big-row kernel.  For k = 2 the
//    counting pass can also keep each row's list in a fixed slot.
//  * big rows: one workgroup per source with two n-bit bitmaps (visited and
//    new; one for k = 2) in LDS when they fit, otherwise in global memory per
//    workgroup slot; the hop-h set is extracted in ascending order by
//    scanning the new bitmap with wave-level prefix sums.  For k = 2 the
//    counting pass keeps each row's hop-2 bitmap for the filling pass, and
//    vertices with long neighbour lists contribute precomputed adjacency
//    bitmaps by OR instead of one mark per neighbour.
// The tile-major copy of the sweep can be built straight from the counting
// pass's state (tilemajor.hip), without the filling pass.
#include <cstdio>
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

constexpr int KS_CAP = 1024;     // list capacity per wave (entries)
constexpr int64_t KS_SLOT = 2 * KS_CAP;  // k = 2: a short row has at most this many entries
constexpr int KS_WAVES = 2;      // waves per block
constexpr int KB_T = 512;        // threads per big-row block
constexpr int KB_NW = KB_T / 64;
constexpr int KB_U = 4;          // frontier vertices per wave step in the bitmap kernel
constexpr int KB_V = 8;          // neighbour loads in flight per lane while marking
constexpr int32_t KB_HUB = 512;  // longer neighbour lists are marked by the whole workgroup
constexpr int KB_HUBCAP = 256;   // hubs deferred per frontier (more: marked by their wave)
constexpr int KB_ORCAP = 4096;   // adjacency bitmaps ORed per row (more: marked)
// the bitmap kernel's static LDS (bytes, rounded up)
constexpr int KB_STATIC_LDS = 4 * (KB_NW + 1 + KB_HUBCAP + 2) + 64;
// 2 x this many bitmap words fit in a CU's 160 KB of LDS beside them
constexpr int KB_LDS_WORDS = (160 * 1024 - KB_STATIC_LDS) / 8;


__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// lower_bound in a sorted LDS list
__device__ inline bool in_sorted(const int32_t* a, int len, int32_t v) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo < len && a[lo] == v;
}

template <bool FILL>
__global__ __launch_bounds__(64 * KS_WAVES) void k_khop_small(
    int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col, int32_t k,
    const int64_t* __restrict__ off, int32_t* __restrict__ hend, int32_t* __restrict__ nbr,
    int32_t* __restrict__ cnt, int32_t* __restrict__ big) {
  __shared__ int32_t lds[KS_WAVES][5][KS_CAP];
  const int w = threadIdx.x >> 6, l = lane_id();
  int32_t u = blockIdx.x * KS_WAVES + w;
  if (u >= n) return;
  if (FILL && big[u]) return;
  int32_t* L0 = lds[w][0];  // hop h-2 list
  int32_t* L1 = lds[w][1];  // hop h-1 list
  int32_t* NW = lds[w][2];  // hop h list
  int32_t* CA = lds[w][3];  // candidates
  int32_t* PF = lds[w][4];  // frontier degree prefix
  const int32_t beg = rp[u], deg = rp[u + 1] - beg;
  // the filling pass writes the row at off[u]; a counting pass given nbr
  // (k = 2) writes it to the fixed slot u * KS_SLOT as well
  const bool put = FILL || nbr != nullptr;
  int64_t o = FILL ? off[u] : (int64_t)u * KS_SLOT;
  if (deg > KS_CAP) {
    if (!FILL) { if (l == 0) big[u] = 1; }
    return;
  }
  // hop 1: N(u)
  for (int i = l; i < deg; i += 64) {
    int32_t v = col[beg + i];
    L1[i] = v;
    if (put) nbr[o + i] = v;
  }
  int len0 = 0, len1 = deg;   // L0 holds {u} implicitly for h = 2
  int32_t total = deg;
  if (!FILL && l == 0) hend[(int64_t)u * k] = deg;
  wave_sync();
  for (int h = 2; h <= k; ++h) {
    // frontier degree prefix
    int32_t run = 0;
    for (int b = 0; b < len1; b += 64) {
      int i = b + l;
      int32_t d = 0;
      if (i < len1) { int32_t x = L1[i]; d = rp[x + 1] - rp[x]; }
      int32_t inc = wave_incl_scan(d);
      if (i < len1) PF[i] = run + inc - d;
      run += __builtin_amdgcn_readlane(inc, 63);
    }
    const int32_t ncand = run;
    if (ncand > KS_CAP) {
      if (!FILL) { if (l == 0) big[u] = 1; }
      return;
    }
    wave_sync();
    int P = 1;
    while (P < ncand) P <<= 1;
    for (int j = l; j < P; j += 64) {
      int32_t v = 0x7fffffff;
      if (j < ncand) {
        int lo = 0, hi = len1;  // last i with PF[i] <= j
        while (hi - lo > 1) {
          int mid = (lo + hi) >> 1;
          if (PF[mid] <= j) lo = mid; else hi = mid;
        }
        int32_t x = L1[lo];
        v = col[rp[x] + (j - PF[lo])];
      }
      CA[j] = v;
    }
    wave_sync();
    // bitonic sort of CA[0..P)
    for (int size = 2; size <= P; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = l; i < (P >> 1); i += 64) {
          int a = 2 * stride * (i / stride) + (i % stride);
          int b = a + stride;
          bool up = (a & size) == 0;
          int32_t x = CA[a], y = CA[b];
          if ((x > y) == up) { CA[a] = y; CA[b] = x; }
        }
        wave_sync();
      }
    }
    // dedupe + filter, compact into NW in order
    int32_t cnt_h = 0;
    for (int b = 0; b < ncand; b += 64) {
      int j = b + l;
      bool keep = false;
      int32_t v = 0;
      if (j < ncand) {
        v = CA[j];
        keep = (j == 0 || CA[j - 1] != v) && v != u && !in_sorted(L1, len1, v) &&
               (h == 2 || !in_sorted(L0, len0, v));
      }
      uint64_t m = __ballot(keep);
      int pos = cnt_h + __popcll(m & lanemask_lt());
      if (keep) {
        NW[pos] = v;
        if (put) nbr[o + total + pos] = v;
      }
      cnt_h += __popcll(m);
    }
    total += cnt_h;
    if (!FILL && l == 0) hend[(int64_t)u * k + (h - 1)] = total;
    wave_sync();
    // rotate lists: L0 <- L1, L1 <- NW
    int32_t* t0 = L0; L0 = L1; L1 = NW; NW = t0;
    len0 = len1; len1 = cnt_h;
  }
  if (!FILL && l == 0) { cnt[u] = total; big[u] = 0; }
}

// ---- big rows: bitmap BFS, one workgroup per source
// ONE (k == 2): a single bitmap; the hop-2 candidates are marked without a
// visited test and u and N(u) are cleared afterwards, which halves the LDS
// footprint (two workgroups per CU for n up to ~650K).
// KEEP (with ONE, when device memory allows): the counting pass stores each
// row's final hop-2 bitmap (n bits per big row, row r at bmkeep + r * Wp,
// Wp = W rounded up to 4 words so that rows start 16-byte aligned) and
// the filling pass extracts from it instead of marking again.
// TEST (with ONE): read a candidate's bit before setting it; pays on dense
// graphs, where most candidates of a row are marked many times.
template <bool FILL, bool LDSBM, bool ONE, bool KEEP, bool TEST>
__global__ __launch_bounds__(KB_T) void k_khop_big(
    int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col, int32_t k,
    const int32_t* __restrict__ rows, int32_t nrows, const int64_t* __restrict__ off,
    int32_t* __restrict__ hend, int32_t* __restrict__ nbr, int32_t* __restrict__ cnt,
    uint32_t* __restrict__ gbm, int32_t* __restrict__ gscratch, uint32_t* __restrict__ bmkeep,
    int32_t hthr, const int32_t* __restrict__ hubidx, const uint32_t* __restrict__ hb,
    int32_t orcap) {
  static_assert(!KEEP || ONE, "kept bitmaps hold hop 2 only");
  constexpr bool LOAD = KEEP && FILL;   // extract from the kept bitmap
  constexpr bool STORE = KEEP && !FILL; // keep the bitmap
  extern __shared__ uint4 dyn4[];  // 16-byte aligned: the OR phase reads it as uint4
  __shared__ int32_t wtot[KB_NW + 1];
  __shared__ int32_t hubs[KB_HUBCAP];
  __shared__ int32_t nhub, norl;
  const int32_t W = (n + 31) >> 5;
  const size_t Wp = (size_t)((W + 3) & ~3);
  const int32_t NB = ONE ? 1 : 2;
  // bitmaps at pitch Wp (the words past W stay 0)
  uint32_t* VIS = LDSBM ? reinterpret_cast<uint32_t*>(dyn4) : gbm + (size_t)blockIdx.x * NB * Wp;
  uint32_t* NEW = ONE ? VIS : VIS + Wp;
  // hub indices to OR (orcap entries, in LDS after the bitmaps; orcap is 0
  // unless hthr is set, which needs the LDS bitmaps)
  int32_t* orl = reinterpret_cast<int32_t*>(dyn4) + NB * Wp;
  int32_t* scratch = gscratch ? gscratch + (size_t)blockIdx.x * (size_t)n : nullptr;
  const int t = threadIdx.x, wv = t >> 6, l = lane_id();
  for (size_t i = t; i < NB * Wp; i += KB_T) VIS[i] = 0;
  if (t == 0) { nhub = 0; norl = 0; }
  __syncthreads();
  // word chunk per wave for the ordered extraction
  const int32_t CW = ((W + KB_NW - 1) / KB_NW + 63) & ~63;
  const int32_t wlo = wv * CW, whi = min(W, wlo + CW);
  for (int32_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int32_t u = rows[r];
    const int32_t beg = rp[u], deg = rp[u + 1] - beg;
    const int64_t o = FILL ? off[u] : 0;
    // hop 1
    for (int32_t i = t; i < deg; i += KB_T) {
      int32_t v = col[beg + i];
      if (!ONE) atomicOr(&VIS[v >> 5], 1u << (v & 31));
      if (FILL) nbr[o + i] = v;
    }
    if (!ONE && t == 0) atomicOr(&VIS[u >> 5], 1u << (u & 31));
    int64_t total = deg;
    if (!FILL && t == 0) hend[(int64_t)u * k] = deg;
    // frontier: hop-(h-1) list
    const int32_t* F = col + beg;
    int32_t flen = deg;
    __syncthreads();
    const uint32_t* kept = LOAD ? bmkeep + (size_t)r * Wp : nullptr;
    for (int h = 2; h <= k; ++h) {
      // mark neighbours of the frontier not yet visited.  The marks are
      // bound by the latency of the neighbour loads and by the instructions
      // around each mark, and most of them come from the few long lists of
      // high-degree vertices (a vertex of degree d lies in d rows'
      // frontiers and costs d marks in each), so:
      //  * a wave takes KB_U frontier vertices at a time and issues their row
      //    bounds and first 64 neighbour loads before marking any;
      //  * the rest of a list is loaded KB_V steps of 64 at a time;
      //  * lists longer than KB_HUB are set aside and marked afterwards by
      //    the whole workgroup, KB_T * KB_V entries per round, so that one
      //    long list does not hold the row on one wave;
      //  * (k = 2) vertices with more than hthr neighbours have their
      //    adjacency bitmap precomputed (hb, row hubidx[x] at pitch Wp): a row
      //    ORs it into its own, 16 bytes per thread and load, instead of
      //    marking the neighbours one by one;
      //  * list bounds are wave-uniform; loads past a list's end read its
      //    last entry instead, so loads need no lane masks, and only the
      //    marks of a list's last, partial step are masked (marking the
      //    clamped copies would send many lanes' atomics to one LDS word,
      //    which serialises them).
      // Bits are only ever set, so the order of the marks does not matter.
      auto mark = [&](int32_t v) {
        const uint32_t bit = 1u << (v & 31);
        if (ONE) {
          if (!TEST || !(NEW[v >> 5] & bit)) atomicOr(&NEW[v >> 5], bit);
        } else {
          if (!(VIS[v >> 5] & bit)) atomicOr(&NEW[v >> 5], bit);
        }
      };
      // entries [e0, len) of the list cb, stride S, this thread's offset me
      auto mark_list = [&](const int32_t* __restrict__ cb, int32_t e0, int32_t len, int32_t S,
                           int32_t me) {
        for (; e0 + S * KB_V <= len; e0 += S * KB_V) {
          int32_t vv[KB_V];
#pragma unroll
          for (int j = 0; j < KB_V; ++j) vv[j] = cb[e0 + S * j + me];
#pragma unroll
          for (int j = 0; j < KB_V; ++j) mark(vv[j]);
        }
        if (e0 < len) {
          int32_t vv[KB_V];
#pragma unroll
          for (int j = 0; j < KB_V; ++j) vv[j] = cb[min(e0 + S * j + me, len - 1)];
#pragma unroll
          for (int j = 0; j < KB_V; ++j)
            if (e0 + S * j + me < len) mark(vv[j]);
        }
      };
      const int32_t wvu = __builtin_amdgcn_readfirstlane(wv);
      for (int32_t i0 = wvu * KB_U; i0 < flen && !LOAD; i0 += KB_NW * KB_U) {
        int32_t b0[KB_U], len[KB_U], v0[KB_U];
#pragma unroll
        for (int uu = 0; uu < KB_U; ++uu) {
          const int32_t x = i0 + uu < flen ? __builtin_amdgcn_readfirstlane(F[i0 + uu]) : -1;
          b0[uu] = x >= 0 ? __builtin_amdgcn_readfirstlane(rp[x]) : 0;
          len[uu] = x >= 0 ? __builtin_amdgcn_readfirstlane(rp[x + 1]) - b0[uu] : 0;
          if (ONE && len[uu] > hthr) {
            // OR its adjacency bitmap after the marks, unless the list is full
            int32_t slot = 0;
            if (l == 0) slot = atomicAdd(&norl, 1);
            slot = __builtin_amdgcn_readfirstlane(__shfl(slot, 0, 64));
            if (slot < orcap) {
              if (l == 0) orl[slot] = hubidx[x];
              len[uu] = 0;
            }
          }
          if (len[uu] > KB_HUB) {
            // defer to the workgroup unless the list is full
            int32_t slot = 0;
            if (l == 0) slot = atomicAdd(&nhub, 1);
            slot = __builtin_amdgcn_readfirstlane(__shfl(slot, 0, 64));
            if (slot < KB_HUBCAP) {
              if (l == 0) hubs[slot] = x;
              len[uu] = 0;
            }
          }
        }
#pragma unroll
        for (int uu = 0; uu < KB_U; ++uu)
          if (len[uu] > 0) v0[uu] = col[b0[uu] + min(l, len[uu] - 1)];
#pragma unroll
        for (int uu = 0; uu < KB_U; ++uu)
          if (l < len[uu]) mark(v0[uu]);
#pragma unroll
        for (int uu = 0; uu < KB_U; ++uu)
          if (len[uu] > 64) mark_list(col + b0[uu], 64, len[uu], 64, l);
      }
      __syncthreads();
      if (!LOAD) {
        const int32_t nh = min(nhub, KB_HUBCAP);
        for (int32_t j = 0; j < nh; ++j) {
          const int32_t x = __builtin_amdgcn_readfirstlane(hubs[j]);
          const int32_t e0 = __builtin_amdgcn_readfirstlane(rp[x]);
          mark_list(col + e0, 0, __builtin_amdgcn_readfirstlane(rp[x + 1]) - e0, KB_T, t);
        }
        __syncthreads();
        if (ONE) {
          // each thread owns 16-byte words of the bitmap: no atomics here
          const int32_t no = min(norl, orcap);
          if (no > 0) {
            const size_t W4 = Wp >> 2;
            uint4* __restrict__ N4 = reinterpret_cast<uint4*>(NEW);
            const uint4* __restrict__ H4 = reinterpret_cast<const uint4*>(hb);
            for (size_t w4 = t; w4 < W4; w4 += KB_T) {
              uint4 a = N4[w4];
              int32_t j = 0;
              for (; j + 4 <= no; j += 4) {
                const uint4 h0 = H4[(size_t)orl[j] * W4 + w4], h1 = H4[(size_t)orl[j + 1] * W4 + w4];
                const uint4 h2 = H4[(size_t)orl[j + 2] * W4 + w4], h3 = H4[(size_t)orl[j + 3] * W4 + w4];
                a.x |= h0.x | h1.x | h2.x | h3.x;
                a.y |= h0.y | h1.y | h2.y | h3.y;
                a.z |= h0.z | h1.z | h2.z | h3.z;
                a.w |= h0.w | h1.w | h2.w | h3.w;
              }
              for (; j < no; ++j) {
                const uint4 h0 = H4[(size_t)orl[j] * W4 + w4];
                a.x |= h0.x;
                a.y |= h0.y;
                a.z |= h0.z;
                a.w |= h0.w;
              }
              N4[w4] = a;
            }
          }
          __syncthreads();
        }
        if (t == 0) { nhub = 0; norl = 0; }
      }
      if (ONE && !LOAD) {
        // drop hop 0 and hop 1 from the candidates
        if (t == 0) atomicAnd(&NEW[u >> 5], ~(1u << (u & 31)));
        for (int32_t i = t; i < deg; i += KB_T) {
          const int32_t v = col[beg + i];
          atomicAnd(&NEW[v >> 5], ~(1u << (v & 31)));
        }
        __syncthreads();
      }
      if (ONE && !FILL) {
        // counting pass of a 2-hop search: the row's hop-2 bits are final;
        // count them, keep them (KEEP) and clear the bitmap for the next row
        // (no positions are needed, so no scans)
        int32_t c = 0;
        uint32_t* __restrict__ keep_row = STORE ? bmkeep + (size_t)r * Wp : nullptr;
        for (int32_t wi = wlo + l; wi < whi; wi += 64) {
          const uint32_t bits = NEW[wi];
          if (STORE) keep_row[wi] = bits;
          c += __popc(bits);
          NEW[wi] = 0u;
        }
        c = wave_sum(c);
        if (l == 0) wtot[wv] = c;
        __syncthreads();
        int32_t cnt_h = 0;
        for (int i = 0; i < KB_NW; ++i) cnt_h += wtot[i];
        total += cnt_h;
        if (t == 0) hend[(int64_t)u * k + (h - 1)] = (int32_t)total;
        __syncthreads();
        flen = cnt_h;
        continue;
      }
      // count per wave chunk
      int32_t c = 0;
      for (int32_t b = wlo; b < whi; b += 64) {
        int32_t wi = b + l;
        if (wi < whi) c += __popc(LOAD ? kept[wi] : NEW[wi]);
      }
      c = wave_sum(c);
      if (l == 0) wtot[wv] = c;
      __syncthreads();
      if (t == 0) {
        int32_t run = 0;
        for (int i = 0; i < KB_NW; ++i) { int32_t x = wtot[i]; wtot[i] = run; run += x; }
        wtot[KB_NW] = run;
      }
      __syncthreads();
      const int32_t cnt_h = wtot[KB_NW];
      const bool last = (h == k);
      int32_t* dst = FILL ? nbr + o + total : (last ? nullptr : scratch);
      int32_t run = wtot[wv];
      for (int32_t b = wlo; b < whi; b += 64) {
        int32_t wi = b + l;
        uint32_t bits = wi < whi ? (LOAD ? kept[wi] : NEW[wi]) : 0u;
        if (STORE && wi < whi) bmkeep[(size_t)r * Wp + wi] = bits;
        int32_t pc = __popc(bits);
        int32_t inc = wave_incl_scan(pc);
        int32_t pos = run + inc - pc;
        if (wi < whi && bits) {
          if (dst) {
            uint32_t bb = bits;
            while (bb) {
              int j = __ffs(bb) - 1;
              bb &= bb - 1;
              dst[pos++] = (wi << 5) + j;
            }
          }
          if (!LOAD) NEW[wi] = 0u;
          if (!ONE && !last) VIS[wi] |= bits;
        }
        run += __builtin_amdgcn_readlane(inc, 63);
      }
      total += cnt_h;
      if (!FILL && t == 0) hend[(int64_t)u * k + (h - 1)] = (int32_t)total;
      __syncthreads();
      F = dst;
      flen = cnt_h;
    }
    // clear VIS: u and hops 1..k-1 (with ONE the extraction already cleared it)
    if (!ONE) {
      if (t == 0) VIS[u >> 5] = 0u;
      for (int32_t i = t; i < deg; i += KB_T) VIS[col[beg + i] >> 5] = 0u;
    }
    if (k >= 3) {
      // hops 2..k-1 are in the output (fill) or were merged into VIS from
      // scratch lists that are gone (count) -> clear the whole bitmap
      for (int32_t i = t; i < W; i += KB_T) VIS[i] = 0u;
    }
    if (!FILL && t == 0) cnt[u] = (int32_t)total;
    __syncthreads();
  }
}

__global__ void k_collect_big(const int32_t* big, int32_t n, const int64_t* pos, int32_t* rows) {
  int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n && big[u]) rows[pos[u]] = u;
}

__global__ void k_hop1(int32_t n, const int32_t* rp, int32_t* hend, int32_t* cnt) {
  int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) { int32_t d = rp[u + 1] - rp[u]; hend[u] = d; cnt[u] = d; }
}

// sum over vertices of deg^2 (the candidate marks of all rows' 2-hop searches)
__global__ __launch_bounds__(256) void k_sum_deg2(int32_t n, const int32_t* rp,
                                                  unsigned long long* out) {
  __shared__ unsigned long long part[4];
  unsigned long long a = 0;
  for (int32_t u = blockIdx.x * 256 + threadIdx.x; u < n; u += gridDim.x * 256) {
    const unsigned long long d = (unsigned long long)(rp[u + 1] - rp[u]);
    a += d * d;
  }
  a = wave_sum(a);
  if (lane_id() == 0) part[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

// vertices with more than thr neighbours: their index among them (or -1)
// and their adjacency bitmaps (row h at hb + h * Wp, zeroed beforehand)
__global__ void k_hub_flags(int32_t n, const int32_t* rp, int32_t thr, int32_t* flag) {
  const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) flag[u] = rp[u + 1] - rp[u] > thr ? 1 : 0;
}
__global__ void k_hub_index(int32_t n, const int32_t* flag, const int64_t* pos, int32_t* hubidx,
                            int32_t* hubv) {
  const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  hubidx[u] = flag[u] ? (int32_t)pos[u] : -1;
  if (flag[u]) hubv[pos[u]] = u;
}
__global__ __launch_bounds__(256) void k_hub_bitmaps(const int32_t* hubv, const int32_t* rp,
                                                     const int32_t* col, int64_t Wp, uint32_t* hb) {
  const int32_t u = hubv[blockIdx.x];
  uint32_t* row = hb + (size_t)blockIdx.x * (size_t)Wp;
  for (int32_t e = rp[u] + threadIdx.x; e < rp[u + 1]; e += 256) {
    const int32_t v = col[e];
    atomicOr(&row[v >> 5], 1u << (v & 31));
  }
}

// counts of the rows the small-row kernel filled (0 for bitmap rows)
__global__ void k_small_counts(int32_t n, const int32_t* cnt, const int32_t* big, int32_t* out) {
  int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) out[u] = big[u] ? 0 : cnt[u];
}

}  // namespace

hipError_t khop_count(int32_t n, const int32_t* rp, const int32_t* col, int32_t k, KhopDev* out,
                      KhopCount* st, hipStream_t s, bool keep_short) {
  out->n = n;
  out->k = k;
  st->k = k;
  MM_TRY(out->b_off.alloc(sizeof(int64_t) * (size_t)(n + 1), s));
  MM_TRY(out->b_hend.alloc(sizeof(int32_t) * (size_t)n * (size_t)k, s));
  out->off = out->b_off.as<int64_t>();
  out->hend = out->b_hend.as<int32_t>();
  MM_TRY(st->cnt.alloc(sizeof(int32_t) * (size_t)n, s));
  if (k == 1) {
    // S_1(u) = N(u): the CSR row itself
    k_hop1<<<(n + 255) / 256, 256, 0, s>>>(n, rp, out->hend, st->cnt.as<int32_t>());
    MM_TRY(scan_excl_i32(st->cnt.as<int32_t>(), out->off, n, s));
    MM_TRY(hipMemcpyAsync(&out->total, out->off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MM_TRY(hipStreamSynchronize(s));
    return hipGetLastError();
  }
  MM_TRY(st->big.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(st->bigpos.alloc(sizeof(int64_t) * (size_t)(n + 1), s));
  MM_TRY(hipMemsetAsync(st->big.p, 0, sizeof(int32_t) * (size_t)n, s));
  const unsigned gs = (unsigned)((n + KS_WAVES - 1) / KS_WAVES);
  // k = 2: keep the short rows' lists (fixed slots of KS_SLOT ids) so that a
  // compact copy needs no second search
  if (keep_short && k == 2) {
    size_t freeb = 0, totb = 0;
    int cur = 0;
    MM_TRY(hipGetDevice(&cur));
    MM_TRY(hipMemGetInfo(&freeb, &totb));
    const size_t sb = sizeof(int32_t) * (size_t)n * KS_SLOT;
    // (at most 8 GB, n <= 2^20: every short row's slot is written whether
    // or not the level's tile-major copy ends up reading it)
    if (sb <= std::min<size_t>((freeb + big_cached_bytes(cur)) / 8, (size_t)8 << 30))
      MM_TRY(st->slots_short.alloc(sb, s));
  }
  k_khop_small<false><<<gs, 64 * KS_WAVES, 0, s>>>(n, rp, col, k, nullptr, out->hend,
                                                  st->slots_short.as<int32_t>(),
                                                  st->cnt.as<int32_t>(), st->big.as<int32_t>());
  MM_TRY(hipGetLastError());
  MM_TRY(scan_excl_i32(st->big.as<int32_t>(), st->bigpos.as<int64_t>(), n, s));
  DevBuf d2;
  MM_TRY(d2.alloc(sizeof(unsigned long long), s));
  MM_TRY(hipMemsetAsync(d2.p, 0, sizeof(unsigned long long), s));
  k_sum_deg2<<<(unsigned)std::min<int64_t>(1024, ((int64_t)n + 255) / 256), 256, 0, s>>>(
      n, rp, d2.as<unsigned long long>());
  MM_TRY(hipGetLastError());
  int64_t nbig = 0;
  unsigned long long sdeg2 = 0;
  MM_TRY(hipMemcpyAsync(&nbig, st->bigpos.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipMemcpyAsync(&sdeg2, d2.p, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  st->nbig = nbig;
  // candidate marks per row (sum deg^2 / n) of at least n: most candidates
  // repeat, and reading the bit first saves their atomics
  st->test = (double)sdeg2 >= (double)n * (double)n;
  const int32_t W = (n + 31) >> 5;
  st->W = W;
  st->Wp = (W + 3) & ~3;
  const bool one = (k == 2);
  st->one = one;
  const int32_t nbw = (one ? 1 : 2) * st->Wp;  // bitmap words per workgroup
  const bool lds_bm = nbw <= 2 * KB_LDS_WORDS;
  st->lds_bm = lds_bm;
  int dev = 0, ncu = 0;
  MM_TRY(hipGetDevice(&dev));
  MM_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  size_t shm = lds_bm ? sizeof(uint32_t) * (size_t)nbw : 0;

  // keep the counting pass's hop-2 bitmaps for the filling pass when they
  // take at most a third of the free device memory
  bool keep = false;
  if (one && nbig > 0) {
    size_t freeb = 0, totb = 0;
    MM_TRY(hipMemGetInfo(&freeb, &totb));
    const size_t kb = sizeof(uint32_t) * (size_t)st->Wp * (size_t)nbig;
    if (kb > freeb / 3) {
      // memory freed by earlier stream-ordered frees may still be held by the
      // device's default pool (not reported as free): release it and look again
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && hipMemPoolTrimTo(pool, 0) == hipSuccess)
        MM_TRY(hipMemGetInfo(&freeb, &totb));
    }
    freeb += big_cached_bytes(dev);  // cached blocks are available too
    if (kb <= freeb / 3) {
      MM_TRY(st->bmk.alloc(kb, s));
      keep = true;
    }
    // MM_VERBOSE=1 reports the decision on stderr
    const char* ev = std::getenv("MM_VERBOSE");
    if (ev && ev[0] == '1')
      std::fprintf(stderr, "[khop] n %d rows with bitmaps %lld (%.2f GB), free %.2f GB: %s\n", n,
                   (long long)nbig, kb / 1e9, freeb / 1e9, keep ? "kept" : "rebuilt");
  }
  st->keep = keep;
  // adjacency bitmaps of the vertices with more than W / 4 neighbours (an
  // OR of W / 4 16-byte words replaces > W / 4 random marks), at most 1 GB.
  // Measured on R-MAT 2^20: they pay on levels whose bitmap rows have at
  // most ~9000 words (levels 2-9: 15-40% less time); on larger levels
  // streaming the hubs' 50-70 KB rows for every row cost more than the marks
  // they replace (+7% and +25% on levels 0 and 1)
  st->hthr = 0x7fffffff;
  st->orcap = 0;
  if (one && lds_bm && nbig > 0 && W <= 9000) {
    int32_t thr = std::max(W / 4, 64);
    DevBuf hf, hpos;
    MM_TRY(hf.alloc(sizeof(int32_t) * (size_t)n, s));
    MM_TRY(hpos.alloc(sizeof(int64_t) * (size_t)(n + 1), s));
    int64_t nh = 0;
    for (;;) {
      k_hub_flags<<<(n + 255) / 256, 256, 0, s>>>(n, rp, thr, hf.as<int32_t>());
      MM_TRY(scan_excl_i32(hf.as<int32_t>(), hpos.as<int64_t>(), n, s));
      MM_TRY(hipMemcpyAsync(&nh, hpos.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      MM_TRY(hipStreamSynchronize(s));
      if (nh * (int64_t)st->Wp * 4 <= ((int64_t)1 << 30) || thr >= n) break;
      thr *= 2;
    }
    if (nh > 0 && nh * (int64_t)st->Wp * 4 <= ((int64_t)1 << 30)) {
      DevBuf hv;
      MM_TRY(st->hubidx.alloc(sizeof(int32_t) * (size_t)n, s));
      MM_TRY(hv.alloc(sizeof(int32_t) * (size_t)nh, s));
      k_hub_index<<<(n + 255) / 256, 256, 0, s>>>(n, hf.as<int32_t>(), hpos.as<int64_t>(),
                                                  st->hubidx.as<int32_t>(), hv.as<int32_t>());
      MM_TRY(st->hb.alloc(sizeof(uint32_t) * (size_t)nh * (size_t)st->Wp, s));
      MM_TRY(hipMemsetAsync(st->hb.p, 0, sizeof(uint32_t) * (size_t)nh * (size_t)st->Wp, s));
      k_hub_bitmaps<<<(unsigned)nh, 256, 0, s>>>(hv.as<int32_t>(), rp, col, st->Wp,
                                                 st->hb.as<uint32_t>());
      MM_TRY(hipGetLastError());
      st->hthr = thr;
      st->orcap = (int32_t)std::min<int64_t>(nh, KB_ORCAP);
      shm += sizeof(int32_t) * (size_t)st->orcap;
    }
  }
  st->shm = shm;
  const int per_cu = lds_bm ? (int)std::max<size_t>(1, (160 * 1024) / (shm + KB_STATIC_LDS)) : 2;
  const int32_t slots = (int32_t)std::min<int64_t>(nbig, (int64_t)ncu * std::min(per_cu, 4));
  st->slots = slots;
#define MM_BIG(FILLV, LDSV, ONEV, KEEPV, TESTV, ...)                                            \
  do {                                                                                         \
    if (LDSV)                                                                                  \
      MM_TRY(hipFuncSetAttribute(                                                              \
          reinterpret_cast<const void*>(&k_khop_big<FILLV, LDSV, ONEV, KEEPV, TESTV>),         \
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)st->shm));                          \
    k_khop_big<FILLV, LDSV, ONEV, KEEPV, TESTV><<<st->slots, KB_T, LDSV ? st->shm : 0, s>>>(   \
        __VA_ARGS__);                                                                          \
  } while (0)
// the filling passes either extract kept bitmaps or mark again (then TEST
// changes nothing but the speed: always on there)
#define MM_BIG_ONE(FILLV, LDSV, KEEPV, ...)                                             \
  do {                                                                                 \
    if (!FILLV && !st->test) MM_BIG(FILLV, LDSV, true, KEEPV, false, __VA_ARGS__);     \
    else MM_BIG(FILLV, LDSV, true, KEEPV, true, __VA_ARGS__);                          \
  } while (0)
#define MM_BIG_ANY(FILLV, ...)                                                          \
  do {                                                                                 \
    if (st->lds_bm) {                                                                  \
      if (st->one && st->keep) MM_BIG_ONE(FILLV, true, true, __VA_ARGS__);             \
      else if (st->one) MM_BIG_ONE(FILLV, true, false, __VA_ARGS__);                   \
      else MM_BIG(FILLV, true, false, false, true, __VA_ARGS__);                       \
    } else {                                                                           \
      if (st->one && st->keep) MM_BIG_ONE(FILLV, false, true, __VA_ARGS__);            \
      else if (st->one) MM_BIG_ONE(FILLV, false, false, __VA_ARGS__);                  \
      else MM_BIG(FILLV, false, false, false, true, __VA_ARGS__);                      \
    }                                                                                  \
  } while (0)
  if (nbig > 0) {
    MM_TRY(st->rows.alloc(sizeof(int32_t) * (size_t)nbig, s));
    k_collect_big<<<(n + 255) / 256, 256, 0, s>>>(st->big.as<int32_t>(), n, st->bigpos.as<int64_t>(),
                                                  st->rows.as<int32_t>());
    if (!lds_bm) MM_TRY(st->gbm.alloc(sizeof(uint32_t) * (size_t)nbw * (size_t)slots, s));
    if (k >= 3) MM_TRY(st->gscr.alloc(sizeof(int32_t) * (size_t)n * (size_t)slots, s));
    MM_BIG_ANY(false, n, rp, col, k, st->rows.as<int32_t>(), (int32_t)nbig, nullptr, out->hend,
               nullptr, st->cnt.as<int32_t>(), st->gbm.as<uint32_t>(), st->gscr.as<int32_t>(),
               st->bmk.as<uint32_t>(), st->hthr, st->hubidx.as<int32_t>(), st->hb.as<uint32_t>(),
               st->orcap);
    MM_TRY(hipGetLastError());
  }
  MM_TRY(scan_excl_i32(st->cnt.as<int32_t>(), out->off, n, s));
  MM_TRY(hipMemcpyAsync(&out->total, out->off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  return hipGetLastError();
}

hipError_t khop_fill(int32_t n, const int32_t* rp, const int32_t* col, KhopDev* out, KhopCount* st,
                     hipStream_t s) {
  const int32_t k = st->k;
  MM_TRY(out->b_nbr.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(out->total, 1), s));
  out->nbr = out->b_nbr.as<int32_t>();
  if (k == 1) {
    if (out->total > 0)
      MM_TRY(hipMemcpyAsync(out->nbr, col, sizeof(int32_t) * (size_t)out->total,
                            hipMemcpyDeviceToDevice, s));
    return hipGetLastError();
  }
  const unsigned gs = (unsigned)((n + KS_WAVES - 1) / KS_WAVES);
  k_khop_small<true><<<gs, 64 * KS_WAVES, 0, s>>>(n, rp, col, k, out->off, out->hend, out->nbr,
                                                 nullptr, st->big.as<int32_t>());
  MM_TRY(hipGetLastError());
  if (st->nbig > 0) {
    MM_BIG_ANY(true, n, rp, col, k, st->rows.as<int32_t>(), (int32_t)st->nbig, out->off, out->hend,
               out->nbr, nullptr, st->gbm.as<uint32_t>(), nullptr, st->bmk.as<uint32_t>(),
               st->hthr, st->hubidx.as<int32_t>(), st->hb.as<uint32_t>(), st->orcap);
    MM_TRY(hipGetLastError());
  }
  return hipGetLastError();
}
#undef MM_BIG_ANY
#undef MM_BIG_ONE
#undef MM_BIG

// off_small[u] = u * KS_SLOT (the short rows' fixed slots)
__global__ void k_slot_offsets(int32_t n, int64_t* off) {
  const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u <= n) off[u] = (int64_t)u * KS_SLOT;
}

hipError_t khop_fill_small(int32_t n, const int32_t* rp, const int32_t* col, const KhopDev& kh,
                           KhopCount* st, DevBuf* off_small, DevBuf* nbr_small, hipStream_t s) {
  if (st->k < 2) return hipErrorInvalidValue;
  MM_TRY(off_small->alloc(sizeof(int64_t) * (size_t)(n + 1), s));
  if (st->slots_short.p) {
    // the counting pass kept them: row u at u * KS_SLOT (its length is its
    // last hop end)
    k_slot_offsets<<<(n + 256) / 256, 256, 0, s>>>(n, off_small->as<int64_t>());
    *nbr_small = std::move(st->slots_short);
    return hipGetLastError();
  }
  DevBuf c;
  MM_TRY(c.alloc(sizeof(int32_t) * (size_t)n, s));
  k_small_counts<<<(n + 255) / 256, 256, 0, s>>>(n, st->cnt.as<int32_t>(), st->big.as<int32_t>(),
                                                 c.as<int32_t>());
  MM_TRY(scan_excl_i32(c.as<int32_t>(), off_small->as<int64_t>(), n, s));
  int64_t tot = 0;
  MM_TRY(hipMemcpyAsync(&tot, off_small->as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  MM_TRY(nbr_small->alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(tot, 1), s));
  const unsigned gs = (unsigned)((n + KS_WAVES - 1) / KS_WAVES);
  k_khop_small<true><<<gs, 64 * KS_WAVES, 0, s>>>(n, rp, col, st->k, off_small->as<int64_t>(),
                                                 kh.hend, nbr_small->as<int32_t>(), nullptr,
                                                 st->big.as<int32_t>());
  return hipGetLastError();
}

hipError_t khop_build(int32_t n, const int32_t* rp, const int32_t* col, int32_t k, KhopDev* out,
                      hipStream_t s) {
  KhopCount st;
  MM_TRY(khop_count(n, rp, col, k, out, &st, s));
  return khop_fill(n, rp, col, out, &st, s);
}

}  // namespace mm
