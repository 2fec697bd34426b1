// Coarsening (Section 3.1): size-constrained label propagation and
// contraction, in a synchronous two-colour form with a fixed tie-break so the
// result is a function of (graph, U, seed, level) only.
//
// Per round r and colour s: v is active iff bit 0 of SplitMix64 draw
// (seed, level, tag 16 + r, v) equals s.  Cluster weights W are frozen at the
// start of the sub-round.  An active v scores each neighbouring label by the
// summed edge weight; a label is feasible iff it is v's own or
// W(L) + c(v) <= U; the best feasible label has the highest score, ties going
// to v's own label, then to the smallest id; foreign labels of score 0 never
// win.  Proposals to L are admitted in ascending v while W(L) plus the running
// sum of c over proposals to L stays <= U.  Every quantity is an integer, so
// the GPU result equals the sequential definition bit for bit.
//
// Scoring uses one wavefront per active vertex with an open-addressing hash
// table (label -> score) in LDS for degree <= 128, in global memory otherwise;
// vertices of degree > 2048 (hubs) get a whole work-group each, so their
// neighbour lists do not leave one wave running long after the others.
// Admission: proposals compacted in v order, stably radix-sorted by target,
// then an int64 prefix sum of c gives every proposal its running sum.
// Contraction: labels are ranked, cut edges keyed (C(u), C(v)) and radix
// sorted, equal keys merged with prefix sums of w (exact integer sums).
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

constexpr int LP_WAVES = 4;
constexpr int LP_SLOTS = 256;  // LDS hash slots per wave (degree <= 128)
constexpr int LP_SMALL = 128;
constexpr int LP_BIG = 2048;   // degree above which a whole work-group scores the vertex
constexpr int LP_BT = 1024;    // threads of that work-group

__global__ void k_weights(int32_t n, const int32_t* __restrict__ label, const int32_t* __restrict__ c,
                          unsigned long long* __restrict__ W) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) atomicAdd(&W[label[v]], (unsigned long long)(c ? c[v] : 1));
}

struct Cand {
  long long sc;
  int32_t lab;
  int32_t own;
};
__device__ inline bool better(const Cand& a, const Cand& b) {
  if (a.sc != b.sc) return a.sc > b.sc;
  if (a.own != b.own) return a.own > b.own;
  return a.lab < b.lab;
}
// one step of the wave reduction: compare with the candidate of the lane
// the DPP control CTRL selects (rows outside RM, and lanes whose source lies
// outside their row, compare with themselves)
template <int CTRL, int RM>
__device__ inline void best_step(Cand& c) {
  const int32_t lo = (int32_t)(uint32_t)(unsigned long long)c.sc;
  const int32_t hi = (int32_t)((unsigned long long)c.sc >> 32);
  Cand d;
  const uint32_t dlo = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, RM, 0xf, false);
  const uint32_t dhi = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, RM, 0xf, false);
  d.sc = (long long)(((unsigned long long)dhi << 32) | dlo);
  d.lab = __builtin_amdgcn_update_dpp(c.lab, c.lab, CTRL, RM, 0xf, false);
  d.own = __builtin_amdgcn_update_dpp(c.own, c.own, CTRL, RM, 0xf, false);
  if (better(d, c)) c = d;
}
// The best candidate of the wave (every lane active; `better` is a total
// order, so the result does not depend on the order of the comparisons):
// DPP row shifts then row broadcasts leave it in lane 63, which every lane
// reads.
__device__ inline Cand wave_best(Cand c) {
  best_step<0x111, 0xf>(c);  // row_shr:1
  best_step<0x112, 0xf>(c);  // row_shr:2
  best_step<0x114, 0xf>(c);  // row_shr:4
  best_step<0x118, 0xf>(c);  // row_shr:8
  best_step<0x142, 0xa>(c);  // row_bcast:15
  best_step<0x143, 0xc>(c);  // row_bcast:31
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(unsigned long long)c.sc, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)((unsigned long long)c.sc >> 32), 63);
  Cand r;
  r.sc = (long long)(((unsigned long long)hi << 32) | lo);
  r.lab = __builtin_amdgcn_readlane(c.lab, 63);
  r.own = __builtin_amdgcn_readlane(c.own, 63);
  return r;
}
__device__ inline uint32_t hslot(int32_t lab, uint32_t mask) {
  return ((uint32_t)lab * 2654435761u) & mask;
}

// big: nonzero => use global tables; gkeys/gsc sized by hoff (per-vertex table offsets).
// Orders a work-group's own hash-table writes and atomics before its reads.
__device__ inline void lp_table_fence(bool global_table) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if (global_table) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__global__ __launch_bounds__(64 * LP_WAVES) void k_lp_propose(
    int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const int32_t* __restrict__ c, const int32_t* __restrict__ ew, const int32_t* __restrict__ label,
    const unsigned long long* __restrict__ W, double U, uint64_t stream, int colour,
    int32_t* __restrict__ prop, const int64_t* __restrict__ hoff, int32_t* __restrict__ gkeys,
    long long* __restrict__ gsc, const int32_t* __restrict__ gid, const int32_t* __restrict__ goff,
    const double* __restrict__ Ug, const int32_t* __restrict__ gstop) {
  __shared__ int32_t skey[LP_WAVES][LP_SLOTS];
  // hubs are scored by k_lp_propose_big
  {
    const int32_t vv = blockIdx.x * LP_WAVES + (threadIdx.x >> 6);
    if (vv < n && rp[vv + 1] - rp[vv] > LP_BIG) return;
  }
  __shared__ long long ssc[LP_WAVES][LP_SLOTS];
  const int w = threadIdx.x >> 6, l = lane_id();
  const int32_t v = blockIdx.x * LP_WAVES + w;
  if (v >= n) return;
  // batches: each graph has its own U, draws keyed by the local vertex id, and
  // graphs that stopped take no part in later rounds
  uint64_t vid = (uint64_t)v;
  if (gid) {
    const int32_t g = gid[v];
    if (gstop[g]) { if (l == 0) prop[v] = -1; return; }
    U = Ug[g];
    vid = (uint64_t)(v - goff[g]);
  }
  const bool active = (int)(sm64_at(stream, vid) & 1ull) == colour;
  if (!active) { if (l == 0) prop[v] = -1; return; }
  const int32_t beg = rp[v], deg = rp[v + 1] - beg;
  const int32_t own = label[v];
  const long long cv = c ? c[v] : 1;
  int32_t* keys;
  long long* sc;
  uint32_t mask;
  if (deg <= LP_SMALL) {
    // the wave's LDS table, cut to a power of two of at least 2 deg slots
    // (and one per lane): it holds the same (label, score) pairs as the
    // full table, so the choice below is the same, with less to clear and scan
    uint32_t slots = 64;
    while (slots < 2u * (uint32_t)deg) slots <<= 1;
    keys = skey[w]; sc = ssc[w]; mask = slots - 1u;
  } else {
    keys = gkeys + hoff[v]; sc = gsc + hoff[v];
    mask = (uint32_t)(hoff[v + 1] - hoff[v]) - 1u;
  }
  for (uint32_t i = l; i <= mask; i += 64) { keys[i] = -1; sc[i] = 0; }
  // the wave's own table writes/atomics before its reads: only this wave
  // touches the table, so a work-group-scope release orders them (a
  // device-scope release would also write back the L2); a global table's
  // reads also take a device-scope acquire, which drops this CU's L1 copies
  lp_table_fence(deg > LP_SMALL);
  __builtin_amdgcn_wave_barrier();
  for (int32_t e = l; e < deg; e += 64) {
    const int32_t lab = label[col[beg + e]];
    const long long wt = ew ? ew[beg + e] : 1;
    uint32_t s = hslot(lab, mask);
    for (;;) {
      int32_t prev = atomicCAS(&keys[s], -1, lab);
      if (prev == -1 || prev == lab) break;
      s = (s + 1) & mask;
    }
    atomicAdd((unsigned long long*)&sc[s], (unsigned long long)wt);
  }
  // the wave's own table writes/atomics before its reads: only this wave
  // touches the table, so a work-group-scope release orders them (a
  // device-scope release would also write back the L2); a global table's
  // reads also take a device-scope acquire, which drops this CU's L1 copies
  lp_table_fence(deg > LP_SMALL);
  __builtin_amdgcn_wave_barrier();
  Cand best;
  best.sc = -1; best.lab = 0x7fffffff; best.own = 0;
  for (uint32_t i = l; i <= mask; i += 64) {
    const int32_t lab = keys[i];
    if (lab < 0) continue;
    Cand cd;
    cd.sc = sc[i];
    cd.lab = lab;
    cd.own = (lab == own);
    if (!cd.own) {
      if (cd.sc <= 0) continue;
      if ((double)((long long)W[lab] + cv) > U) continue;  // infeasible
    }
    if (better(cd, best)) best = cd;
  }
  // own label always competes (score 0 when no neighbour carries it)
  if (l == 0) {
    Cand o; o.sc = 0; o.lab = own; o.own = 1;
    if (better(o, best)) best = o;
  }
  best = wave_best(best);
  if (l == 0) prop[v] = (best.lab != own) ? best.lab : -1;
}

// One work-group per hub vertex (degree > LP_BIG): the same scoring as
// k_lp_propose over the vertex's global table, with the block's threads
// sharing the neighbour list and the table scan.
__global__ __launch_bounds__(LP_BT) void k_lp_propose_big(
    const int32_t* __restrict__ bigv, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ col, const int32_t* __restrict__ c,
    const int32_t* __restrict__ ew, const int32_t* __restrict__ label,
    const unsigned long long* __restrict__ W, double U, uint64_t stream, int colour,
    int32_t* __restrict__ prop, const int64_t* __restrict__ hoff, int32_t* __restrict__ gkeys,
    long long* __restrict__ gsc, const int32_t* __restrict__ gid, const int32_t* __restrict__ goff,
    const double* __restrict__ Ug, const int32_t* __restrict__ gstop) {
  __shared__ Cand wb[LP_BT / 64];
  const int t = threadIdx.x, w = t >> 6, l = lane_id();
  const int32_t v = bigv[blockIdx.x];
  uint64_t vid = (uint64_t)v;
  if (gid) {
    const int32_t g = gid[v];
    if (gstop[g]) { if (t == 0) prop[v] = -1; return; }
    U = Ug[g];
    vid = (uint64_t)(v - goff[g]);
  }
  const bool active = (int)(sm64_at(stream, vid) & 1ull) == colour;
  if (!active) { if (t == 0) prop[v] = -1; return; }
  const int32_t beg = rp[v], deg = rp[v + 1] - beg;
  const int32_t own = label[v];
  const long long cv = c ? c[v] : 1;
  int32_t* keys = gkeys + hoff[v];
  long long* sc = gsc + hoff[v];
  const uint32_t mask = (uint32_t)(hoff[v + 1] - hoff[v]) - 1u;
  for (uint32_t i = t; i <= mask; i += LP_BT) { keys[i] = -1; sc[i] = 0; }
  // the table is this work-group's: the barrier (work-group-scope fences)
  // orders its global writes and atomics, the acquire drops stale L1 lines
  __syncthreads();
  lp_table_fence(true);
  for (int32_t e = t; e < deg; e += LP_BT) {
    const int32_t lab = label[col[beg + e]];
    const long long wt = ew ? ew[beg + e] : 1;
    uint32_t sl = hslot(lab, mask);
    for (;;) {
      int32_t prev = atomicCAS(&keys[sl], -1, lab);
      if (prev == -1 || prev == lab) break;
      sl = (sl + 1) & mask;
    }
    atomicAdd((unsigned long long*)&sc[sl], (unsigned long long)wt);
  }
  __syncthreads();
  lp_table_fence(true);
  Cand best;
  best.sc = -1; best.lab = 0x7fffffff; best.own = 0;
  for (uint32_t i = t; i <= mask; i += LP_BT) {
    const int32_t lab = keys[i];
    if (lab < 0) continue;
    Cand cd;
    cd.sc = sc[i];
    cd.lab = lab;
    cd.own = (lab == own);
    if (!cd.own) {
      if (cd.sc <= 0) continue;
      if ((double)((long long)W[lab] + cv) > U) continue;  // infeasible
    }
    if (better(cd, best)) best = cd;
  }
  best = wave_best(best);
  if (l == 0) wb[w] = best;
  __syncthreads();
  if (t == 0) {
    Cand b = wb[0];
    for (int i = 1; i < LP_BT / 64; ++i) if (better(wb[i], b)) b = wb[i];
    // own label always competes (score 0 when no neighbour carries it)
    Cand o; o.sc = 0; o.lab = own; o.own = 1;
    if (better(o, b)) b = o;
    prop[v] = (b.lab != own) ? b.lab : -1;
  }
}

__global__ void k_big_flags(int32_t n, const int32_t* __restrict__ rp, int32_t* __restrict__ flag) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) flag[v] = rp[v + 1] - rp[v] > LP_BIG ? 1 : 0;
}
__global__ void k_big_list(int32_t n, const int32_t* __restrict__ flag,
                           const int64_t* __restrict__ pos, int32_t* __restrict__ bigv) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && flag[v]) bigv[pos[v]] = v;
}

__global__ void k_prop_flags(int32_t n, const int32_t* __restrict__ prop, int32_t* __restrict__ flag) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) flag[v] = prop[v] >= 0 ? 1 : 0;
}
__global__ void k_prop_compact(int32_t n, const int32_t* __restrict__ prop,
                               const int64_t* __restrict__ pos, uint64_t* __restrict__ keys,
                               int32_t* __restrict__ vals) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && prop[v] >= 0) {
    keys[pos[v]] = (uint64_t)prop[v];
    vals[pos[v]] = v;
  }
}
__global__ void k_gather_c(int64_t m, const int32_t* __restrict__ vals, const int32_t* __restrict__ c,
                           int32_t* __restrict__ cs) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) cs[j] = c ? c[vals[j]] : 1;
}
__global__ void k_admit(int64_t m, const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals,
                        const int64_t* __restrict__ csum, const unsigned long long* __restrict__ W,
                        double U, int32_t* __restrict__ label, int32_t* __restrict__ moves,
                        const int32_t* __restrict__ gid, const double* __restrict__ Ug,
                        int32_t* __restrict__ gmoves) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const uint64_t L = keys[j];
  if (gid) U = Ug[gid[vals[j]]];
  int64_t lo = 0, hi = j;  // first index with key == L
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < L) lo = mid + 1; else hi = mid;
  }
  const long long run = csum[j + 1] - csum[lo];
  if ((double)((long long)W[L] + run) <= U) {
    label[vals[j]] = (int32_t)L;
    atomicAdd(moves, 1);
    if (gid) atomicAdd(&gmoves[gid[vals[j]]], 1);
  }
}

// After a round: graphs without moves stop (their result would not change
// in the single-graph run, which ends there).
__global__ void k_round_end(int32_t M, int32_t* __restrict__ gmoves, int32_t* __restrict__ gstop) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M) return;
  if (gmoves[g] == 0) gstop[g] = 1;
  gmoves[g] = 0;
}

__global__ void k_hash_sizes(int32_t n, const int32_t* __restrict__ rp, int64_t* __restrict__ sz) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t d = rp[v + 1] - rp[v];
  int64_t s = 0;
  if (d > LP_SMALL) { s = 1; while (s < 2 * (int64_t)d) s <<= 1; }
  sz[v] = s;
}

// ---- contraction
__global__ void k_mark(int32_t n, const int32_t* __restrict__ label, int32_t* __restrict__ present) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) present[label[v]] = 1;
}
__global__ void k_cluster(int32_t n, const int32_t* __restrict__ label, const int64_t* __restrict__ rank,
                          const int32_t* __restrict__ c, int32_t* __restrict__ cluster,
                          int32_t* __restrict__ cc) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t C = (int32_t)rank[label[v]];
  cluster[v] = C;
  atomicAdd(&cc[C], c ? c[v] : 1);
}
__global__ void k_cut_flags(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ cluster, int32_t* __restrict__ flag) {
  int32_t v = blockIdx.x;
  const int32_t cv = cluster[v];
  for (int32_t e = rp[v] + threadIdx.x; e < rp[v + 1]; e += blockDim.x)
    flag[e] = cluster[col[e]] != cv ? 1 : 0;
}
__global__ void k_cut_emit(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const int32_t* __restrict__ ew, const int32_t* __restrict__ cluster,
                           const int64_t* __restrict__ pos, int64_t nc, uint64_t* __restrict__ keys,
                           int32_t* __restrict__ vals) {
  int32_t v = blockIdx.x;
  const int32_t cv = cluster[v];
  for (int32_t e = rp[v] + threadIdx.x; e < rp[v + 1]; e += blockDim.x) {
    const int32_t cu = cluster[col[e]];
    if (cu != cv) {
      keys[pos[e]] = (uint64_t)cv * (uint64_t)nc + (uint64_t)cu;
      vals[pos[e]] = ew ? ew[e] : 1;
    }
  }
}
__global__ void k_heads(int64_t m, const uint64_t* __restrict__ keys, int32_t* __restrict__ head) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) head[j] = (j == 0 || keys[j - 1] != keys[j]) ? 1 : 0;
}
__global__ void k_coarse_edges(int64_t m, const uint64_t* __restrict__ keys,
                               const int32_t* __restrict__ head, const int64_t* __restrict__ hpos,
                               const int64_t* __restrict__ wsum, int64_t nc,
                               int32_t* __restrict__ ccol, int32_t* __restrict__ cw,
                               int32_t* __restrict__ rowcnt) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m || !head[j]) return;
  const uint64_t K = keys[j];
  int64_t lo = j + 1, hi = m;  // end of run
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (keys[mid] <= K) lo = mid + 1; else hi = mid;
  }
  const int64_t q = hpos[j];
  ccol[q] = (int32_t)(K % (uint64_t)nc);
  cw[q] = (int32_t)(wsum[lo] - wsum[j]);
  atomicAdd(&rowcnt[(int32_t)(K / (uint64_t)nc)], 1);
}
__global__ void k_i64_to_i32(int64_t n, const int64_t* __restrict__ a, int32_t* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (int32_t)a[i];
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t lp_cluster(const GraphDev& g, double U, int32_t rounds, uint64_t seed, int32_t level_h,
                      int32_t* label, int32_t* rounds_run, int64_t* moves_host, hipStream_t s,
                      const LpSeg* seg) {
  const int32_t n = g.n;
  const int32_t* gid = seg ? seg->gid : nullptr;
  const int32_t* goff = seg ? seg->goff : nullptr;
  const double* Ug = seg ? seg->Ug : nullptr;
  int32_t* gstop = seg ? seg->gstop : nullptr;
  DevBuf gmoves;
  if (seg) {
    MM_TRY(gmoves.alloc(sizeof(int32_t) * (size_t)seg->M, s));
    MM_TRY(hipMemsetAsync(gmoves.p, 0, sizeof(int32_t) * (size_t)seg->M, s));
  }
  DevBuf W, prop, flag, pos, keys, vals, cs, csum, moves, hsz, hoff, gk, gsc;
  MM_TRY(W.alloc(sizeof(unsigned long long) * (size_t)n, s));
  MM_TRY(prop.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(flag.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(pos.alloc(sizeof(int64_t) * (size_t)(n + 1), s));
  MM_TRY(keys.alloc(sizeof(uint64_t) * (size_t)n, s));
  MM_TRY(vals.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(cs.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(csum.alloc(sizeof(int64_t) * (size_t)(n + 1), s));
  MM_TRY(moves.alloc(sizeof(int32_t) * 2, s));
  MM_TRY(hsz.alloc(sizeof(int64_t) * (size_t)n, s));
  MM_TRY(hoff.alloc(sizeof(int64_t) * (size_t)(n + 1), s));
  k_hash_sizes<<<nblk(n), 256, 0, s>>>(n, g.row_ptr, hsz.as<int64_t>());
  MM_TRY(scan_excl_i64(hsz.as<int64_t>(), hoff.as<int64_t>(), n, s));
  int64_t hslots = 0;
  MM_TRY(hipMemcpyAsync(&hslots, hoff.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  MM_TRY(gk.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(hslots, 1), s));
  MM_TRY(gsc.alloc(sizeof(long long) * (size_t)std::max<int64_t>(hslots, 1), s));
  // hub vertices, scored one work-group each
  DevBuf bigv;
  int64_t nbig = 0;
  k_big_flags<<<nblk(n), 256, 0, s>>>(n, g.row_ptr, flag.as<int32_t>());
  MM_TRY(scan_excl_i32(flag.as<int32_t>(), pos.as<int64_t>(), n, s));
  MM_TRY(hipMemcpyAsync(&nbig, pos.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  if (nbig > 0) {
    MM_TRY(bigv.alloc(sizeof(int32_t) * (size_t)nbig, s));
    k_big_list<<<nblk(n), 256, 0, s>>>(n, flag.as<int32_t>(), pos.as<int64_t>(), bigv.as<int32_t>());
  }
  MM_TRY(iota_i32(label, n, s));
  int lbits = 1;
  while ((1ll << lbits) < (int64_t)n) lbits++;
  int32_t r_done = 0;
  for (int32_t r = 0; r < rounds; ++r) {
    const uint64_t st = rng_stream(seed, (uint32_t)level_h, TAG_LP + (uint32_t)r);
    MM_TRY(hipMemsetAsync(moves.p, 0, sizeof(int32_t), s));
    for (int colour = 0; colour < 2; ++colour) {
      MM_TRY(hipMemsetAsync(W.p, 0, sizeof(unsigned long long) * (size_t)n, s));
      k_weights<<<nblk(n), 256, 0, s>>>(n, label, g.c, W.as<unsigned long long>());
      k_lp_propose<<<nblk(n, LP_WAVES), 64 * LP_WAVES, 0, s>>>(
          n, g.row_ptr, g.col, g.c, g.w, label, W.as<unsigned long long>(), U, st, colour,
          prop.as<int32_t>(), hoff.as<int64_t>(), gk.as<int32_t>(), gsc.as<long long>(), gid, goff,
          Ug, gstop);
      if (nbig > 0)
        k_lp_propose_big<<<(unsigned)nbig, LP_BT, 0, s>>>(
            bigv.as<int32_t>(), g.row_ptr, g.col, g.c, g.w, label, W.as<unsigned long long>(), U, st,
            colour, prop.as<int32_t>(), hoff.as<int64_t>(), gk.as<int32_t>(), gsc.as<long long>(),
            gid, goff, Ug, gstop);
      k_prop_flags<<<nblk(n), 256, 0, s>>>(n, prop.as<int32_t>(), flag.as<int32_t>());
      MM_TRY(scan_excl_i32(flag.as<int32_t>(), pos.as<int64_t>(), n, s));
      int64_t m = 0;
      MM_TRY(hipMemcpyAsync(&m, pos.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      MM_TRY(hipStreamSynchronize(s));
      if (m == 0) continue;
      k_prop_compact<<<nblk(n), 256, 0, s>>>(n, prop.as<int32_t>(), pos.as<int64_t>(),
                                             keys.as<uint64_t>(), vals.as<int32_t>());
      MM_TRY(radix_sort_pairs(keys.as<uint64_t>(), vals.as<int32_t>(), m, lbits, s));
      k_gather_c<<<nblk(m), 256, 0, s>>>(m, vals.as<int32_t>(), g.c, cs.as<int32_t>());
      MM_TRY(scan_excl_i32(cs.as<int32_t>(), csum.as<int64_t>(), m, s));
      k_admit<<<nblk(m), 256, 0, s>>>(m, keys.as<uint64_t>(), vals.as<int32_t>(), csum.as<int64_t>(),
                                      W.as<unsigned long long>(), U, label, moves.as<int32_t>(),
                                      gid, Ug, gmoves.as<int32_t>());
      MM_TRY(hipGetLastError());
    }
    if (seg) k_round_end<<<nblk(seg->M), 256, 0, s>>>(seg->M, gmoves.as<int32_t>(), gstop);
    int32_t mv = 0;
    MM_TRY(hipMemcpyAsync(&mv, moves.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MM_TRY(hipStreamSynchronize(s));
    if (moves_host) moves_host[r] = mv;
    r_done = r + 1;
    if (mv == 0) break;
  }
  *rounds_run = r_done;
  return hipGetLastError();
}

hipError_t contract(const GraphDev& g, const int32_t* label, int32_t* cluster, GraphDev* out,
                    hipStream_t s) {
  const int32_t n = g.n;
  const int64_t nnz = g.nnz;
  DevBuf present, rank, flag, pos, keys, vals, head, hpos, wsum, rowcnt, rp64;
  MM_TRY(present.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(rank.alloc(sizeof(int64_t) * (size_t)(n + 1), s));
  MM_TRY(hipMemsetAsync(present.p, 0, sizeof(int32_t) * (size_t)n, s));
  k_mark<<<nblk(n), 256, 0, s>>>(n, label, present.as<int32_t>());
  MM_TRY(scan_excl_i32(present.as<int32_t>(), rank.as<int64_t>(), n, s));
  int64_t nc = 0;
  MM_TRY(hipMemcpyAsync(&nc, rank.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  out->n = (int32_t)nc;
  MM_TRY(out->b_c.alloc(sizeof(int32_t) * (size_t)nc, s));
  out->c = out->b_c.as<int32_t>();
  MM_TRY(hipMemsetAsync(out->c, 0, sizeof(int32_t) * (size_t)nc, s));
  k_cluster<<<nblk(n), 256, 0, s>>>(n, label, rank.as<int64_t>(), g.c, cluster, out->c);
  MM_TRY(flag.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1), s));
  MM_TRY(pos.alloc(sizeof(int64_t) * (size_t)(nnz + 1), s));
  k_cut_flags<<<n, 128, 0, s>>>(n, g.row_ptr, g.col, cluster, flag.as<int32_t>());
  MM_TRY(scan_excl_i32(flag.as<int32_t>(), pos.as<int64_t>(), nnz, s));
  int64_t m = 0;
  MM_TRY(hipMemcpyAsync(&m, pos.as<int64_t>() + nnz, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  MM_TRY(keys.alloc(sizeof(uint64_t) * (size_t)std::max<int64_t>(m, 1), s));
  MM_TRY(vals.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1), s));
  k_cut_emit<<<n, 128, 0, s>>>(n, g.row_ptr, g.col, g.w, cluster, pos.as<int64_t>(), nc,
                               keys.as<uint64_t>(), vals.as<int32_t>());
  MM_TRY(hipGetLastError());
  int kb = 1;
  while ((1ull << kb) < (uint64_t)nc * (uint64_t)nc) kb++;
  MM_TRY(radix_sort_pairs(keys.as<uint64_t>(), vals.as<int32_t>(), m, kb, s));
  MM_TRY(head.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1), s));
  MM_TRY(hpos.alloc(sizeof(int64_t) * (size_t)(m + 1), s));
  MM_TRY(wsum.alloc(sizeof(int64_t) * (size_t)(m + 1), s));
  k_heads<<<nblk(m), 256, 0, s>>>(m, keys.as<uint64_t>(), head.as<int32_t>());
  MM_TRY(scan_excl_i32(head.as<int32_t>(), hpos.as<int64_t>(), m, s));
  MM_TRY(scan_excl_i32(vals.as<int32_t>(), wsum.as<int64_t>(), m, s));
  int64_t cnnz = 0;
  MM_TRY(hipMemcpyAsync(&cnnz, hpos.as<int64_t>() + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  out->nnz = cnnz;
  MM_TRY(out->b_col.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(cnnz, 1), s));
  MM_TRY(out->b_w.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(cnnz, 1), s));
  MM_TRY(out->b_rp.alloc(sizeof(int32_t) * (size_t)(nc + 1), s));
  out->col = out->b_col.as<int32_t>();
  out->w = out->b_w.as<int32_t>();
  out->row_ptr = out->b_rp.as<int32_t>();
  MM_TRY(rowcnt.alloc(sizeof(int32_t) * (size_t)nc, s));
  MM_TRY(hipMemsetAsync(rowcnt.p, 0, sizeof(int32_t) * (size_t)nc, s));
  k_coarse_edges<<<nblk(m), 256, 0, s>>>(m, keys.as<uint64_t>(), head.as<int32_t>(),
                                         hpos.as<int64_t>(), wsum.as<int64_t>(), nc, out->col,
                                         out->w, rowcnt.as<int32_t>());
  MM_TRY(rp64.alloc(sizeof(int64_t) * (size_t)(nc + 1), s));
  MM_TRY(scan_excl_i32(rowcnt.as<int32_t>(), rp64.as<int64_t>(), nc, s));
  k_i64_to_i32<<<nblk(nc + 1), 256, 0, s>>>(nc + 1, rp64.as<int64_t>(), out->row_ptr);
  return hipGetLastError();
}

}  // namespace mm
