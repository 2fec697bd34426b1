// Batched layout of many independent graphs: the graphs of a batch are held
// as one block-diagonal union (graph g owns vertices [goff[g], goff[g+1])),
// so every kernel of the single-graph path runs once per step for the whole
// batch.  What is per graph lives here: relative change of each graph,
// each graph's alpha schedule as a device-side state machine (no host round
// trip per graph), graph offsets after a contraction, and the extraction of
// the graphs that keep coarsening into the next level's union.
#include "common.hpp"
#include "kernels.hpp"

namespace mm {
namespace {

inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

// gid[v] = g for v in [goff[g], goff[g+1]) (block per graph).
__global__ void k_fill_gid(const int32_t* __restrict__ goff, int32_t* __restrict__ gid) {
  const int32_t g = blockIdx.x;
  for (int32_t v = goff[g] + threadIdx.x; v < goff[g + 1]; v += blockDim.x) gid[v] = g;
}

// Largest node weight of each graph (block per graph).
__global__ void k_seg_max(const int32_t* __restrict__ goff, const int32_t* __restrict__ c,
                          int32_t* __restrict__ out) {
  const int32_t g = blockIdx.x;
  int32_t m = 1;
  for (int32_t v = goff[g] + threadIdx.x; v < goff[g + 1]; v += blockDim.x) m = max(m, c[v]);
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  __shared__ int32_t sh[4];
  if (lane_id() == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[g] = max(max(sh[0], sh[1]), max(sh[2], sh[3]));
}

// Per graph: sum |x' - x|^2 and sum |x|^2 in FP64 (block per graph, fixed
// order: strided thread sums, then a fixed tree).
__global__ __launch_bounds__(256) void k_seg_delta(const int32_t* __restrict__ goff,
                                                   const float2* __restrict__ x,
                                                   const float2* __restrict__ xn,
                                                   double2* __restrict__ out,
                                                   int32_t* __restrict__ zero2) {
  const int32_t g = blockIdx.x;
  // counters of the following schedule step start at zero (a kernel rather
  // than a memset: this sequence is replayed from HIP graphs)
  if (zero2 && g == 0 && threadIdx.x < 2) zero2[threadIdx.x] = 0;
  double a = 0.0, b = 0.0;
  for (int32_t v = goff[g] + threadIdx.x; v < goff[g + 1]; v += 256) {
    const float2 p = x[v], q = xn[v];
    const double ex = (double)q.x - p.x, ey = (double)q.y - p.y;
    a += ex * ex + ey * ey;
    b += (double)p.x * p.x + (double)p.y * p.y;
  }
  __shared__ double sa[256], sb[256];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sa[threadIdx.x] += sa[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[g] = make_double2(sa[0], sb[0]);
}

// The alpha schedule of Section 3.2 per graph, one step after an iteration
// with relative change delta:
//   rounds (alpha > alpha_min): after `a` iterations or when delta < eps_round,
//     alpha := max(decay * alpha, alpha_min);
//   final phase (alpha_min): until delta < eps_final or max_final iterations.
// Returns the alpha of the next iteration (-1 once finished); counters[0]
// counts the graphs still iterating, counters[1] those with a non-finite
// layout.
__device__ float sched_step(const double2 d, const BatchSched& prm, BatchState* __restrict__ sp,
                            int32_t* __restrict__ counters) {
  BatchState S = *sp;
  if (S.phase >= 2) return -1.f;
  const double delta = d.y > 0.0 ? sqrt(d.x / d.y) : INFINITY;
  S.delta = delta;
  S.iters++;
  if (!isfinite(delta)) {
    S.phase = 3;
    atomicAdd(&counters[1], 1);
  } else if (S.phase == 0) {
    S.k++;
    if (delta < prm.eps_round || S.k >= prm.a) {
      S.alpha = fmax(S.alpha * prm.decay, prm.alpha_min);
      S.k = 0;
      if (!(S.alpha > prm.alpha_min)) S.phase = prm.max_final > 0 ? 1 : 2;
    }
  } else {
    S.k++;
    S.final_iters++;
    if (delta < prm.eps_final) {
      S.phase = 2;
    } else if (S.k >= prm.max_final) {
      S.phase = 2;
      S.cap_hit = 1;
    }
  }
  *sp = S;
  if (S.phase < 2) atomicAdd(&counters[0], 1);
  return S.phase == 0 ? (float)S.alpha : S.phase == 1 ? (float)prm.alpha_min : -1.f;
}
__global__ void k_schedule(int32_t M, const double2* __restrict__ gd, BatchSched prm,
                           BatchState* __restrict__ st, float* __restrict__ galpha,
                           int32_t* __restrict__ counters) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M) return;
  galpha[g] = sched_step(gd[g], prm, &st[g], counters);
}
// One graph (single layouts): the counters start at zero here (a kernel, not
// a memset: the step is replayed from HIP graphs).
__global__ void k_schedule_one(const double2* __restrict__ d, BatchSched prm,
                               BatchState* __restrict__ st, float* __restrict__ alpha,
                               int32_t* __restrict__ counters) {
  counters[0] = 0;
  counters[1] = 0;
  alpha[0] = sched_step(d[0], prm, st, counters);
}

__global__ void k_sched_init(int32_t M, BatchSched prm, double alpha_start,
                             BatchState* __restrict__ st, float* __restrict__ galpha) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= M) return;
  BatchState S;
  S.alpha = alpha_start;
  S.phase = alpha_start > prm.alpha_min ? 0 : (prm.max_final > 0 ? 1 : 2);
  S.k = 0;
  S.iters = 0;
  S.final_iters = 0;
  S.cap_hit = 0;
  S.delta = 0.0;
  st[g] = S;
  galpha[g] = S.phase == 0 ? (float)S.alpha : S.phase == 1 ? (float)prm.alpha_min : -1.f;
}

// Graph of every coarse vertex (all members of a cluster share it).
__global__ void k_coarse_gid(int32_t n, const int32_t* __restrict__ cluster,
                             const int32_t* __restrict__ gid, int32_t* __restrict__ gidc) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) gidc[cluster[v]] = gid[v];
}
// goffc[g] = first coarse vertex of graph >= g (coarse ids are graph-major).
__global__ void k_offsets(int32_t M, int32_t nc, const int32_t* __restrict__ gidc,
                          int32_t* __restrict__ goffc) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g > M) return;
  int32_t lo = 0, hi = nc;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (gidc[mid] < g) lo = mid + 1; else hi = mid;
  }
  goffc[g] = lo;
}

// Subset of a union: vertices of kept graphs, renumbered in order.
__global__ void k_vkeep(int32_t n, const int32_t* __restrict__ gid, const uint8_t* __restrict__ keep,
                        const int32_t* __restrict__ rp, int32_t* __restrict__ flag,
                        int32_t* __restrict__ deg) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const bool k = keep[gid[v]] != 0;
  flag[v] = k ? 1 : 0;
  deg[v] = k ? rp[v + 1] - rp[v] : 0;
}
__global__ void k_subset_rows(int32_t n, const int32_t* __restrict__ flag,
                              const int64_t* __restrict__ newid, const int64_t* __restrict__ epos,
                              const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                              const int32_t* __restrict__ c, const int32_t* __restrict__ w,
                              int32_t* __restrict__ rp2, int32_t* __restrict__ col2,
                              int32_t* __restrict__ c2, int32_t* __restrict__ w2) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || !flag[v]) return;
  const int32_t u = (int32_t)newid[v];
  const int64_t o = epos[v];
  rp2[u] = (int32_t)o;
  if (c2) c2[u] = c ? c[v] : 1;
  for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
    col2[o + (e - rp[v])] = (int32_t)newid[col[e]];
    if (w2) w2[o + (e - rp[v])] = w ? w[e] : 1;
  }
}
__global__ void k_set_last(int32_t* rp2, int32_t n2, const int64_t* __restrict__ epos, int32_t n) {
  rp2[n2] = (int32_t)epos[n];
}
// Map of fine vertices to the next level: -1 when their graph stops here.
__global__ void k_cl_map(int32_t n, const int32_t* __restrict__ cluster,
                         const int32_t* __restrict__ cflag, const int64_t* __restrict__ cnewid,
                         int32_t* __restrict__ cl) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t C = cluster[v];
  cl[v] = cflag[C] ? (int32_t)cnewid[C] : -1;
}

}  // namespace

hipError_t batch_fill_gid(int32_t M, const int32_t* goff, int32_t* gid, hipStream_t s) {
  if (M > 0) k_fill_gid<<<M, 256, 0, s>>>(goff, gid);
  return hipGetLastError();
}

hipError_t batch_max_c(int32_t M, const int32_t* goff, const int32_t* c, int32_t* out,
                       hipStream_t s) {
  k_seg_max<<<M, 256, 0, s>>>(goff, c, out);
  return hipGetLastError();
}

hipError_t batch_delta(int32_t M, const int32_t* goff, const float* x, const float* xn,
                       double* out, hipStream_t s, int32_t* zero2) {
  k_seg_delta<<<M, 256, 0, s>>>(goff, (const float2*)x, (const float2*)xn, (double2*)out, zero2);
  return hipGetLastError();
}

hipError_t batch_sched_init(int32_t M, const BatchSched& prm, double alpha_start, BatchState* st,
                            float* galpha, hipStream_t s) {
  k_sched_init<<<nb256(M), 256, 0, s>>>(M, prm, alpha_start, st, galpha);
  return hipGetLastError();
}

hipError_t batch_schedule(int32_t M, const double* gd, const BatchSched& prm, BatchState* st,
                          float* galpha, int32_t* counters, hipStream_t s) {
  k_schedule<<<nb256(M), 256, 0, s>>>(M, (const double2*)gd, prm, st, galpha, counters);
  return hipGetLastError();
}

hipError_t schedule_one(const double* d2, const BatchSched& prm, BatchState* st, float* alpha,
                        int32_t* counters, hipStream_t s) {
  k_schedule_one<<<1, 1, 0, s>>>(reinterpret_cast<const double2*>(d2), prm, st, alpha, counters);
  return hipGetLastError();
}

hipError_t batch_coarse_offsets(int32_t n, int32_t M, int32_t nc, const int32_t* cluster,
                                const int32_t* gid, int32_t* gidc, int32_t* goffc, hipStream_t s) {
  k_coarse_gid<<<nb256(n), 256, 0, s>>>(n, cluster, gid, gidc);
  k_offsets<<<nb256(M + 1), 256, 0, s>>>(M, nc, gidc, goffc);
  return hipGetLastError();
}

hipError_t batch_subset(const GraphDev& g, const int32_t* gid, const uint8_t* keep, GraphDev* out,
                        int32_t* flag, int64_t* newid, hipStream_t s) {
  const int32_t n = g.n;
  DevBuf deg, epos;
  MM_TRY(deg.alloc(sizeof(int32_t) * (size_t)n, s));
  MM_TRY(epos.alloc(sizeof(int64_t) * (size_t)(n + 1), s));
  k_vkeep<<<nb256(n), 256, 0, s>>>(n, gid, keep, g.row_ptr, flag, deg.as<int32_t>());
  MM_TRY(hipGetLastError());
  MM_TRY(scan_excl_i32(flag, newid, n, s));
  MM_TRY(scan_excl_i32(deg.as<int32_t>(), epos.as<int64_t>(), n, s));
  int64_t cnt[2];
  MM_TRY(hipMemcpyAsync(&cnt[0], newid + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipMemcpyAsync(&cnt[1], epos.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MM_TRY(hipStreamSynchronize(s));
  const int32_t n2 = (int32_t)cnt[0];
  const int64_t m2 = cnt[1];
  out->n = n2;
  out->nnz = m2;
  MM_TRY(out->b_rp.alloc(sizeof(int32_t) * (size_t)(n2 + 1), s));
  MM_TRY(out->b_col.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(m2, 1), s));
  MM_TRY(out->b_c.alloc(sizeof(int32_t) * (size_t)std::max(n2, 1), s));
  MM_TRY(out->b_w.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(m2, 1), s));
  out->row_ptr = out->b_rp.as<int32_t>();
  out->col = out->b_col.as<int32_t>();
  out->c = out->b_c.as<int32_t>();
  out->w = out->b_w.as<int32_t>();
  k_subset_rows<<<nb256(n), 256, 0, s>>>(n, flag, newid, epos.as<int64_t>(), g.row_ptr, g.col, g.c,
                                         g.w, out->row_ptr, out->col, out->c, out->w);
  k_set_last<<<1, 1, 0, s>>>(out->row_ptr, n2, epos.as<int64_t>(), n);
  return hipGetLastError();
}

hipError_t batch_cl_map(int32_t n, const int32_t* cluster, const int32_t* cflag,
                        const int64_t* cnewid, int32_t* cl, hipStream_t s) {
  k_cl_map<<<nb256(n), 256, 0, s>>>(n, cluster, cflag, cnewid, cl);
  return hipGetLastError();
}

}  // namespace mm
