// Barnes-Hut quadtree shared by the plain and the learned far field
// (internal to libmulment).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace mm {

// Pre-order node record.  The centre of mass stays in FP64: rounding it to
// FP32 would add an absolute error of half an ulp of |x|, which dominates the
// offset to nearby targets in dense regions.
struct BHNode {
  double cx, cy;
  float mass;
  int32_t skip;
  uint32_t ox, oy;
  int32_t meta;   // depth | c << 8: c = 0 for an internal node, else the leaf's
                  // point count (kLeafCountSat and above: read mass)
  int32_t first;  // first point (sorted order)
};
constexpr int32_t kLeafCountSat = (1 << 23) - 1;

struct BoxInfo {
  double xmin, ymin, scale;
  int32_t e;
  int32_t pad;
};

// Buffers of the tree of the current coordinates (sized by n, reused).
// After bh_build_tree: codes/order/xsx/xsy/ix hold the points in (code, id)
// order, nodes[0..*counter) the pre-order node records, box the box.
struct BHWork {
  int32_t cap = 0;
  DevBuf codes, order, xsx, xsy, ix, px, py, nmask, npart, ntmp, first_at, nodes, counter, box,
      partial, statc, pparts;
  SortWork sort;
  // learned far field: per-node moments and cell records, sample offsets
  DevBuf mom, cell, ndepth, scount, soff;
  // exact far field: per-slab partial sums
  DevBuf expart;
};

template <typename T>
hipError_t ensure(DevBuf& b, size_t count, hipStream_t s) {
  size_t need = sizeof(T) * (count ? count : 1);
  if (b.bytes >= need) return hipSuccess;
  return b.alloc(need, s);
}

// Steps 1-4 of the Barnes-Hut far field: box, Morton codes, sort, nodes in
// pre-order with skip links and FP64 centres of mass.  The node count stays
// on the device (w->counter).
hipError_t bh_build_tree(BHWork* w, int32_t n, const float* xy, int64_t* nodes_out,
                         hipStream_t s, const BHSeg* seg = nullptr);

// Adds m * r_q for the offset (dx, dy); coincident points add nothing.  The
// fused forms are written out so that every kernel using this term rounds it
// the same way, whatever the compiler's contraction choices.
__device__ inline bool rq_add(float dx, float dy, float q, float m, float& fx, float& fy) {
  const float d2 = fmaf(dx, dx, dy * dy);
  if (d2 > 0.f) {
    float f = (q == 0.f) ? __builtin_amdgcn_rcpf(d2) : powf(d2, -0.5f * (q + 2.f));
    f *= m;
    fx = fmaf(dx, f, fx);
    fy = fmaf(dy, f, fy);
    return true;
  }
  return false;
}

}  // namespace mm
