// setup_kernels.hpp -- the per-point set-up on the device: eight lanes per
// point, the descriptor and the append to its plan's work list.  Used by the
// set-up kernel of every fitness call and by the kernel that ends a PSO
// iteration.
#pragma once

#include "eval_kernels.hpp"

namespace fcas {

// The detectors of one point as a group of 8 lanes, lane g holding detector g;
// sums over detectors are butterfly reductions inside the group (every lane
// gets the same, order-independent total: IEEE addition commutes).
struct DetLanes {
  int n_det, g;
  template <class F> __device__ double sum(F f) const {
    double x = g < n_det ? f(g) : 0.0;
    x += __shfl_xor(x, 1, 8);
    x += __shfl_xor(x, 2, 8);
    x += __shfl_xor(x, 4, 8);
    return x;
  }
  template <class F> __device__ void each(F f) const {
    if (g < n_det) f(g);
  }
  template <class F> __device__ void all(F f) const { f(g); }
};
static_assert(kMaxDet == 8, "one lane per detector slot in a group of 8");

// What the set-up of one point reads of its segment: the segment id, whether
// it can be evaluated, and the segment's plan, bin width, pass-1 register
// stride and (lane g) detector g's template norm.
struct SetupSeg {
  int32_t s, ok, plan, dk1;
  double df, sigma_g;
};

__device__ __forceinline__ SetupSeg setup_seg_load(const NetDesc& net, const SegDesc* __restrict__ segs,
                                                   const int32_t* __restrict__ seg_ids, int e, bool valid) {
  SetupSeg q{};
  if (!valid) return q;
  q.s = seg_ids[e];
  if (q.s < 0 || q.s >= net.max_segments) return q;
  const SegDesc& sg = segs[q.s];
  q.ok = sg.registered;
  q.plan = sg.plan;
  q.dk1 = sg.dk1;
  q.df = sg.df;
  const int g = threadIdx.x & 7;
  q.sigma_g = g < net.n_det ? sg.sigma[g] : 0.0;
  return q;
}

// Set-up of point e (valid) by the 8-lane group holding it, given its segment
// (setup_seg_load) and its parameters th[4]: status, the FP64 set-up with the
// per-detector work spread over the lanes, and (build_lists) the append to
// its plan's work list.  Every lane of the wavefront calls it, lanes without
// a point with valid = false: list entries of one wavefront that share a plan
// are appended with a single atomic.
__device__ __forceinline__ void setup_group(const NetDesc& net, const SetupSeg& q, const double* th, int e,
                                            bool valid, EvalDesc* __restrict__ evals, int32_t* __restrict__ lists,
                                            int32_t* __restrict__ counts, int list_stride, int build_lists,
                                            int32_t* __restrict__ err) {
  const int lane = threadIdx.x & 63, g = threadIdx.x & 7;
  int plan = -1;   // on lane 0 of a group: plan of a point to append to its list, else -1
  if (valid) {
    EvalDesc& ev = evals[e];
    if (!q.ok) {
      if (g == 0) {
        ev.seg = q.s;
        ev.status = -2;
        ev.plan = 0;
        atomicOr(err, 1);
      }
    } else {
      bool inside = true;
      for (int d = 0; d < 4; ++d) {
        const double t = th[d];
        inside = inside && isfinite(t) && t >= net.box_lo[d] && t <= net.box_hi[d];
      }
      if (inside) {
        double coef[4];
        SkyFrame fr;
        setup_point(net, th, coef, fr);
        if (g < net.n_det) setup_detector(net, q.df, q.dk1, q.sigma_g, fr, g, ev);
        const int rank = setup_basis(ev, DetLanes{net.n_det, g});
        if (g == 0) {
          for (int k = 0; k < 4; ++k) ev.coef[k] = coef[k];
          ev.rank = rank;
          if (build_lists) plan = q.plan;
        }
      }
      if (g == 0) {
        ev.seg = q.s;
        ev.plan = q.plan;
        ev.status = inside ? 1 : 0;
      }
    }
  }
  unsigned long long todo = __ballot(plan >= 0);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lp = __shfl(plan, leader, 64);
    const unsigned long long same = __ballot(plan == lp);
    int base = 0;
    if (lane == leader) base = atomicAdd(counts + lp, __popcll(same));
    base = __shfl(base, leader, 64);
    if (plan == lp) lists[(int64_t)lp * list_stride + base + __popcll(same & ((1ull << lane) - 1))] = e;
    todo &= ~same;
  }
}

}  // namespace fcas
