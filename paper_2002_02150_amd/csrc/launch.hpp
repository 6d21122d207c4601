// launch.hpp -- host-side launchers shared by the C ABI layer (fcas_api.cpp)
// and the kernel translation units.  Every launcher only enqueues work on the
// given stream and returns the hipError_t of the launch.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "eval_kernels.hpp"

namespace fcas {

// A pass-kernel launch; with timing events (e0, e1 not null) the events are
// recorded by the kernel's own dispatch (hipExtLaunchKernel), so that they
// bracket the kernel and not the event packets around it.  Capturable code
// passes no events and takes the plain launch.
template <typename K, typename... A>
inline void launch_k(K kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0, hipEvent_t e1, A... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t s);
hipError_t launch_setup(const NetDesc* net, const SegDesc* segs, const double* theta, const int32_t* seg_ids,
                        int n, EvalDesc* evals, int32_t* lists, int32_t* counts, int list_stride, int build_lists,
                        int32_t* err, hipStream_t s);

// fused persistent schedule (float plans)
hipError_t launch_fused_f32(int plan, const FusedArgs& f, int grid, hipStream_t s);
int fused_blocks_per_cu(int plan);

// precision: 0 float, 1 double; e0 / e1: optional timing events (launch_k)
hipError_t launch_pass1(int precision, int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
hipError_t launch_passm(int precision, int plan, const PassArgs& a, int grid, hipStream_t s,   // three-pass plans
                        hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_pass2(int precision, int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
hipError_t launch_finalize(int precision, const EvalDesc* evals, const SegDesc* segs, const void* part_g,
                           const int32_t* part_j, int n, int part_stride, const int32_t* plan_parts2,
                           int32_t* counts, unsigned long long* evaluated, double* fitness, int32_t* argmax,
                           hipStream_t s);

// Per-plan launch helpers of the per-precision translation units: the middle
// pass exists only for three-pass plans, the fused kernel only for two-pass
// plans whose passes have equal work items (kFusable); asked for another plan
// they return hipErrorInvalidValue.
template <class PL>
constexpr bool kFusable = !PL::THREE && PL::T1 == PL::T2;

template <typename Real, class PL>
hipError_t launch_passm_plan(const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if constexpr (PL::THREE) {
    launch_k(k_passm<Real, PL>, dim3(grid), dim3(PL::TM), s, e0, e1, a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <class PL>
hipError_t launch_fused_plan(const FusedArgs& f, int grid, hipStream_t s) {
  if constexpr (kFusable<PL>) {
    hipLaunchKernelGGL((k_fused<float, PL>), dim3(grid), dim3(PL::T1), 0, s, f);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <class PL>
int fused_occupancy_plan() {
  int nb = 0;
  if constexpr (kFusable<PL>) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_fused<float, PL>, PL::T1, 0) != hipSuccess)
      nb = 0;
  }
  return nb;
}

// The end of one PSO iteration in one launch (tail.hip): finalize of every
// point, the swarm update, and (setup) the set-up of the next positions with
// their entries in the other work-list set.  Up to kTailMaxParticles
// particles per run (8 lanes each).
constexpr int kTailMaxParticles = 128;
constexpr int kTailMaxThreads = 8 * kTailMaxParticles;
struct TailArgs {
  const NetDesc* net;
  const SegDesc* segs;
  EvalDesc* evals;
  const void* part_g;
  const int32_t* part_j;
  int32_t part_stride;
  int32_t list_stride;
  const int32_t* plan_parts2;
  int32_t* counts_cur;           // list counts of the iteration just evaluated (cleared here)
  int32_t* lists_next;           // work lists of the next iteration, [kNumPlans][list_stride]
  int32_t* counts_next;          // their counts (zero on entry)
  unsigned long long* evaluated;
  double* fitness;
  int32_t* argmax;
  double* theta;                 // the next points, written by the update (the set-up reads its LDS copy)
  const int32_t* seg_ids;
  int32_t* err;
  int32_t setup;                 // 0: last iteration, no set-up
};
struct PsoDev;
hipError_t launch_pso_tail(int precision, const PsoDev& p, const TailArgs& t, hipStream_t s);

// segment preparation: sigma_i^2 = 4 df sum_B f^-7/3 / S, y = 4 df x f^-7/6 / (S sigma), b = (f/f*)^-1/3
hipError_t launch_segment_sigma(const double* psd, int n_det, int64_t half, int k_lo, int k_hi, double df,
                                double* sigma2_out, hipStream_t s);
hipError_t launch_segment_prep(int precision, const double* xf, const double* psd, const double* sigma2,
                               int n_det, int64_t half, int k_lo, int k_hi, double df, double f_star,
                               void* y_out, double* b_out, hipStream_t s);

// synthetic signal: params = (alpha, delta, tau0, tau1.5, psi, phi_c, cos_iota, t_c [s]);
// parts_scratch holds kInjectParts (256) partial sums
constexpr int kInjectScratch = 256;
hipError_t launch_inject(const NetDesc& net, const double* params, double snr, int64_t n_samples, int k_lo,
                         int k_hi, double df, const double* psd, double* parts_scratch, double* snr2_scratch,
                         double* xf, hipStream_t s);

}  // namespace fcas
