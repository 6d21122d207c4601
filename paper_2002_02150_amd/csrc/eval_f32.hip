// eval_f32.hip -- float instantiation of the FFT passes and the finalize kernel.
#include "launch.hpp"

namespace fcas {

#define FCAS_CASE_P1(id, ...)                                                                   \
  case id:                                                                                       \
    switch (a.n_det) {                                                                           \
      case 1: launch_k(k_pass1<float, PlanF##id, 1>, dim3(grid), dim3(PlanF##id::T1), s, e0, e1, a); break; \
      case 2: launch_k(k_pass1<float, PlanF##id, 2>, dim3(grid), dim3(PlanF##id::T1), s, e0, e1, a); break; \
      case 3: launch_k(k_pass1<float, PlanF##id, 3>, dim3(grid), dim3(PlanF##id::T1), s, e0, e1, a); break; \
      case 4: launch_k(k_pass1<float, PlanF##id, 4>, dim3(grid), dim3(PlanF##id::T1), s, e0, e1, a); break; \
      default: launch_k(k_pass1<float, PlanF##id, 0>, dim3(grid), dim3(PlanF##id::T1), s, e0, e1, a); break; \
    }                                                                                            \
    break;
#define FCAS_CASE_P2(id, ...)                                                              \
  case id:                                                                                  \
    launch_k(k_pass2<float, PlanF##id>, dim3(grid), dim3(PlanF##id::T2), s, e0, e1, a); \
    break;

hipError_t launch_pass1_f32(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (plan) {
    FCAS_PLAN_LIST(FCAS_CASE_P1)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define FCAS_CASE_PM(id, ...) \
  case id:                    \
    return launch_passm_plan<float, PlanF##id>(a, grid, s, e0, e1);

hipError_t launch_passm_f32(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (plan) {
    FCAS_PLAN_LIST(FCAS_CASE_PM)
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_pass2_f32(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (plan) {
    FCAS_PLAN_LIST(FCAS_CASE_P2)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define FCAS_CASE_FUSED(id, ...) \
  case id:                       \
    return launch_fused_plan<PlanF##id>(f, grid, s);
#define FCAS_CASE_OCC(id, ...) \
  case id:                     \
    return fused_occupancy_plan<PlanF##id>();

hipError_t launch_fused_f32(int plan, const FusedArgs& f, int grid, hipStream_t s) {
  switch (plan) {
    FCAS_PLAN_LIST(FCAS_CASE_FUSED)
    default:
      return hipErrorInvalidValue;
  }
}

// Work-groups of the fused kernel of `plan` that one compute unit holds at
// once (0 for three-pass plans, which have no fused kernel).
int fused_blocks_per_cu(int plan) {
  switch (plan) {
    FCAS_PLAN_LIST(FCAS_CASE_OCC)
    default:
      return 0;
  }
}

hipError_t launch_finalize_f32(const EvalDesc* evals, const SegDesc* segs, const void* part_g,
                                  const int32_t* part_j, int n, int part_stride, const int32_t* plan_parts2,
                                  int32_t* counts, unsigned long long* evaluated, double* fitness, int32_t* argmax,
                                  hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize<float>, dim3((n + 3) / 4), dim3(256), 0, s, evals, segs,
                     (const float*)part_g, part_j, n, part_stride, plan_parts2, counts, evaluated, fitness, argmax);
  return hipGetLastError();
}

}  // namespace fcas
