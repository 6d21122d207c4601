// eval_f64.hip -- double instantiation of the FFT passes and the finalize kernel.
#include "launch.hpp"

namespace fcas {

#define FCAS_CASE_P1(id, ...)                                                                   \
  case id:                                                                                       \
    switch (a.n_det) {                                                                           \
      case 1: launch_k(k_pass1<double, PlanD##id, 1>, dim3(grid), dim3(PlanD##id::T1), s, e0, e1, a); break; \
      case 2: launch_k(k_pass1<double, PlanD##id, 2>, dim3(grid), dim3(PlanD##id::T1), s, e0, e1, a); break; \
      case 3: launch_k(k_pass1<double, PlanD##id, 3>, dim3(grid), dim3(PlanD##id::T1), s, e0, e1, a); break; \
      case 4: launch_k(k_pass1<double, PlanD##id, 4>, dim3(grid), dim3(PlanD##id::T1), s, e0, e1, a); break; \
      default: launch_k(k_pass1<double, PlanD##id, 0>, dim3(grid), dim3(PlanD##id::T1), s, e0, e1, a); break; \
    }                                                                                            \
    break;
#define FCAS_CASE_P2(id, ...)                                                              \
  case id:                                                                                  \
    launch_k(k_pass2<double, PlanD##id>, dim3(grid), dim3(PlanD##id::T2), s, e0, e1, a); \
    break;

hipError_t launch_pass1_f64(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (plan) {
    FCAS_PLAN_LIST(FCAS_CASE_P1)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define FCAS_CASE_PM(id, ...) \
  case id:                    \
    return launch_passm_plan<double, PlanD##id>(a, grid, s, e0, e1);

hipError_t launch_passm_f64(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (plan) {
    FCAS_PLAN_LIST(FCAS_CASE_PM)
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_pass2_f64(int plan, const PassArgs& a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  switch (plan) {
    FCAS_PLAN_LIST(FCAS_CASE_P2)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize_f64(const EvalDesc* evals, const SegDesc* segs, const void* part_g,
                                  const int32_t* part_j, int n, int part_stride, const int32_t* plan_parts2,
                                  int32_t* counts, unsigned long long* evaluated, double* fitness, int32_t* argmax,
                                  hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize<double>, dim3((n + 3) / 4), dim3(256), 0, s, evals, segs,
                     (const double*)part_g, part_j, n, part_stride, plan_parts2, counts, evaluated, fitness, argmax);
  return hipGetLastError();
}

}  // namespace fcas
