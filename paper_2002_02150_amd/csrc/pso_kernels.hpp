// pso_kernels.hpp -- lbest particle swarm (Sec. III) on the device.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcas {

struct PsoDev {
  int32_t n_runs, n_particles, n_iter;
  double w0, w1, c1, c2, vmax;
  uint64_t seed;
  double lo[4], span[4];     // theta = lo + x * span
  double* x;
  double* v;
  double* pbest_x;
  double* pbest_f;
  int32_t* pbest_j;
  double* best_x;
  double* best_f;
  int32_t* best_j;
  int32_t* iteration;
};

hipError_t launch_pso_init(const PsoDev& p, double* theta_out, hipStream_t s);
hipError_t launch_pso_step(const PsoDev& p, const double* fitness, const int32_t* argmax, double* theta_next,
                           hipStream_t s);
hipError_t launch_pso_best(const PsoDev& p, int runs_per_group, int runs_used, double* out_f, double* out_theta,
                           int32_t* out_j, int32_t* out_run, hipStream_t s);

}  // namespace fcas
