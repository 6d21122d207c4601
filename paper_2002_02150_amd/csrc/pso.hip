// pso.hip -- lbest PSO kernels: one work-group per run, one thread per particle.
//
// Reading of the dynamics (Sec. III defers the equations to earlier work):
// unit-cube coordinates of the search rectangle; x0 ~ U[0,1]^4, v0 = clamp(u - x0);
// v <- w v + c1 r1 (pbest - x) + c2 r2 (lbest - x), |v| <= vmax, x <- x + v;
// w linear from w0 to w1; lbest = best personal best among ring indices
// (i-1, i, i+1), first of equal values in that order; personal bests update on
// a strictly larger fitness; particles outside the rectangle keep flying with
// fitness -inf.  Random numbers: Philox4x32-10 (Salmon et al., SC'11), key =
// seed, counter = (iteration, particle, run, stream).  All FP64 arithmetic is
// written in a fixed order without contraction into fused multiply-adds, so the
// trajectories are reproducible bit for bit.
#include "pso_kernels.hpp"

namespace fcas {

__global__ void k_pso_init(PsoDev p, double* __restrict__ theta) {
#pragma clang fp contract(off)
  const int r = blockIdx.x, i = threadIdx.x;
  if (i >= p.n_particles) return;
  const int64_t o = (int64_t)r * p.n_particles + i;
  double x[4], u[4];
  uniforms4(p.seed, 0, i, r, 0, x);
  uniforms4(p.seed, 0, i, r, 1, u);
  for (int d = 0; d < 4; ++d) {
    p.x[4 * o + d] = x[d];
    p.v[4 * o + d] = clampv(u[d] - x[d], p.vmax);
    p.pbest_x[4 * o + d] = x[d];
    theta[4 * o + d] = p.lo[d] + x[d] * p.span[d];
  }
  p.pbest_f[o] = -INFINITY;
  p.pbest_j[o] = -1;
  if (i == 0) {
    p.best_f[r] = -INFINITY;
    p.best_j[r] = -1;
    for (int d = 0; d < 4; ++d) p.best_x[4 * r + d] = 0.0;
    if (r == 0) {
      p.iteration[0] = 0;
      p.iteration[1] = 0;
    }
  }
}

__global__ void k_pso_step(PsoDev p, const double* __restrict__ fitness, const int32_t* __restrict__ argmax,
                           double* __restrict__ theta) {
  extern __shared__ double sm[];   // PsoShared: pf[P], px[P][4], then pj[P]
  const int P = p.n_particles;
  const PsoShared sh{sm, sm + P, (int32_t*)(sm + 5 * P)};
  PsoLocal L = pso_load(p, blockIdx.x, threadIdx.x);
  pso_step_run(p, L, fitness, argmax, theta, sh, nullptr, blockIdx.x, threadIdx.x);
}

// Best of the first u runs of each group of m consecutive runs (one group per
// searched segment; m = u = n_runs: the whole swarm): the largest run best,
// lowest run index on ties, mapped from unit-cube to rectangle coordinates.
// One thread per group.
__global__ void k_pso_best(PsoDev p, int m, int u, double* out_f, double* out_theta, int32_t* out_j,
                           int32_t* out_run) {
#pragma clang fp contract(off)
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= p.n_runs / m) return;
  int b = g * m;
  for (int r = b + 1; r < g * m + u; ++r)
    if (p.best_f[r] > p.best_f[b]) b = r;
  out_f[g] = p.best_f[b];
  out_j[g] = p.best_j[b];
  out_run[g] = b;
  for (int d = 0; d < 4; ++d) out_theta[4 * g + d] = p.lo[d] + p.best_x[4 * b + d] * p.span[d];
}

static int block_for(int P) { return ((P + 63) / 64) * 64; }

hipError_t launch_pso_init(const PsoDev& p, double* theta_out, hipStream_t s) {
  hipLaunchKernelGGL(k_pso_init, dim3(p.n_runs), dim3(block_for(p.n_particles)), 0, s, p, theta_out);
  return hipGetLastError();
}

hipError_t launch_pso_step(const PsoDev& p, const double* fitness, const int32_t* argmax, double* theta_next,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_pso_step, dim3(p.n_runs), dim3(block_for(p.n_particles)),
                     pso_shared_bytes(p.n_particles), s, p, fitness, argmax, theta_next);
  return hipGetLastError();
}

hipError_t launch_pso_best(const PsoDev& p, int runs_per_group, int runs_used, double* out_f, double* out_theta,
                           int32_t* out_j, int32_t* out_run, hipStream_t s) {
  const int groups = p.n_runs / runs_per_group;
  hipLaunchKernelGGL(k_pso_best, dim3((groups + 63) / 64), dim3(64), 0, s, p, runs_per_group, runs_used, out_f,
                     out_theta, out_j, out_run);
  return hipGetLastError();
}

}  // namespace fcas
