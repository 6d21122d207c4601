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

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t lo0 = M0 * c[0], hi0 = __umulhi(M0, c[0]);
    const uint32_t lo1 = M1 * c[2], hi1 = __umulhi(M1, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ void uniforms4(uint64_t seed, uint32_t it, uint32_t particle, uint32_t run,
                                          uint32_t stream, double u[4]) {
  uint32_t c[4] = {it, particle, run, stream};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
#pragma unroll
  for (int d = 0; d < 4; ++d) u[d] = ((double)c[d] + 0.5) * 2.3283064365386962890625e-10;   // 2^-32
}

__device__ __forceinline__ double clampv(double v, double vmax) {
  v = v < -vmax ? -vmax : v;
  return v > vmax ? vmax : v;
}

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
#pragma clang fp contract(off)
  extern __shared__ double pf[];   // personal-best fitness of the run's particles
  const int r = blockIdx.x, i = threadIdx.x, P = p.n_particles;
  const int iter = p.iteration[0];
  const int64_t base = (int64_t)r * P;
  if (i < P) {
    const int64_t o = base + i;
    double pb = p.pbest_f[o];
    const double f = fitness[o];
    if (f > pb) {
      pb = f;
      p.pbest_f[o] = f;
      p.pbest_j[o] = argmax[o];
      for (int d = 0; d < 4; ++d) p.pbest_x[4 * o + d] = p.x[4 * o + d];
    }
    pf[i] = pb;
  }
  __syncthreads();
  if (i == 0) {
    int b = 0;
    for (int k = 1; k < P; ++k)
      if (pf[k] > pf[b]) b = k;
    if (pf[b] > p.best_f[r]) {
      p.best_f[r] = pf[b];
      p.best_j[r] = p.pbest_j[base + b];
      for (int d = 0; d < 4; ++d) p.best_x[4 * r + d] = p.pbest_x[4 * (base + b) + d];
    }
  }
  if (i < P) {
    const int cand[3] = {(i + P - 1) % P, i, (i + 1) % P};
    int lb = cand[0];
    for (int c = 1; c < 3; ++c)
      if (pf[cand[c]] > pf[lb]) lb = cand[c];
    const double w = p.n_iter <= 1 ? p.w0 : p.w0 - (p.w0 - p.w1) * ((double)iter / (double)(p.n_iter - 1));
    double r1[4], r2[4];
    uniforms4(p.seed, (uint32_t)(iter + 1), i, r, 2, r1);
    uniforms4(p.seed, (uint32_t)(iter + 1), i, r, 3, r2);
    const int64_t o = base + i, ol = base + lb;
    for (int d = 0; d < 4; ++d) {
      const double xv = p.x[4 * o + d];
      const double t0 = w * p.v[4 * o + d];
      const double t1 = (p.c1 * r1[d]) * (p.pbest_x[4 * o + d] - xv);
      const double t2 = (p.c2 * r2[d]) * (p.pbest_x[4 * ol + d] - xv);
      const double vn = clampv((t0 + t1) + t2, p.vmax);
      const double xn = xv + vn;
      p.v[4 * o + d] = vn;
      p.x[4 * o + d] = xn;
      theta[4 * o + d] = p.lo[d] + xn * p.span[d];
    }
  }
  // The iteration count advances once every run has read it: each run's
  // work-group counts itself in iteration[1] (a device-scope atomic), and the
  // last one stores count + 1 and clears the tally.
  __syncthreads();
  if (i == 0) {
    const int done = __hip_atomic_fetch_add(p.iteration + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (done == (int)gridDim.x - 1) {
      __hip_atomic_store(p.iteration + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(p.iteration, iter + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
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
                     sizeof(double) * p.n_particles, s, p, fitness, argmax, theta_next);
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
