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

// A particle's swarm state as its iteration begins (read before its fitness
// is known), and the iteration count and its run's best fitness.
struct PsoLocal {
  double x[4], v[4], pbx[4];
  double pb;
  int32_t pbj;
  int32_t iter;
  double run_best;
};

__device__ __forceinline__ PsoLocal pso_load(const PsoDev& p, int r, int i) {
  PsoLocal L{};
  L.iter = p.iteration[0];
  L.run_best = p.best_f[r];
  if (i < p.n_particles) {
    const int64_t o = (int64_t)r * p.n_particles + i;
    for (int d = 0; d < 4; ++d) {
      L.x[d] = p.x[4 * o + d];
      L.v[d] = p.v[4 * o + d];
      L.pbx[d] = p.pbest_x[4 * o + d];
    }
    L.pb = p.pbest_f[o];
    L.pbj = p.pbest_j[o];
  }
  return L;
}

// LDS of one run's update: personal-best fitness pf[P], positions px[P][4]
// and samples pj[P] after this iteration's personal-best update.
struct PsoShared {
  double* pf;
  double* px;
  int32_t* pj;
};

// One iteration of run r (Sec. III), thread i of the run's work-group, from
// the state pso_load read: every thread of the work-group calls it (threads
// i >= P only synchronise).  Given the fitness and argmax of the current
// positions: personal, local and run bests, the move, and theta of the next
// positions (also to theta_lds[P][4] when not null).  The last run to finish
// advances the iteration count.
__device__ __forceinline__ void pso_step_run(const PsoDev& p, PsoLocal& L, const double* __restrict__ fitness,
                                             const int32_t* __restrict__ argmax, double* __restrict__ theta,
                                             PsoShared sh, double* theta_lds, int r, int i) {
#pragma clang fp contract(off)
  const int P = p.n_particles;
  const int iter = L.iter;
  const int64_t base = (int64_t)r * P;
  if (i < P) {
    const int64_t o = base + i;
    const double f = fitness[o];
    if (f > L.pb) {
      L.pb = f;
      L.pbj = argmax[o];
      p.pbest_f[o] = f;
      p.pbest_j[o] = L.pbj;
      for (int d = 0; d < 4; ++d) {
        L.pbx[d] = L.x[d];
        p.pbest_x[4 * o + d] = L.x[d];
      }
    }
    sh.pf[i] = L.pb;
    sh.pj[i] = L.pbj;
    for (int d = 0; d < 4; ++d) sh.px[4 * i + d] = L.pbx[d];
  }
  __syncthreads();
  if (i < 64) {
    // run best: the first particle with the largest personal best, found by
    // wavefront 0 (lane l scans particles l, l + 64, ...; then a butterfly
    // keeps the larger value, the smaller index among equal ones)
    double bv = -INFINITY;
    int b = 0x7fffffff;
    for (int k = i; k < P; k += 64)
      if (b == 0x7fffffff || sh.pf[k] > bv) {
        bv = sh.pf[k];
        b = k;
      }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off, 64);
      const int ob = __shfl_xor(b, off, 64);
      if (ob != 0x7fffffff && (b == 0x7fffffff || ov > bv || (ov == bv && ob < b))) {
        bv = ov;
        b = ob;
      }
    }
    if (i == 0 && sh.pf[b] > L.run_best) {
      p.best_f[r] = sh.pf[b];
      p.best_j[r] = sh.pj[b];
      for (int d = 0; d < 4; ++d) p.best_x[4 * r + d] = sh.px[4 * b + d];
    }
  }
  if (i < P) {
    const int cand[3] = {(i + P - 1) % P, i, (i + 1) % P};
    int lb = cand[0];
    for (int c = 1; c < 3; ++c)
      if (sh.pf[cand[c]] > sh.pf[lb]) lb = cand[c];
    const double w = p.n_iter <= 1 ? p.w0 : p.w0 - (p.w0 - p.w1) * ((double)iter / (double)(p.n_iter - 1));
    double r1[4], r2[4];
    uniforms4(p.seed, (uint32_t)(iter + 1), i, r, 2, r1);
    uniforms4(p.seed, (uint32_t)(iter + 1), i, r, 3, r2);
    const int64_t o = base + i;
    for (int d = 0; d < 4; ++d) {
      const double xv = L.x[d];
      const double t0 = w * L.v[d];
      const double t1 = (p.c1 * r1[d]) * (L.pbx[d] - xv);
      const double t2 = (p.c2 * r2[d]) * (sh.px[4 * lb + d] - xv);
      const double vn = clampv((t0 + t1) + t2, p.vmax);
      const double xn = xv + vn;
      p.v[4 * o + d] = vn;
      p.x[4 * o + d] = xn;
      const double th = p.lo[d] + xn * p.span[d];
      theta[4 * o + d] = th;
      if (theta_lds) theta_lds[4 * i + d] = th;
    }
  }
  // The iteration count advances once every run has read it: each run's
  // work-group counts itself in iteration[1] (a device-scope atomic), and the
  // last one stores count + 1 and clears the tally.
  __syncthreads();
  if (i == 0) {
    const int done = __hip_atomic_fetch_add(p.iteration + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (done == p.n_runs - 1) {
      __hip_atomic_store(p.iteration + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(p.iteration, iter + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// LDS bytes of one run's update (PsoShared) for P particles.
constexpr size_t pso_shared_bytes(int P) { return (size_t)P * (sizeof(double) * 5 + sizeof(int32_t)); }

hipError_t launch_pso_init(const PsoDev& p, double* theta_out, hipStream_t s);
hipError_t launch_pso_step(const PsoDev& p, const double* fitness, const int32_t* argmax, double* theta_next,
                           hipStream_t s);
hipError_t launch_pso_best(const PsoDev& p, int runs_per_group, int runs_used, double* out_f, double* out_theta,
                           int32_t* out_j, int32_t* out_run, hipStream_t s);

}  // namespace fcas
