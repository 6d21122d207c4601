// tail.hip -- the end of one PSO iteration in one launch: the fitness of the
// run's points from their pass-2 partials (finalize), the swarm update
// (Sec. III), and the set-up of the next points with their work-list entries.
// One work-group per run, 8 lanes per particle.  Each phase runs the same
// device code as the separate finalize, pso_step and set-up kernels, so an
// iteration ends with the same fitness, swarm and descriptors bit for bit.
#include "launch.hpp"
#include "pso_kernels.hpp"
#include "setup_kernels.hpp"

namespace fcas {

template <typename Real>
__global__ void __launch_bounds__(kTailMaxThreads) k_pso_tail(PsoDev p, TailArgs t) {
  __shared__ double pf[kTailMaxParticles];
  const int r = blockIdx.x, tid = threadIdx.x, P = p.n_particles;
  const int base = r * P;
  const int k = tid >> 3;   // the particle of this thread's group of 8 lanes
  if (r == 0 && tid < kNumPlans) {
    // running total of points evaluated in this iteration (one thread per
    // plan); its list counts are cleared for the iteration after next (the
    // appends below go to the other list set)
    const int c = t.counts_cur[tid];
    t.counts_cur[tid] = 0;
    if (c) atomicAdd(t.evaluated, (unsigned long long)c);
  }
  if (k < P)
    finalize_group<Real>(t.evals[base + k], (const Real*)t.part_g, t.part_j, t.part_stride, t.plan_parts2,
                         base + k, tid & 7, t.fitness, t.argmax);
  __syncthreads();   // the run's fitness, written by its groups, is read by the swarm update
  pso_step_run(p, t.fitness, t.argmax, t.theta, pf, r, tid);
  if (!t.setup) return;
  __syncthreads();   // the next positions, written by the update, are read by the set-up
  setup_group(*t.net, t.segs, t.theta, t.seg_ids, base + k, k < P, t.evals, t.lists_next, t.counts_next,
              t.list_stride, 1, t.err);
}

hipError_t launch_pso_tail(int precision, const PsoDev& p, const TailArgs& t, hipStream_t s) {
  if (p.n_particles < 1 || p.n_particles > kTailMaxParticles) return hipErrorInvalidValue;
  int threads = ((8 * p.n_particles + 63) / 64) * 64;
  if (threads < kNumPlans) threads = ((kNumPlans + 63) / 64) * 64;   // one thread per plan count
  if (precision == 0)
    hipLaunchKernelGGL(k_pso_tail<float>, dim3(p.n_runs), dim3(threads), 0, s, p, t);
  else
    hipLaunchKernelGGL(k_pso_tail<double>, dim3(p.n_runs), dim3(threads), 0, s, p, t);
  return hipGetLastError();
}

}  // namespace fcas
