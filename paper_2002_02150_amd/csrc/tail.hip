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
  constexpr int PM = kTailMaxParticles;
  __shared__ double s_pf[PM], s_px[4 * PM], s_theta[4 * PM];
  __shared__ int32_t s_pj[PM];
  __shared__ double s_net[(sizeof(NetDesc) + 7) / 8];
  const int r = blockIdx.x, tid = threadIdx.x, P = p.n_particles;
  const int base = r * P;
  const int k = tid >> 3;   // the particle of this thread's group of 8 lanes
  // Everything that does not depend on this iteration's fitness is read
  // first, so that its latency overlaps the finalize: the network (to LDS),
  // the particle's swarm state, and its segment's set-up fields.
  for (int w = tid; w < (int)((sizeof(NetDesc) + 7) / 8); w += blockDim.x) s_net[w] = ((const double*)t.net)[w];
  PsoLocal L = pso_load(p, r, tid);
  const SetupSeg q = t.setup ? setup_seg_load(*t.net, t.segs, t.seg_ids, base + k, k < P) : SetupSeg{};
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
  pso_step_run(p, L, t.fitness, t.argmax, t.theta, PsoShared{s_pf, s_px, s_pj}, s_theta, r, tid);
  if (!t.setup) return;
  // pso_step_run ends with a work-group barrier after its last LDS write: the
  // next positions in s_theta and the network in s_net are visible here
  const NetDesc& net = *(const NetDesc*)s_net;
  setup_group(net, q, s_theta + 4 * (k < P ? k : 0), base + k, k < P, t.evals, t.lists_next, t.counts_next,
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
