// setup.hip -- per-point set-up kernel, counters, and segment preparation.
#include "launch.hpp"

namespace fcas {

__global__ void k_zero_i32(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

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

// Eight lanes per point: status, plan list entry, and the FP64 set-up, the
// per-detector work spread over the lanes.  With build_lists = 0 only the
// descriptors are refreshed (the work lists and their counts are left
// alone).  List entries of one wavefront that share a plan are appended with
// a single atomic.
__global__ void __launch_bounds__(64) k_setup(const NetDesc* __restrict__ netp, const SegDesc* __restrict__ segs,
                                              const double* __restrict__ theta, const int32_t* __restrict__ seg_ids,
                                              int n, EvalDesc* __restrict__ evals, int32_t* __restrict__ lists,
                                              int32_t* __restrict__ counts, int list_stride, int build_lists,
                                              int32_t* __restrict__ err) {
  const int lane = threadIdx.x & 63, g = threadIdx.x & 7;
  const int e = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 3);
  const NetDesc& net = *netp;
  int plan = -1;   // on lane 0 of a group: plan of a point to append to its list, else -1
  if (e < n) {
    EvalDesc& ev = evals[e];
    const int s = seg_ids[e];
    if (s < 0 || s >= net.max_segments || !segs[s].registered) {
      if (g == 0) {
        ev.seg = s;
        ev.status = -2;
        ev.plan = 0;
        atomicOr(err, 1);
      }
    } else {
      const SegDesc& sg = segs[s];
      const double* th = theta + 4 * (int64_t)e;
      bool inside = true;
      for (int d = 0; d < 4; ++d) {
        const double t = th[d];
        inside = inside && isfinite(t) && t >= net.box_lo[d] && t <= net.box_hi[d];
      }
      if (inside) {
        double coef[4];
        SkyFrame fr;
        setup_point(net, th, coef, fr);
        if (g < net.n_det) setup_detector(net, sg, fr, g, ev);
        const int rank = setup_basis(ev, DetLanes{net.n_det, g});
        if (g == 0) {
          for (int k = 0; k < 4; ++k) ev.coef[k] = coef[k];
          ev.rank = rank;
          if (build_lists) plan = sg.plan;
        }
      }
      if (g == 0) {
        ev.seg = s;
        ev.plan = sg.plan;
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

// sigma_i^2 = 4 df sum_{k in B} f_k^(-7/3) / S^i_k  (template norm, Sec. II.D).
// One 256-thread block per detector; fixed-order tree reduction (deterministic).
__global__ void __launch_bounds__(256) k_segment_sigma(const double* __restrict__ psd, int64_t half, int k_lo,
                                                       int k_hi, double df, double* __restrict__ sigma2) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  const double* row = psd + (int64_t)i * half;
  double acc = 0.0;
  for (int k = k_lo + threadIdx.x; k <= k_hi; k += 256) {
    const double f = k * df;
    acc += pow(f, -7.0 / 3.0) / row[k];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sigma2[i] = 4.0 * df * red[0];
}

// y^i_k = 4 df x^i_k f_k^(-7/6) / (S^i_k sigma_i), stored [k - k_lo][i]
// (over-whitening once, Sec. II.D), and the per-bin basis b_k = (f_k/f*)^(-1/3).
template <typename Real>
__global__ void k_segment_prep(const double* __restrict__ xf, const double* __restrict__ psd,
                               const double* __restrict__ sigma2, int n_det, int64_t half, int k_lo, int k_hi,
                               double df, double f_star, cplx<Real>* __restrict__ y, double* __restrict__ b) {
  const int kk = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = k_lo + kk;
  if (k > k_hi) return;
  const double f = k * df;
  const double amp = 4.0 * df * pow(f, -7.0 / 6.0);
  for (int i = 0; i < n_det; ++i) {
    const int64_t o = (int64_t)i * half + k;
    const double sc = amp / (psd[o] * sqrt(sigma2[i]));
    y[(int64_t)kk * n_det + i] = mk<Real>((Real)(xf[2 * o] * sc), (Real)(xf[2 * o + 1] * sc));
  }
  b[kk] = cbrt(f_star / f);
}

hipError_t launch_zero_i32(int32_t* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_setup(const NetDesc* net, const SegDesc* segs, const double* theta, const int32_t* seg_ids,
                        int n, EvalDesc* evals, int32_t* lists, int32_t* counts, int list_stride, int build_lists,
                        int32_t* err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_setup, dim3((n + 7) / 8), dim3(64), 0, s, net, segs, theta, seg_ids, n, evals, lists,
                     counts, list_stride, build_lists, err);
  return hipGetLastError();
}

hipError_t launch_segment_sigma(const double* psd, int n_det, int64_t half, int k_lo, int k_hi, double df,
                                double* sigma2_out, hipStream_t s) {
  hipLaunchKernelGGL(k_segment_sigma, dim3(n_det), dim3(256), 0, s, psd, half, k_lo, k_hi, df, sigma2_out);
  return hipGetLastError();
}

hipError_t launch_segment_prep(int precision, const double* xf, const double* psd, const double* sigma2,
                               int n_det, int64_t half, int k_lo, int k_hi, double df, double f_star,
                               void* y_out, double* b_out, hipStream_t s) {
  const int K = k_hi - k_lo + 1;
  const dim3 grid((K + 255) / 256), block(256);
  if (precision == 0)
    hipLaunchKernelGGL(k_segment_prep<float>, grid, block, 0, s, xf, psd, sigma2, n_det, half, k_lo, k_hi, df,
                       f_star, (cplx<float>*)y_out, b_out);
  else
    hipLaunchKernelGGL(k_segment_prep<double>, grid, block, 0, s, xf, psd, sigma2, n_det, half, k_lo, k_hi, df,
                       f_star, (cplx<double>*)y_out, b_out);
  return hipGetLastError();
}

}  // namespace fcas
