// setup.hip -- per-point set-up kernel, counters, and segment preparation.
#include "launch.hpp"
#include "setup_kernels.hpp"

namespace fcas {

__global__ void k_zero_i32(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Eight lanes per point (setup_group).  With build_lists = 0 only the
// descriptors are refreshed (the work lists and their counts are left alone).
__global__ void __launch_bounds__(64) k_setup(const NetDesc* __restrict__ netp, const SegDesc* __restrict__ segs,
                                              const double* __restrict__ theta, const int32_t* __restrict__ seg_ids,
                                              int n, EvalDesc* __restrict__ evals, int32_t* __restrict__ lists,
                                              int32_t* __restrict__ counts, int list_stride, int build_lists,
                                              int32_t* __restrict__ err) {
  const int e = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 3);
  const NetDesc& net = *netp;
  const SetupSeg q = setup_seg_load(net, segs, seg_ids, e, e < n);
  setup_group(net, q, theta + 4 * (int64_t)(e < n ? e : 0), e, e < n, evals, lists, counts, list_stride, build_lists,
              err);
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
