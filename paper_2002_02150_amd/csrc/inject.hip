// inject.hip -- adds a restricted-2PN SPA signal to raw one-sided Fourier data
// (synthetic inputs: the H1 data model of Sec. II, eq. detresponse, with the
// polarisation waveforms of Sec. II.B), scaled to a network SNR (eq. optimalSNR).
//
// h^i_k = [F+^i A+ - i Fx^i Ax] f_k^-7/6 exp(-2 pi i [Phi_k + f_k (t_c + Delta^i)]) e^{i (phi_c + pi/4)}
// on the in-band bins, F(psi) = U(psi = 0) rotated by 2 psi, A+ = (1 + cos^2 iota)/2, Ax = cos iota.
#include "launch.hpp"

namespace fcas {

struct InjectArgs {
  NetDesc net;
  double theta[4];
  double psi, phi_c, cos_iota, t_c, snr;
  int64_t half;
  int k_lo, k_hi;
  double df;
};

__device__ void injection_bin(const InjectArgs& a, const EvalDesc& ev, int k, int i, double* re, double* im) {
  const double f = k * a.df;
  const double b = cbrt(a.net.f_star / f);
  const double ph = common_phase(ev.coef, b) + (double)k * ev.dly[i] + f * a.t_c;   // cycles
  const double r = ph - rint(ph);
  double s, c;
  sincospi(-2.0 * r, &s, &c);                 // exp(-2 pi i r)
  double s0, c0;
  sincos(a.phi_c + 0.25 * kPi, &s0, &c0);     // exp(i (phi_c + pi/4))
  double s2, c2;
  sincos(2.0 * a.psi, &s2, &c2);
  const double up = ev.v[i][0], uc = ev.v[i][1];   // U (sigma = 1 in the set-up below)
  const double fp = up * c2 + uc * s2, fc = -up * s2 + uc * c2;
  const double ap = 0.5 * (1.0 + a.cos_iota * a.cos_iota), ac = a.cos_iota;
  // (fp ap - i fc ac) * amp * (c + i s) * (c0 + i s0)
  const double amp = pow(f, -7.0 / 6.0);
  const double pr = c * c0 - s * s0, pi_ = c * s0 + s * c0;
  *re = amp * (fp * ap * pr + fc * ac * pi_);
  *im = amp * (fp * ap * pi_ - fc * ac * pr);
}

__device__ void injection_setup(const InjectArgs& a, EvalDesc& ev) {
  SegDesc sg{};
  sg.df = a.df;
  for (int i = 0; i < kMaxDet; ++i) sg.sigma[i] = 1.0;
  setup_one(a.net, sg, a.theta, ev);
}

// Fixed-order tree sum of one value per thread of a 256-thread block.
__device__ double block_sum256(double x, double* red) {
  red[threadIdx.x] = x;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// Network SNR^2 of the unit-amplitude signal, sum_i 4 df sum_B |h|^2 / S, in
// two fixed-order stages (deterministic): thread t of block b sums the bins
// k_lo + 256 b + t + m 256 kInjectParts (m = 0, 1, ...) of every detector,
// the block's tree sum goes to parts[b], then one block adds the parts.
constexpr int kInjectParts = 256;
static_assert(kInjectParts == kInjectScratch, "the context's scratch holds one partial per block");

__global__ void __launch_bounds__(256) k_inject_norm_parts(InjectArgs a, const double* __restrict__ psd,
                                                           double* __restrict__ parts) {
  __shared__ double red[256];
  __shared__ EvalDesc ev;
  if (threadIdx.x == 0) injection_setup(a, ev);
  __syncthreads();
  double acc = 0.0;
  const int stride = kInjectParts * 256;
  for (int i = 0; i < a.net.n_det; ++i)
    for (int k = a.k_lo + blockIdx.x * 256 + threadIdx.x; k <= a.k_hi; k += stride) {
      double re, im;
      injection_bin(a, ev, k, i, &re, &im);
      acc += (re * re + im * im) / psd[(int64_t)i * a.half + k];
    }
  const double t = block_sum256(acc, red);
  if (threadIdx.x == 0) parts[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_inject_norm(InjectArgs a, const double* __restrict__ parts,
                                                     double* __restrict__ snr2) {
  __shared__ double red[256];
  static_assert(kInjectParts == 256, "one part per thread");
  const double t = block_sum256(parts[threadIdx.x], red);
  if (threadIdx.x == 0) snr2[0] = 4.0 * a.df * t;
}

__global__ void k_inject_add(InjectArgs a, const double* __restrict__ snr2, double* __restrict__ xf) {
  const int k = a.k_lo + blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  __shared__ EvalDesc ev;
  if (threadIdx.x == 0) injection_setup(a, ev);
  __syncthreads();
  if (k > a.k_hi) return;
  const double scale = a.snr > 0 ? a.snr / sqrt(snr2[0]) : 1.0;
  double re, im;
  injection_bin(a, ev, k, i, &re, &im);
  const int64_t o = (int64_t)i * a.half + k;
  xf[2 * o] += scale * re;
  xf[2 * o + 1] += scale * im;
}

hipError_t launch_inject(const NetDesc& net, const double* params, double snr, int64_t n_samples, int k_lo,
                         int k_hi, double df, const double* psd, double* parts_scratch, double* snr2_scratch,
                         double* xf, hipStream_t s) {
  InjectArgs a{};
  a.net = net;
  for (int d = 0; d < 4; ++d) a.theta[d] = params[d];
  a.psi = params[4];
  a.phi_c = params[5];
  a.cos_iota = params[6];
  a.t_c = params[7];
  a.snr = snr;
  a.half = n_samples / 2 + 1;
  a.k_lo = k_lo;
  a.k_hi = k_hi;
  a.df = df;
  hipLaunchKernelGGL(k_inject_norm_parts, dim3(kInjectParts), dim3(256), 0, s, a, psd, parts_scratch);
  hipLaunchKernelGGL(k_inject_norm, dim3(1), dim3(256), 0, s, a, parts_scratch, snr2_scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int K = k_hi - k_lo + 1;
  hipLaunchKernelGGL(k_inject_add, dim3((K + 255) / 256, net.n_det), dim3(256), 0, s, a, snr2_scratch, xf);
  return hipGetLastError();
}

}  // namespace fcas
