// grad.hip -- dGamma^2/dtheta at the maximising sample j* (held fixed).
//
// Gamma^2 = z^H P z with z^i = sum_k a^i_k,  a^i_k = y^i_k exp(2 pi i [Phi_k + k dly_i + k j*/N]),
// P the projector onto span(V), V = diag(sigma) U(alpha, delta).  For a
// parameter t:
//   d z^i   = 2 pi i [ sum_p (d coef_p / dt) sum_k a_k b_k^{e_p} + (d dly_i / dt) sum_k a_k k ]
//   d Gamma^2 = 2 Re[(P z)^H dz] + 2 Re[r^H dV w],   w = (V^T V)^-1 V^T z,  r = z - V w,
// the second term being z^H dP z for the derivative of an orthogonal projector.
#include "grad_kernels.hpp"

namespace fcas {

// Blocks (point, detector, part): each part sums a strided share of the
// in-band bins into six complex FP64 partial sums; the chain kernel adds the
// parts in a fixed order (deterministic).
template <typename Real>
__global__ void __launch_bounds__(256) k_adjoint_sums(const SegDesc* __restrict__ segs,
                                                      const EvalDesc* __restrict__ evals,
                                                      const int32_t* __restrict__ argmax, int n_det, int parts,
                                                      double* __restrict__ sums) {
  const int e = blockIdx.x, i = blockIdx.y, part = blockIdx.z;
  const EvalDesc& ev = evals[e];
  double* out = sums + (((int64_t)e * n_det + i) * parts + part) * kAdjSums * 2;
  if (ev.status != 1) {
    if (threadIdx.x < kAdjSums * 2) out[threadIdx.x] = 0.0;
    return;
  }
  const SegDesc& sg = segs[ev.seg];
  const int64_t N = sg.n;
  const int64_t jstar = argmax[e];
  const cplx<Real>* y = (const cplx<Real>*)sg.y;
  double acc[kAdjSums][2];
  for (int m = 0; m < kAdjSums; ++m) acc[m][0] = acc[m][1] = 0.0;
  for (int k = sg.k_lo + part * 256 + threadIdx.x; k <= sg.k_hi; k += 256 * parts) {
    const int kk = k - sg.k_lo;
    const double b = sg.b[kk];
    const double phc = common_phase(ev.coef, b);
    const double ramp = (double)(((int64_t)k * jstar) % N) / (double)N;
    const double ph = (double)k * ev.dly[i] + phc + ramp;
    const double r = ph - rint(ph);
    Real sn, cs;
    sincos_rev((Real)r, &sn, &cs);
    const cplx<Real> a = mul(y[(int64_t)kk * n_det + i], mk<Real>(cs, sn));
    const double ax = (double)a.x, ay = (double)a.y;
    const double b2 = b * b, b3 = b2 * b, b5 = b3 * b2;
    const double w[kAdjSums] = {1.0, b5, b3, b2, b, (double)k};
#pragma unroll
    for (int m = 0; m < kAdjSums; ++m) {
      acc[m][0] += w[m] * ax;
      acc[m][1] += w[m] * ay;
    }
  }
  __shared__ double red[256];
  for (int m = 0; m < kAdjSums; ++m)
    for (int c = 0; c < 2; ++c) {
      red[threadIdx.x] = acc[m][c];
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
      }
      if (threadIdx.x == 0) out[m * 2 + c] = red[0];
      __syncthreads();
    }
}

// d coef / d tau0, d coef / d tau1.5 for coef = f* (0.6 tau0, tau1, -1.5 tau1.5, 3 tau2).
__device__ void coef_derivatives(double tau0, double tau15, double fs, double dc[2][4]) {
  const double v0 = cbrt(5.0 * tau15 / (32.0 * kPi * tau0));
  const double eta = 1.0 / (8.0 * fs * tau15 * v0 * v0);
  // logarithmic derivatives of v0 and eta
  const double dlv[2] = {-1.0 / (3.0 * tau0), 1.0 / (3.0 * tau15)};
  const double dle[2] = {2.0 / (3.0 * tau0), -5.0 / (3.0 * tau15)};
  const double A1 = 5.0 / (192.0 * kPi * fs), A2 = 5.0 / (128.0 * kPi * fs);
  const double iv3 = 1.0 / (v0 * v0 * v0), iv = 1.0 / v0;
  const double B0 = 3058673.0 / 1016064.0, B1 = 5429.0 / 1008.0, B2 = 617.0 / 144.0;
  for (int q = 0; q < 2; ++q) {
    // tau1 = A1 [ (743/336) eta^-1 v0^-3 + (11/4) v0^-3 ]
    const double dtau1 = A1 * ((743.0 / 336.0) / eta * iv3 * (-dle[q] - 3.0 * dlv[q]) + 2.75 * iv3 * (-3.0 * dlv[q]));
    // tau2 = A2 [ B0 eta^-1 v0^-1 + B1 v0^-1 + B2 eta v0^-1 ]
    const double dtau2 = A2 * (B0 / eta * iv * (-dle[q] - dlv[q]) + B1 * iv * (-dlv[q]) + B2 * eta * iv * (dle[q] - dlv[q]));
    dc[q][0] = fs * (q == 0 ? 0.6 : 0.0);
    dc[q][1] = fs * dtau1;
    dc[q][2] = fs * (q == 1 ? -1.5 : 0.0);
    dc[q][3] = fs * 3.0 * dtau2;
  }
}

// One 64-thread block per point: the threads add the parts of the six sums
// (fixed order, deterministic), then thread 0 applies the chain rule in FP64.
// Per-point work arrays live in LDS rather than in per-lane scratch.
__global__ void __launch_bounds__(64) k_chain(const NetDesc* __restrict__ netp, const SegDesc* __restrict__ segs,
                                              const EvalDesc* __restrict__ evals, const double* __restrict__ theta,
                                              const double* __restrict__ sums, int parts, int n,
                                              double* __restrict__ grad) {
  const int e = blockIdx.x;
  const NetDesc& net = *netp;
  const EvalDesc& ev = evals[e];
  double* g = grad + 4 * (int64_t)e;
  if (ev.status != 1) {
    if (threadIdx.x < 4) g[threadIdx.x] = 0.0;
    return;
  }
  const int D = net.n_det;
  __shared__ double S[kMaxDet * kAdjSums * 2];
  for (int m = threadIdx.x; m < D * kAdjSums * 2; m += 64) {
    const int i = m / (kAdjSums * 2), c = m - i * (kAdjSums * 2);
    double t = 0.0;
    for (int part = 0; part < parts; ++part) t += sums[(((int64_t)e * D + i) * parts + part) * kAdjSums * 2 + c];
    S[m] = t;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const SegDesc& sg = segs[ev.seg];
  const double* th = theta + 4 * (int64_t)e;
  const double alpha = th[0], delta = th[1];
  double dc[2][4];
  coef_derivatives(th[2], th[3], net.f_star, dc);
  double sa, ca, sd, cd;
  sincos(alpha, &sa, &ca);
  sincos(delta, &sd, &cd);
  const double ex[3] = {sa, -ca, 0.0}, ey[3] = {-sd * ca, -sd * sa, cd};
  // derivatives of n, e_X = -alpha_hat, e_Y = delta_hat with respect to (alpha, delta)
  const double dn[2][3] = {{-cd * sa, cd * ca, 0.0}, {-sd * ca, -sd * sa, cd}};
  const double dex[2][3] = {{ca, sa, 0.0}, {0.0, 0.0, 0.0}};
  const double dey[2][3] = {{sd * sa, -sd * ca, 0.0}, {-cd * ca, -cd * sa, -sd}};
  __shared__ double dV[2][kMaxDet][2], ddl[2][kMaxDet];
  __shared__ double zr[kMaxDet], zi[kMaxDet], pz_r[kMaxDet], pz_i[kMaxDet], rr[kMaxDet], ri[kMaxDet];
  for (int i = 0; i < D; ++i) {
    for (int q = 0; q < 2; ++q) {
      const double* r = net.pos[i];
      ddl[q][i] = -(dn[q][0] * r[0] + dn[q][1] * r[1] + dn[q][2] * r[2]) / kC * sg.df;
      double up = 0.0, uc = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const double d = net.ten[i][a][b];
          up += d * (dex[q][a] * ex[b] + ex[a] * dex[q][b] - dey[q][a] * ey[b] - ey[a] * dey[q][b]);
          uc += d * (dex[q][a] * ey[b] + ex[a] * dey[q][b] + dey[q][a] * ex[b] + ey[a] * dex[q][b]);
        }
      dV[q][i][0] = sg.sigma[i] * up;
      dV[q][i][1] = sg.sigma[i] * uc;
    }
    zr[i] = S[(i * kAdjSums + 0) * 2];
    zi[i] = S[(i * kAdjSums + 0) * 2 + 1];
  }
  // P z = Q (Q^T z)
  double c0r = 0, c0i = 0, c1r = 0, c1i = 0;
  for (int i = 0; i < D; ++i) {
    c0r += ev.q[i][0] * zr[i]; c0i += ev.q[i][0] * zi[i];
    c1r += ev.q[i][1] * zr[i]; c1i += ev.q[i][1] * zi[i];
  }
  for (int i = 0; i < D; ++i) {
    pz_r[i] = ev.q[i][0] * c0r + ev.q[i][1] * c1r;
    pz_i[i] = ev.q[i][0] * c0i + ev.q[i][1] * c1i;
  }
  // w = (V^T V)^-1 V^T z (rank two only), r = z - V w
  double wr[2] = {0, 0}, wi[2] = {0, 0};
  const bool full = (ev.rank == 2);
  for (int i = 0; i < D; ++i) rr[i] = ri[i] = 0.0;
  if (full) {
    double G00 = 0, G01 = 0, G11 = 0, br0 = 0, bi0 = 0, br1 = 0, bi1 = 0;
    for (int i = 0; i < D; ++i) {
      G00 += ev.v[i][0] * ev.v[i][0];
      G01 += ev.v[i][0] * ev.v[i][1];
      G11 += ev.v[i][1] * ev.v[i][1];
      br0 += ev.v[i][0] * zr[i]; bi0 += ev.v[i][0] * zi[i];
      br1 += ev.v[i][1] * zr[i]; bi1 += ev.v[i][1] * zi[i];
    }
    const double det = G00 * G11 - G01 * G01;
    wr[0] = (G11 * br0 - G01 * br1) / det; wi[0] = (G11 * bi0 - G01 * bi1) / det;
    wr[1] = (G00 * br1 - G01 * br0) / det; wi[1] = (G00 * bi1 - G01 * bi0) / det;
    for (int i = 0; i < D; ++i) {
      rr[i] = zr[i] - (ev.v[i][0] * wr[0] + ev.v[i][1] * wr[1]);
      ri[i] = zi[i] - (ev.v[i][0] * wi[0] + ev.v[i][1] * wi[1]);
    }
  }
  const double twopi = 2.0 * kPi;
  for (int q = 0; q < 4; ++q) {
    double acc = 0.0;
    for (int i = 0; i < D; ++i) {
      // d z^i = 2 pi i * s, s = sum_p dcoef_p S_p + ddly S_k
      double sr = 0.0, si = 0.0;
      if (q >= 2) {
        for (int p = 0; p < 4; ++p) {
          sr += dc[q - 2][p] * S[(i * kAdjSums + 1 + p) * 2];
          si += dc[q - 2][p] * S[(i * kAdjSums + 1 + p) * 2 + 1];
        }
      } else {
        sr = ddl[q][i] * S[(i * kAdjSums + 5) * 2];
        si = ddl[q][i] * S[(i * kAdjSums + 5) * 2 + 1];
      }
      const double dzr = -twopi * si, dzi = twopi * sr;
      // 2 Re(conj(Pz_i) dz_i)
      acc += 2.0 * (pz_r[i] * dzr + pz_i[i] * dzi);
      if (q < 2 && full) {
        // 2 Re(conj(r_i) (dV_i0 w_0 + dV_i1 w_1))
        const double tr = dV[q][i][0] * wr[0] + dV[q][i][1] * wr[1];
        const double ti = dV[q][i][0] * wi[0] + dV[q][i][1] * wi[1];
        acc += 2.0 * (rr[i] * tr + ri[i] * ti);
      }
    }
    g[q] = acc;
  }
}

// Polish trials: theta_t = theta + step_frac 2^-t w^2 g / |w g|, t = 0..T-1
// (w = widths of the search rectangle), same segment as the point.
__global__ void k_polish_trials(const double* __restrict__ theta, const double* __restrict__ grad,
                                const int32_t* __restrict__ seg, const NetDesc* __restrict__ netp, int n, int trials,
                                double step_frac, double* __restrict__ cand, int32_t* __restrict__ cand_seg) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const NetDesc& net = *netp;
  double w[4], nrm = 0.0;
  for (int d = 0; d < 4; ++d) {
    w[d] = net.box_hi[d] - net.box_lo[d];
    nrm += (w[d] * grad[4 * e + d]) * (w[d] * grad[4 * e + d]);
  }
  nrm = sqrt(nrm);
  double s = step_frac;
  for (int t = 0; t < trials; ++t) {
    const int64_t o = (int64_t)e * trials + t;
    for (int d = 0; d < 4; ++d)
      cand[4 * o + d] = theta[4 * e + d] + (nrm > 0.0 ? s * w[d] * w[d] * grad[4 * e + d] / nrm : 0.0);
    cand_seg[o] = seg[e];
    s *= 0.5;
  }
}

// Moves each point to its best trial if that raises the fitness.
__global__ void k_polish_select(double* __restrict__ theta, double* __restrict__ fitness,
                                int32_t* __restrict__ argmax, const double* __restrict__ cand,
                                const double* __restrict__ cand_f, const int32_t* __restrict__ cand_j, int n,
                                int trials) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  int best = -1;
  double fb = fitness[e];
  for (int t = 0; t < trials; ++t) {
    const double f = cand_f[(int64_t)e * trials + t];
    if (f > fb) {
      fb = f;
      best = t;
    }
  }
  if (best >= 0) {
    const int64_t o = (int64_t)e * trials + best;
    for (int d = 0; d < 4; ++d) theta[4 * e + d] = cand[4 * o + d];
    fitness[e] = fb;
    argmax[e] = cand_j[o];
  }
}

hipError_t launch_polish_trials(const double* theta, const double* grad, const int32_t* seg, const NetDesc* net,
                                int n, int trials, double step_frac, double* cand, int32_t* cand_seg,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_polish_trials, dim3((n + 63) / 64), dim3(64), 0, s, theta, grad, seg, net, n, trials,
                     step_frac, cand, cand_seg);
  return hipGetLastError();
}

hipError_t launch_polish_select(double* theta, double* fitness, int32_t* argmax, const double* cand,
                                const double* cand_f, const int32_t* cand_j, int n, int trials, hipStream_t s) {
  hipLaunchKernelGGL(k_polish_select, dim3((n + 63) / 64), dim3(64), 0, s, theta, fitness, argmax, cand, cand_f,
                     cand_j, n, trials);
  return hipGetLastError();
}

int grad_parts(int n, int n_det) {
  // enough blocks to cover the chip for small batches, one part for large ones
  int parts = (kAdjMinBlocks + n * n_det - 1) / (n * n_det);
  return parts < 1 ? 1 : (parts > kAdjMaxParts ? kAdjMaxParts : parts);
}

int alloc_grad_buffers(GradBuffers& g, int max_batch, int n_det) {
  g.max_batch = max_batch;
  g.n_det = n_det;
  // n * n_det * parts <= n * n_det + kAdjMinBlocks for every n
  const size_t entries = (size_t)max_batch * n_det + kAdjMinBlocks + kAdjMaxParts;
  const size_t bytes = entries * kAdjSums * 2 * sizeof(double);
  if (hipMalloc((void**)&g.sums, bytes) != hipSuccess) {
    g.sums = nullptr;
    return -5;
  }
  return 0;
}

void free_grad_buffers(GradBuffers& g) {
  if (g.sums) hipFree(g.sums);
  g.sums = nullptr;
}

hipError_t launch_gradient(int precision, const GradBuffers& g, const NetDesc* net, const SegDesc* segs,
                           const EvalDesc* evals, const double* theta, const int32_t* argmax, int n, int n_det,
                           double* grad, hipStream_t s) {
  const int parts = grad_parts(n, n_det);
  const dim3 grid(n, n_det, parts);
  if (precision == 0)
    hipLaunchKernelGGL(k_adjoint_sums<float>, grid, dim3(256), 0, s, segs, evals, argmax, n_det, parts, g.sums);
  else
    hipLaunchKernelGGL(k_adjoint_sums<double>, grid, dim3(256), 0, s, segs, evals, argmax, n_det, parts, g.sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chain, dim3(n), dim3(64), 0, s, net, segs, evals, theta, g.sums, parts, n, grad);
  return hipGetLastError();
}

}  // namespace fcas
