// fitness_tiles.hpp -- the two passes of the coherent-fitness evaluation, per
// work item and per thread, written once for the gfx950 kernels and the CPU
// emulator used by the tests.
//
// For one parameter point the library forms, for every in-band bin k (Sec. II.D),
//   w^i_k = y^i_k exp(2 pi i [Phi_k + k dly_i])     (template phase and the
//            detector delay as an exact frequency-domain shift, eq.
//            data_template_innprod; y already carries 4 df f^-7/6 / (S sigma))
//   W_m(k) = sum_i Q_im w^i_k,  m = 0, 1
// where the columns of Q are an orthonormal basis of span(diag(sigma) U).  By
// linearity the inverse FFTs of W_0, W_1 give a_m(j) = sum_i Q_im z^i_j, and
//   Gamma^2_j = |a_0(j)|^2 + |a_1(j)|^2 = z_j^H Q Q^T z_j,
// the log-likelihood ratio maximised over the four amplitudes (Sec. II.C).
//
// The length-N inverse FFT is a four-step transform, N = N1 N2,
//   k = k1 N2 + k2,  j = j1 + N1 j2,
//   pass 1 (per column k2): B(j1, k2) = w_N^{k2 j1} sum_{k1} W(k1 N2 + k2) w_N1^{k1 j1}
//   pass 2 (per row j1):    a(j1 + N1 j2) = sum_{k2} B(j1, k2) w_N2^{k2 j2}
// with B stored row-major [series][j1][k2] in the workspace.  Lengths too long
// for two passes insert a middle pass (see Plan below).
#pragma once

#include <stdint.h>

#include "fft_core.hpp"

namespace fcas {

constexpr int kMaxDet = 8;

// Per registered segment (device resident).
struct SegDesc {
  const void* y;        // [K][n_det] complex (float2 or double2 by precision)
  const double* b;      // [K] (f_k / f*)^(-1/3)
  int64_t n;            // samples
  int32_t k_lo, k_hi;   // inclusive in-band bins
  int32_t plan;         // FFT plan index
  int32_t registered;   // 1 once fcas_set_segment has completed
  int32_t dk1;          // the plan's pass-1 register stride in bins (P1 W1)
  int32_t reserved;
  double df;            // 1 / T
  double sigma[kMaxDet];
  int64_t j_lo, j_hi;   // coalescence samples searched: j_lo <= j < j_hi
};

// Per parameter point, written by the set-up kernel.
struct EvalDesc {
  double coef[4];             // Phi_k = coef0 b^5 + coef1 b^3 + coef2 b^2 + coef3 b (cycles)
  double dly[kMaxDet];        // Delta^i * df: delay ramp in cycles per bin
  double q[kMaxDet][2];       // orthonormal basis of span(diag(sigma) U), FP64
  float qf[kMaxDet][2];       // same, rounded to float
  double v[kMaxDet][2];       // V = diag(sigma) U (kept for the gradient)
  double step1[kMaxDet][2];   // exp(2 pi i dk1 (dly_i - dly_0)): ramp of detector i relative to
                              // detector 0 across one pass-1 register stride
  float step1f[kMaxDet][2];   // same, rounded to float
  int32_t seg;
  int32_t status;             // 1 evaluate, 0 outside the rectangle, -2 bad segment
  int32_t plan;
  int32_t rank;               // rank of V (0, 1 or 2)
};

// Network, search rectangle and band reference frequency (device resident).
struct NetDesc {
  int32_t n_det;
  int32_t max_segments;
  double pos[kMaxDet][3];
  double ten[kMaxDet][3][3];
  double box_lo[4], box_hi[4];
  double f_star;
};

constexpr double kPi = 3.14159265358979323846;
constexpr double kC = 299792458.0;

// ---------------------------------------------------------------------------
// Set-up of one parameter point, FP64 (chirp times, delays, antenna patterns,
// orthonormal basis).  Sec. II.B (chirp times), Sec. II (eq. detresponse:
// delays, antenna pattern matrix), Sec. II.C (U = F(psi = 0)).
//
// Written once for two executions: `Dets` is either a loop over the
// detectors (setup_one, one thread per point) or a group of lanes with one
// detector each, whose sums over detectors are lane reductions (the kernel).
// Per-detector values live in the point's descriptor; a lane only ever reads
// back the entries it wrote itself.
// ---------------------------------------------------------------------------
struct SkyFrame {
  double n[3], ex[3], ey[3];   // propagation direction and wave axes (-alpha_hat, delta_hat)
};

// Phase coefficients (cycles) and the sky frame of a point.
FCAS_HD void setup_point(const NetDesc& net, const double* th, double coef[4], SkyFrame& fr) {
  const double alpha = th[0], delta = th[1], tau0 = th[2], tau15 = th[3];
  const double fs = net.f_star;
  const double v0 = cbrt(5.0 * tau15 / (32.0 * kPi * tau0));
  const double eta = 1.0 / (8.0 * fs * tau15 * v0 * v0);
  const double tau1 = 5.0 / (192.0 * kPi * fs * eta * v0 * v0 * v0) * (743.0 / 336.0 + 11.0 * eta / 4.0);
  const double tau2 = 5.0 / (128.0 * kPi * fs * eta * v0) *
                      (3058673.0 / 1016064.0 + 5429.0 * eta / 1008.0 + 617.0 * eta * eta / 144.0);
  coef[0] = fs * 0.6 * tau0;
  coef[1] = fs * tau1;
  coef[2] = -fs * 1.5 * tau15;
  coef[3] = fs * 3.0 * tau2;
  double sa, ca, sd, cd;
  sincos(alpha, &sa, &ca);
  sincos(delta, &sd, &cd);
  fr.n[0] = cd * ca; fr.n[1] = cd * sa; fr.n[2] = sd;
  fr.ex[0] = sa; fr.ex[1] = -ca; fr.ex[2] = 0.0;
  fr.ey[0] = -sd * ca; fr.ey[1] = -sd * sa; fr.ey[2] = cd;
}

// Delay ramp of detector i in cycles per bin of width df (delay relative to
// the geocentre).
FCAS_HD double detector_delay(const NetDesc& net, double df, const SkyFrame& fr, int i) {
  const double* r = net.pos[i];
  return -(fr.n[0] * r[0] + fr.n[1] * r[1] + fr.n[2] * r[2]) / kC * df;
}

// Detector i of a segment with bin width df, pass-1 register stride dk1 and
// template norm sigma_i: delay ramp (cycles per bin), its pass-1 step
// relative to detector 0, and row i of V.
FCAS_HD void setup_detector(const NetDesc& net, double df, int dk1, double sigma_i, const SkyFrame& fr, int i,
                            EvalDesc& ev) {
  ev.dly[i] = detector_delay(net, df, fr, i);
  const double ps = (double)dk1 * (ev.dly[i] - detector_delay(net, df, fr, 0));
  double ss, cs;
  sincos_rev(ps - rint(ps), &ss, &cs);
  ev.step1[i][0] = cs;
  ev.step1[i][1] = ss;
  ev.step1f[i][0] = (float)cs;
  ev.step1f[i][1] = (float)ss;
  double up = 0.0, uc = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const double d = net.ten[i][a][b];
      up += d * (fr.ex[a] * fr.ex[b] - fr.ey[a] * fr.ey[b]);
      uc += d * (fr.ex[a] * fr.ey[b] + fr.ey[a] * fr.ex[b]);
    }
  ev.v[i][0] = sigma_i * up;
  ev.v[i][1] = sigma_i * uc;
}

// Orthonormal basis Q of span(V): modified Gram-Schmidt, twice, larger
// column first; q[i][1] holds the residual of the second column until it is
// normalised.  Returns the rank (0, 1 or 2).
template <class Dets>
FCAS_HD int setup_basis(EvalDesc& ev, const Dets& dets) {
  const double n0 = dets.sum([&](int i) { return ev.v[i][0] * ev.v[i][0]; });
  const double n1 = dets.sum([&](int i) { return ev.v[i][1] * ev.v[i][1]; });
  const double vf = n0 + n1;
  const int ca = (n1 > n0) ? 1 : 0, cb = 1 - ca;
  const double na = sqrt(ca ? n1 : n0);
  dets.all([&](int i) { ev.q[i][0] = ev.q[i][1] = 0.0; });
  int rank = 0;
  if (na > 0.0) {
    rank = 1;
    dets.each([&](int i) {
      ev.q[i][0] = ev.v[i][ca] / na;
      ev.q[i][1] = ev.v[i][cb];
    });
    for (int pass = 0; pass < 2; ++pass) {
      const double dot = dets.sum([&](int i) { return ev.q[i][0] * ev.q[i][1]; });
      dets.each([&](int i) { ev.q[i][1] -= dot * ev.q[i][0]; });
    }
    const double nb = sqrt(dets.sum([&](int i) { return ev.q[i][1] * ev.q[i][1]; }));
    if (nb > 1e-10 * sqrt(vf)) {
      rank = 2;
      dets.each([&](int i) { ev.q[i][1] /= nb; });
    } else {
      dets.each([&](int i) { ev.q[i][1] = 0.0; });
    }
  }
  dets.all([&](int i) {
    ev.qf[i][0] = (float)ev.q[i][0];
    ev.qf[i][1] = (float)ev.q[i][1];
  });
  return rank;
}

// The detectors as a loop of one thread.
struct DetLoop {
  int n_det;
  template <class F> FCAS_HD double sum(F f) const {
    double acc = 0.0;
    for (int i = 0; i < n_det; ++i) acc += f(i);
    return acc;
  }
  template <class F> FCAS_HD void each(F f) const {
    for (int i = 0; i < n_det; ++i) f(i);
  }
  template <class F> FCAS_HD void all(F f) const {   // every descriptor slot, used or not
    for (int i = 0; i < kMaxDet; ++i) f(i);
  }
};

FCAS_HD void setup_one(const NetDesc& net, const SegDesc& sg, const double* th, EvalDesc& ev) {
  SkyFrame fr;
  setup_point(net, th, ev.coef, fr);
  for (int i = 0; i < net.n_det; ++i) setup_detector(net, sg.df, sg.dk1, sg.sigma[i], fr, i, ev);
  ev.rank = setup_basis(ev, DetLoop{net.n_det});
}

// Common phase of bin k in cycles, b = (f_k / f*)^(-1/3): FP64 throughout.
FCAS_HD double common_phase(const double* coef, double b) {
  const double b2 = b * b;
  return b * (coef[3] + b * (coef[2] + b * (coef[1] + coef[0] * b2)));
}

template <typename Real> struct Basis;
template <> struct Basis<float> {
  FCAS_HD static float get(const EvalDesc& e, int i, int m) { return e.qf[i][m]; }
};
template <> struct Basis<double> {
  FCAS_HD static double get(const EvalDesc& e, int i, int m) { return e.q[i][m]; }
};

template <typename Real> FCAS_HD cplx<Real> ramp_step(const EvalDesc& e, int i);
template <> FCAS_HD cplx<float> ramp_step<float>(const EvalDesc& e, int i) {
  return mk<float>(e.step1f[i][0], e.step1f[i][1]);
}
template <> FCAS_HD cplx<double> ramp_step<double>(const EvalDesc& e, int i) {
  return mk<double>(e.step1[i][0], e.step1[i][1]);
}

// W_0(k), W_1(k) for one in-band bin.  kk = k - k_lo.
template <typename Real>
FCAS_HD void project_bin(const EvalDesc& ev, const cplx<Real>* y, const double* bt, int n_det, int k,
                         int kk, cplx<Real>& w0, cplx<Real>& w1) {
  const double phc = common_phase(ev.coef, bt[kk]);
  const double kd = (double)k;
  const cplx<Real>* yr = y + (int64_t)kk * n_det;
  w0 = mk<Real>(0, 0);
  w1 = mk<Real>(0, 0);
  for (int i = 0; i < n_det; ++i) {
    const double ph = kd * ev.dly[i] + phc;   // cycles
    const double r = ph - rint(ph);           // reduced to [-1/2, 1/2] in FP64
    Real s, c;
    sincos_rev((Real)r, &s, &c);
    const cplx<Real> w = mul(yr[i], mk<Real>(c, s));
    const Real q0 = Basis<Real>::get(ev, i, 0), q1 = Basis<Real>::get(ev, i, 1);
    w0 = mk<Real>(w0.x + q0 * w.x, w0.y + q0 * w.y);
    w1 = mk<Real>(w1.x + q1 * w.x, w1.y + q1 * w.y);
  }
}

// ---------------------------------------------------------------------------
// One Stockham stage for one series of one transform (see fft_core.hpp).
// Either leaves the outputs in registers (last stage) or scatters them to the
// transform's LDS buffer, to be gathered back in natural strided order.
// ---------------------------------------------------------------------------
template <typename Real, int L, int E, int R, int Ns, bool LAST, bool HALF, int PAD>
FCAS_HD void stage_butterflies(cplx<Real>* vs, cplx<Real>* buf, const cplx<Real>* tw, int t) {
  constexpr int P = L / E;
  constexpr int B = E / R;
  static_assert(E % R == 0, "radix must divide the elements per thread");
  static_assert(!HALF || (Ns == 1 && B == 1), "half-zero inputs only in a first stage with one butterfly");
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int v = t + b * P;
    cplx<Real> x[R];
#pragma unroll
    for (int p = 0; p < (HALF ? R / 2 : R); ++p) x[p] = vs[b + p * B];
    if constexpr (Ns > 1) {
#pragma unroll
      for (int p = 1; p < R; ++p) x[p] = mul(x[p], tw[stockham_tw(v, Ns, R, p, L)]);
    }
    if constexpr (HALF)
      dft_half<R>(x);
    else
      dft<R>(x);
    if constexpr (LAST) {
#pragma unroll
      for (int p = 0; p < R; ++p) vs[b + p * B] = x[p];
    } else {
#pragma unroll
      for (int p = 0; p < R; ++p) buf[lds_pad<PAD>(stockham_dst(v, Ns, R, p))] = x[p];
    }
  }
}

template <typename Real, int L, int E, int PAD>
FCAS_HD void stage_gather(cplx<Real>* vs, const cplx<Real>* buf, int t) {
  constexpr int P = L / E;
#pragma unroll
  for (int q = 0; q < E; ++q) vs[q] = buf[lds_pad<PAD>(t + q * P)];
}

// Compile-time description of a plan.
// Two-pass plans (NM = 1): N = N1 * N2,
//   pass 1: C columns per work item, P1 = N1 / E1 threads per column
//   pass 2: RW rows per work item,   P2 = N2 / E2 threads per row
// Three-pass plans (NM > 1): N = N1 * NM * N2 with
//   k = k1 NM N2 + km N2 + k2,  j = j1 + N1 jm + N1 NM j2,
//   pass 1 (per column km N2 + k2 of its W1 = NM N2): the length-N1 transform over k1,
//           stored as B1[j1][km N2 + k2]
//   middle pass (per j1 and k2; CM adjacent k2 per work item, PM = NM / EM
//           threads per transform): times w_N^{j1 (km N2 + k2)}, the
//           length-NM transform over km, times w_{NM N2}^{jm k2}, stored in
//           place as B2[j1][jm N2 + k2]
//   pass 2 (per row j1 NM + jm, contiguous): the length-N2 transform over k2
//           and the maximum of |a_0|^2 + |a_1|^2 over its samples
// which is the four-step factorisation applied twice: both passes' row
// segments stay contiguous, so every store and load moves whole 64-byte or
// longer pieces even when N1 N2 exceeds what one work item can hold.
// LDS padding of the exchanges (see lds_pad): one spare element in 16 for all
// passes (on gfx950 pass 1 runs 1.7x slower unpadded, pass 2 ~8%).
constexpr int kPad1 = 4, kPad2 = 4, kPadM = 4;

template <int N1_, int E1_, class Rad1_, int C_, int N2_, int E2_, class Rad2_, int RW_, int NM_ = 1, int EM_ = 1,
          class RadM_ = Radices<1>, int CM_ = 1>
struct Plan {
  static constexpr int N1 = N1_, E1 = E1_, C = C_, N2 = N2_, E2 = E2_, RW = RW_;
  static constexpr int NM = NM_, EM = EM_, CM = CM_;
  using Rad1 = Rad1_;
  using Rad2 = Rad2_;
  using RadM = RadM_;
  static constexpr bool THREE = NM > 1;
  static constexpr int W1 = NM * N2;                        // columns of pass 1 (its output row length)
  static constexpr int ROWS2 = N1 * NM;                     // rows of pass 2
  static constexpr int64_t N = (int64_t)N1 * NM * N2;
  static constexpr int P1 = N1 / E1, P2 = N2 / E2, PM = NM / EM;
  static constexpr int T1 = C * P1, T2 = RW * P2, TM = CM * PM;   // threads per work item
  static constexpr int TILES1 = W1 / C, TILES2 = ROWS2 / RW;      // work items per evaluation
  static constexpr int TILESM = THREE ? N1 * (N2 / CM) : 0;
  static constexpr int DK1 = P1 * W1;                       // bin stride between a pass-1 thread's registers
  static constexpr int PARTS2 = TILES2 * (T2 / 64);         // pass-2 partials (one per wavefront)
  static_assert(Rad1::product() == N1, "pass-1 radices must multiply to N1");
  static_assert(Rad2::product() == N2, "pass-2 radices must multiply to N2");
  static_assert(RadM::product() == NM, "middle-pass radices must multiply to NM");
  static_assert(N1 % E1 == 0 && N2 % E2 == 0 && NM % EM == 0, "elements per thread must divide the length");
  static_assert(W1 % C == 0 && ROWS2 % RW == 0 && N2 % CM == 0, "tiles must divide the transform");
  static_assert(T2 % 64 == 0 && (64 % P2 == 0 || P2 % 64 == 0), "pass-2 rows and wavefronts must nest");
  // the middle pass works in place: at least one work-group barrier (between
  // two stages) separates an item's loads from its stores
  static_assert(!THREE || RadM::count >= 2, "the middle pass needs two or more stages");
  static_assert(N < ((int64_t)1 << 30), "sample and bin indices are 32-bit");
};

// First output sample of pass-2 row `row`; the row's samples follow at a
// stride of ROWS2.
template <class PL>
FCAS_HD int row_base(int row) {
  if constexpr (PL::THREE) {
    const int j1 = row / PL::NM;
    return j1 + PL::N1 * (row - j1 * PL::NM);
  } else {
    return row;
  }
}

// ---------------------------------------------------------------------------
// Pass 1, thread (c, p) of column tile `tile`: prologue into registers.
// Register q holds k1 = p + q P1, i.e. bin k = k1 W1 + k2.  Only positive
// frequencies are in band (k <= k_hi < N/2), so registers q >= E1/2
// (k1 >= N1/2) are always zero and are left unset: the first stage reads
// only the lower half.
//
// With the delay ramps r_i(k) = exp(2 pi i k dly_i) and the template phase
// Phi_k, W_m(k) = exp(2 pi i Phi_k) sum_i Q_im y^i_k r_i(k).  Detector 0's ramp
// is taken out of the sum into the common factor,
//   W_m(k) = e(k) [Q_0m y^0_k + sum_{i>0} Q_im y^i_k r'_i(k)],
//   e(k) = exp(2 pi i (Phi_k + k dly_0)),  r'_i(k) = exp(2 pi i k (dly_i - dly_0)),
// so detector 0 needs no ramp.  e is one sine/cosine per bin of an FP64 phase
// reduced mod 1; r'_i is exact (FP64-reduced) at the thread's first bin and
// advanced by the constant factor exp(2 pi i (P1 W1)(dly_i - dly_0)) of the
// point's descriptor from register to register.  Out-of-band registers read
// bin k_lo (any finite value) and are cleared by a zero e, so no lane
// branches.
// ---------------------------------------------------------------------------
// Segment data one pass-1 thread needs for a work item: y of its in-band
// registers and detectors, and the basis b of those bins (DT > 0 only).
template <typename Real, class PL, int DT>
struct Pass1Data {
  static constexpr int QH = PL::E1 / 2;
  cplx<Real> y[DT > 0 ? DT : 1][QH];
  double b[QH];
  bool in[QH];
  int k0;
};

template <typename Real, class PL, int DT>
FCAS_HD void pass1_fetch(Pass1Data<Real, PL, DT>& d, const SegDesc& sg, int tile, int c, int p) {
  constexpr int QH = PL::E1 / 2;
  constexpr int DK = PL::DK1;
  static_assert(DT > 0, "prefetch needs a compile-time detector count");
  const int k2 = tile * PL::C + c;
  d.k0 = p * PL::W1 + k2;
  const FCAS_AS_GLOBAL cplx<Real>* y = global_view((const cplx<Real>*)sg.y);
  const FCAS_AS_GLOBAL double* bt = global_view(sg.b);
#pragma unroll
  for (int q = 0; q < QH; ++q) {
    const int k = d.k0 + q * DK;
    d.in[q] = (k >= sg.k_lo) && (k <= sg.k_hi);
    const int kk = d.in[q] ? k - sg.k_lo : 0;
    d.b[q] = bt[kk];
#pragma unroll
    for (int i = 0; i < DT; ++i) d.y[i][q] = y[(int64_t)kk * DT + i];
  }
}

// What the pass-1 arithmetic reads of a point's descriptor, in the working
// precision: phase coefficients, delay ramps, basis Q and ramp steps of the
// DT detectors.  `ev` points to an EvalDesc (through the constant address
// space in the kernels, so that these uniform values are scalar loads held in
// scalar registers).
template <typename Real, int DT>
struct Pass1Point {
  double coef[4];
  double dly[DT];
  Real q[DT][2];
  Real step[DT][2];
};

template <typename Real, int DT, class P>
FCAS_HD Pass1Point<Real, DT> pass1_point(P ev) {
  Pass1Point<Real, DT> r;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.coef[k] = ev->coef[k];
#pragma unroll
  for (int i = 0; i < DT; ++i) {
    r.dly[i] = ev->dly[i];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if constexpr (sizeof(Real) == 4) {
        r.q[i][m] = ev->qf[i][m];
        r.step[i][m] = ev->step1f[i][m];
      } else {
        r.q[i][m] = ev->q[i][m];
        r.step[i][m] = ev->step1[i][m];
      }
    }
  }
  return r;
}

// e(k) = exp(2 pi i (Phi_k + k dly_0)) for an in-band bin k with basis value
// b, 0 otherwise (Ev: a descriptor with the phase coefficients `coef` and the
// delay ramps `dly`).
template <typename Real, class Ev>
FCAS_HD cplx<Real> band_phase(const Ev& ev, double b, int k, bool in) {
  const double ph = common_phase(ev.coef, b) + (double)k * ev.dly[0];
  Real s, cc;
  sincos_rev((Real)(ph - rint(ph)), &s, &cc);
  return in ? mk<Real>(cc, s) : mk<Real>(0, 0);
}

// Ramp r'_i of detector i > 0 at the thread's first bin k0 (FP64 reduction).
template <typename Real, class Ev>
FCAS_HD cplx<Real> first_ramp(const Ev& ev, int i, int k0) {
  const double ph0 = (double)k0 * (ev.dly[i] - ev.dly[0]);
  Real s, cc;
  sincos_rev((Real)(ph0 - rint(ph0)), &s, &cc);
  return mk<Real>(cc, s);
}

// The prologue arithmetic on prefetched data (same results as pass1_prologue).
template <typename Real, class PL, int DT>
FCAS_HD void pass1_compute(cplx<Real> (&v)[2][PL::E1], const Pass1Data<Real, PL, DT>& d,
                           const Pass1Point<Real, DT>& ev) {
  constexpr int QH = PL::E1 / 2;
  {
    const Real q0 = ev.q[0][0], q1 = ev.q[0][1];
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const cplx<Real> u = d.y[0][q];
      v[0][q] = mk<Real>(q0 * u.x, q0 * u.y);
      v[1][q] = mk<Real>(q1 * u.x, q1 * u.y);
    }
  }
#pragma unroll
  for (int i = 1; i < DT; ++i) {
    cplx<Real> ramp = first_ramp<Real>(ev, i, d.k0);
    const cplx<Real> step = mk<Real>(ev.step[i][0], ev.step[i][1]);
    const Real q0 = ev.q[i][0], q1 = ev.q[i][1];
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const cplx<Real> u = mul(d.y[i][q], ramp);
      v[0][q] = mk<Real>(v[0][q].x + q0 * u.x, v[0][q].y + q0 * u.y);
      v[1][q] = mk<Real>(v[1][q].x + q1 * u.x, v[1][q].y + q1 * u.y);
      if (q + 1 < QH) ramp = mul(ramp, step);
    }
  }
#pragma unroll
  for (int q = 0; q < QH; ++q) {
    const cplx<Real> e = band_phase<Real>(ev, d.b[q], d.k0 + q * PL::DK1, d.in[q]);
    v[0][q] = mul(v[0][q], e);
    v[1][q] = mul(v[1][q], e);
  }
}

// DT > 0: the detector count is the compile-time constant DT (loops unrolled,
// every load of the thread issued up front); DT = 0: n_det at run time.
template <typename Real, class PL, int DT = 0>
FCAS_HD void pass1_prologue(cplx<Real> (&v)[2][PL::E1], const EvalDesc& ev, const SegDesc& sg, int n_det_rt,
                            int tile, int c, int p) {
  constexpr int QH = PL::E1 / 2;
  constexpr int DK = PL::DK1;
  const int n_det = DT > 0 ? DT : n_det_rt;
  const int k2 = tile * PL::C + c;
  const int k0 = p * PL::W1 + k2;
  const cplx<Real>* y = (const cplx<Real>*)sg.y;
  bool in[QH];
  int kk[QH];
#pragma unroll
  for (int q = 0; q < QH; ++q) {
    const int k = k0 + q * DK;
    in[q] = (k >= sg.k_lo) && (k <= sg.k_hi);
    kk[q] = in[q] ? k - sg.k_lo : 0;
  }
  {
    const Real q0 = Basis<Real>::get(ev, 0, 0), q1 = Basis<Real>::get(ev, 0, 1);
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const cplx<Real> u = y[(int64_t)kk[q] * n_det];
      v[0][q] = mk<Real>(q0 * u.x, q0 * u.y);
      v[1][q] = mk<Real>(q1 * u.x, q1 * u.y);
    }
  }
#pragma unroll
  for (int i = 1; i < (DT > 0 ? DT : kMaxDet); ++i) {
    if (DT == 0 && i >= n_det) break;
    cplx<Real> ramp = first_ramp<Real>(ev, i, k0);
    const cplx<Real> step = ramp_step<Real>(ev, i);
    const Real q0 = Basis<Real>::get(ev, i, 0), q1 = Basis<Real>::get(ev, i, 1);
#pragma unroll
    for (int q = 0; q < QH; ++q) {
      const cplx<Real> u = mul(y[(int64_t)kk[q] * n_det + i], ramp);
      v[0][q] = mk<Real>(v[0][q].x + q0 * u.x, v[0][q].y + q0 * u.y);
      v[1][q] = mk<Real>(v[1][q].x + q1 * u.x, v[1][q].y + q1 * u.y);
      if (q + 1 < QH) ramp = mul(ramp, step);
    }
  }
#pragma unroll
  for (int q = 0; q < QH; ++q) {
    const cplx<Real> e = band_phase<Real>(ev, sg.b[kk[q]], k0 + q * DK, in[q]);
    v[0][q] = mul(v[0][q], e);
    v[1][q] = mul(v[1][q], e);
  }
}

// Pass 1 epilogue: store B[m][j1][k2] (the four-step twiddle is applied when
// the next pass loads the rows).
template <typename Real, class PL>
FCAS_HD void pass1_store(cplx<Real> (&v)[2][PL::E1], cplx<Real>* slot, int tile, int c, int p) {
  static_assert(2 * (int64_t)PL::N * sizeof(cplx<Real>) < (int64_t(1) << 31), "byte offsets fit in 31 bits");
  const StreamOut<Real> out(slot, 2 * (int64_t)PL::N);
  const int o = p * PL::W1 + tile * PL::C + c;      // row j1 = p, column k2
#pragma unroll
  for (int q = 0; q < PL::E1; ++q) {
    out.store(o, q * PL::P1 * PL::W1, v[0][q]);       // row j1 = p + q P1
    out.store(o, PL::N + q * PL::P1 * PL::W1, v[1][q]);
  }
}

// ---------------------------------------------------------------------------
// Middle pass of a three-pass plan, thread (c, p) of tile `tile`: the tile is
// pass-1 row j1 = tile / (N2 / CM) and the CM adjacent columns k2 from
// (tile mod (N2 / CM)) CM; register q holds km = p + q PM on input and
// jm = p + q PM on output.
// ---------------------------------------------------------------------------
template <class PL>
FCAS_HD void passm_coords(int tile, int c, int& j1, int& k2) {
  constexpr int KT = PL::N2 / PL::CM;
  j1 = tile / KT;
  k2 = (tile - j1 * KT) * PL::CM + c;
}

// The middle-pass functions act on S series held in registers, series s0
// onwards (S = 2, s0 = 0: both).
template <typename Real, class PL, int S>
FCAS_HD void passm_fetch(cplx<Real> (&v)[S][PL::EM], const cplx<Real>* slot, int tile, int c, int p, int s0 = 0) {
  int j1, k2;
  passm_coords<PL>(tile, c, j1, k2);
  const cplx<Real>* at = slot + (int64_t)s0 * PL::N + (int64_t)j1 * PL::W1 + k2;
#pragma unroll
  for (int q = 0; q < PL::EM; ++q) {
    const int o = (p + q * PL::PM) * PL::N2;
#pragma unroll
    for (int s = 0; s < S; ++s) v[s][q] = stream_load(at + s * PL::N + o);
  }
}

// w_N^{j1 (km N2 + k2)} on input: exact at q = 0, then advanced by
// w_N^{j1 PM N2} from register to register.
template <typename Real, class PL, int S>
FCAS_HD void passm_twiddle_in(cplx<Real> (&v)[S][PL::EM], int tile, int c, int p) {
  int j1, k2;
  passm_coords<PL>(tile, c, j1, k2);
  cplx<Real> t = twiddle<Real>(j1 * (p * PL::N2 + k2), (int)PL::N);     // < N1 W1 = N
  const cplx<Real> st = twiddle<Real>(j1 * (PL::PM * PL::N2), (int)PL::N);
#pragma unroll
  for (int q = 0; q < PL::EM; ++q) {
#pragma unroll
    for (int s = 0; s < S; ++s) v[s][q] = mul(v[s][q], t);
    if (q + 1 < PL::EM) t = mul(t, st);
  }
}

// w_{NM N2}^{jm k2} on output: exact at q = 0, then advanced by w_{NM N2}^{PM k2}.
template <typename Real, class PL, int S>
FCAS_HD void passm_twiddle_out(cplx<Real> (&v)[S][PL::EM], int tile, int c, int p) {
  int j1, k2;
  passm_coords<PL>(tile, c, j1, k2);
  cplx<Real> t = twiddle<Real>(p * k2, PL::W1);                      // < PM N2 <= W1
  const cplx<Real> st = twiddle<Real>(PL::PM * k2, PL::W1);
#pragma unroll
  for (int q = 0; q < PL::EM; ++q) {
#pragma unroll
    for (int s = 0; s < S; ++s) v[s][q] = mul(v[s][q], t);
    if (q + 1 < PL::EM) t = mul(t, st);
  }
}

// Store B2[m][j1][jm N2 + k2], over the elements the tile loaded.
template <typename Real, class PL, int S>
FCAS_HD void passm_store(cplx<Real> (&v)[S][PL::EM], cplx<Real>* slot, int tile, int c, int p, int s0 = 0) {
  int j1, k2;
  passm_coords<PL>(tile, c, j1, k2);
  cplx<Real>* at = slot + (int64_t)s0 * PL::N + (int64_t)j1 * PL::W1 + k2;
#pragma unroll
  for (int q = 0; q < PL::EM; ++q) {
    const int o = (p + q * PL::PM) * PL::N2;
#pragma unroll
    for (int s = 0; s < S; ++s) stream_store(at + s * PL::N + o, v[s][q]);
  }
}

// Pass 2 prologue: thread (r, p) of row tile `tile` reads row tile RW + r,
// register q holds k2 = p + q P2 (pass2_fetch); in a two-pass plan the row is
// j1 and the four-step twiddle w_N^{k2 j1} follows (pass2_twiddle), in a
// three-pass plan the middle pass has applied it.
template <typename Real, class PL>
FCAS_HD void pass2_fetch(cplx<Real> (&v)[2][PL::E2], const cplx<Real>* slot, int tile, int r, int p) {
  const int j1 = tile * PL::RW + r;
  const int64_t row = (int64_t)j1 * PL::N2;
#pragma unroll
  for (int q = 0; q < PL::E2; ++q) {
    const int k2 = p + q * PL::P2;
    v[0][q] = stream_load(slot + row + k2);
    v[1][q] = stream_load(slot + PL::N + row + k2);
  }
}

// w_N^{k2 j1} for k2 = p + q P2: exact (one sine/cosine pair) at q = 0, then
// advanced by the factor w_N^{P2 j1} from register to register.
template <typename Real, class PL>
FCAS_HD void pass2_twiddle(cplx<Real> (&v)[2][PL::E2], int tile, int r, int p) {
  static_assert(!PL::THREE, "three-pass plans twiddle in the middle pass");
  const int j1 = tile * PL::RW + r;
  cplx<Real> t = twiddle<Real>(p * j1, (int)PL::N);                // p j1 < N
  const cplx<Real> st = twiddle<Real>(PL::P2 * j1, (int)PL::N);    // P2 j1 < N
#pragma unroll
  for (int q = 0; q < PL::E2; ++q) {
    v[0][q] = mul(v[0][q], t);
    v[1][q] = mul(v[1][q], t);
    if (q + 1 < PL::E2) t = mul(t, st);
  }
}

template <typename Real, class PL>
FCAS_HD void pass2_load(cplx<Real> (&v)[2][PL::E2], const cplx<Real>* slot, int tile, int r, int p) {
  pass2_fetch<Real, PL>(v, slot, tile, r, p);
  if constexpr (!PL::THREE) pass2_twiddle<Real, PL>(v, tile, r, p);
}

// Pass 2 epilogue: Gamma^2_j = |a_0|^2 + |a_1|^2 at j = row_base + ROWS2 (p + q P2),
// for j_lo <= j < j_hi; the thread's largest value and, among equal values,
// its smallest j (value -1 if none of its samples is in range).
template <typename Real, class PL>
FCAS_HD void pass2_best(const cplx<Real> (&v)[2][PL::E2], int tile, int r, int p, Real& best, int& best_j,
                        int64_t j_lo = 0, int64_t j_hi = PL::N) {
  const int j0 = row_base<PL>(tile * PL::RW + r);
  const int lo = j_lo > 0 ? (int)j_lo : 0;
  const int hi = j_hi < PL::N ? (int)j_hi : (int)PL::N;
  best = (Real)-1;
  best_j = 0x7fffffff;
  if (lo == 0 && hi == (int)PL::N) {   // whole series (uniform branch)
#pragma unroll
    for (int q = 0; q < PL::E2; ++q) {
      const Real g = norm2(v[0][q]) + norm2(v[1][q]);
      if (g > best) {   // j grows with q: ties keep the smaller j
        best = g;
        best_j = j0 + PL::ROWS2 * (p + q * PL::P2);
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < PL::E2; ++q) {
      const Real g = norm2(v[0][q]) + norm2(v[1][q]);
      const int j = j0 + PL::ROWS2 * (p + q * PL::P2);
      if (g > best && j >= lo && j < hi) {
        best = g;
        best_j = j;
      }
    }
  }
}

// Work item `item` of the fused schedule (cnt evaluations, lag L, T1 pass-1
// and T2 pass-2 tiles each): kind 1 / 2 = pass 1 / pass 2, list position ep,
// tile.  Sequence: [P1(0..L-1)] then rounds [P1(L + r) P2(r)] then [P2(cnt-L..cnt-1)].
FCAS_HD void fused_decode(int item, int cnt, int L, int T1, int T2, int& kind, int& ep, int& tile) {
  const int T = T1 + T2;
  if (item < L * T1) {
    kind = 1; ep = item / T1; tile = item - ep * T1;
    return;
  }
  const int j = item - L * T1, mid = (cnt - L) * T;
  if (j < mid) {
    const int r = j / T, w = j - r * T;
    if (w < T1) { kind = 1; ep = L + r; tile = w; }
    else { kind = 2; ep = r; tile = w - T1; }
  } else {
    const int k = j - mid;
    kind = 2; ep = (cnt - L) + k / T2; tile = k - (k / T2) * T2;
  }
}

// (g, j) ordering used by every reduction: larger g wins, then smaller j.
template <typename Real>
FCAS_HD bool better(Real g, int j, Real g_ref, int j_ref) {
  return g > g_ref || (g == g_ref && j < j_ref);
}

}  // namespace fcas
