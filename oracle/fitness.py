"""Plain FP64 CPU oracle of the coherent fitness Gamma^2(alpha, delta, tau0, tau1.5).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It shares no code with the HIP
library: it is written directly from the paper's equations, in NumPy, in
float64, one detector at a time, with no blocking or fusion.

Every function cites the passage of Normandin & Mohanty (arXiv:2002.02150) it
follows.  Where the paper defers to earlier work or is ambiguous, the reading
taken is stated in the docstring (the list of readings is kept with the design
notes of the repository).

Conventions
  * Fourier transform: x(f_k) = dt * sum_n x_n exp(-2 pi i k n / N); one-sided
    PSD S with E|n(f_k)|^2 = T S(f_k) / 2.
  * Phases are carried in cycles.
  * theta = (alpha, delta, tau0, tau1.5): alpha azimuth in the Earth-fixed
    frame, delta latitude-like in [-pi/2, pi/2], chirp times in seconds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GM_SUN_S = 4.925490947e-6          # G Msun / c^3 in seconds
C_MPS = 299792458.0                # speed of light


# --------------------------------------------------------------------------
# Chirp times (Sec. II.B, the tau0 / tau1.5 definitions)
# --------------------------------------------------------------------------

def chirp_times_from_masses(m1, m2, f_star):
    """tau0 and tau1.5 (s) from component masses in Msun (Sec. II.B).

    tau0   = 5/(256 pi) f*^-1 (pi G M f*/c^3)^(-5/3) / eta
    tau1.5 = 1/8        f*^-1 (pi G M f*/c^3)^(-2/3) / eta
    """
    M = (m1 + m2) * GM_SUN_S
    eta = m1 * m2 / (m1 + m2) ** 2
    u = math.pi * M * f_star
    tau0 = 5.0 / (256.0 * math.pi) / f_star * u ** (-5.0 / 3.0) / eta
    tau15 = 1.0 / 8.0 / f_star * u ** (-2.0 / 3.0) / eta
    return tau0, tau15


def mass_params_from_chirp_times(tau0, tau15, f_star):
    """Invert the two definitions: returns (pi M f*)^(1/3) =: v0 and eta.

    Dividing the definitions gives v0^3 = 5 tau1.5 / (32 pi tau0); then the
    tau1.5 definition gives eta = 1 / (8 f* tau1.5 v0^2).
    """
    v0 = (5.0 * tau15 / (32.0 * math.pi * tau0)) ** (1.0 / 3.0)
    eta = 1.0 / (8.0 * f_star * tau15 * v0 * v0)
    return v0, eta


def higher_chirp_times(tau0, tau15, f_star):
    """tau1 and tau2 of the restricted-2PN chirp-time family.

    The paper names psi(f) only as a two-parameter family and defers the
    formulas to earlier work; the reading taken is the standard chirp-time
    form, with (v0 = (pi M f*)^(1/3)):
      tau1 = 5/(192 pi f* eta v0^3) (743/336 + 11 eta / 4)
      tau2 = 5/(128 pi f* eta v0)  (3058673/1016064 + 5429 eta/1008 + 617 eta^2/144)
    """
    v0, eta = mass_params_from_chirp_times(tau0, tau15, f_star)
    tau1 = 5.0 / (192.0 * math.pi * f_star * eta * v0 ** 3) * (743.0 / 336.0 + 11.0 * eta / 4.0)
    tau2 = 5.0 / (128.0 * math.pi * f_star * eta * v0) * (
        3058673.0 / 1016064.0 + 5429.0 * eta / 1008.0 + 617.0 * eta * eta / 144.0)
    return tau1, tau2


def phase_cycles(f, tau0, tau15, f_star):
    """Frequency-dependent SPA phase psi(f) / (2 pi) in cycles (Sec. II.B).

    Phi(f) = f* [ (3/5) tau0 x^(-5/3) + tau1 x^(-1) - (3/2) tau1.5 x^(-2/3)
                  + 3 tau2 x^(-1/3) ],   x = f / f*.
    The 2 pi f t_c term is applied separately (it becomes the matched-filter
    time index and the detector delay); -phi_c - pi/4 is a constant phase that
    the maximisation over amplitudes absorbs.
    """
    tau1, tau2 = higher_chirp_times(tau0, tau15, f_star)
    x = np.asarray(f, dtype=np.float64) / f_star
    return f_star * (0.6 * tau0 * x ** (-5.0 / 3.0) + tau1 / x
                     - 1.5 * tau15 * x ** (-2.0 / 3.0) + 3.0 * tau2 * x ** (-1.0 / 3.0))


# --------------------------------------------------------------------------
# Network response (Sec. II, eq. detresponse)
# --------------------------------------------------------------------------

def sky_unit_vector(alpha, delta):
    """Direction from the Earth's centre to the source (Earth-fixed frame)."""
    return np.array([math.cos(delta) * math.cos(alpha),
                     math.cos(delta) * math.sin(alpha),
                     math.sin(delta)])


def delays(alpha, delta, pos_m):
    """Delta^i: arrival time at detector i minus arrival time at the origin.

    A plane wave from direction n reaches position r at t0 - n.r / c, so
    Delta^i = -n . r^i / c.
    """
    n = sky_unit_vector(alpha, delta)
    return -(np.asarray(pos_m) @ n) / C_MPS


def wave_basis(alpha, delta):
    """Fiducial wave-frame axes (e_X, e_Y) = (-alpha_hat, delta_hat) (Sec. II)."""
    a_hat = np.array([-math.sin(alpha), math.cos(alpha), 0.0])
    d_hat = np.array([-math.sin(delta) * math.cos(alpha),
                      -math.sin(delta) * math.sin(alpha),
                      math.cos(delta)])
    return -a_hat, d_hat


def antenna_patterns(alpha, delta, psi, tensors):
    """(F_plus, F_cross) for each detector: contraction of D^i with the
    polarisation tensors of the wave frame rotated by psi from (-alpha_hat,
    delta_hat)."""
    ex, ey = wave_basis(alpha, delta)
    c, s = math.cos(psi), math.sin(psi)
    ex_p = c * ex + s * ey
    ey_p = -s * ex + c * ey
    e_plus = np.outer(ex_p, ex_p) - np.outer(ey_p, ey_p)
    e_cross = np.outer(ex_p, ey_p) + np.outer(ey_p, ex_p)
    tensors = np.asarray(tensors)
    fp = np.einsum("iab,ab->i", tensors, e_plus)
    fc = np.einsum("iab,ab->i", tensors, e_cross)
    return fp, fc


def template_matrix_U(alpha, delta, tensors, psi=0.0):
    """U = F(alpha, delta, psi = 0), a D x 2 matrix (Sec. II.C, template waveforms).

    A non-zero psi gives F(alpha, delta, psi) instead; the statistic must not
    depend on it (the polarisation angle is absorbed by the amplitudes)."""
    fp, fc = antenna_patterns(alpha, delta, psi, tensors)
    return np.stack([fp, fc], axis=1)


# --------------------------------------------------------------------------
# Segment preparation (Sec. II.D: precomputed template norms, over-whitening)
# --------------------------------------------------------------------------

def band_bins(n_samples, fs, f_low, f_high):
    """Inclusive in-band bin range: f* < f_k <= min(f_high, fs/2), 1 <= k < N/2.

    The template is zero at and below f* (Sec. II.B); the generic upper cutoff
    is f_high; DC and Nyquist are excluded.
    """
    T = n_samples / fs
    k_lo = int(math.floor(f_low * T)) + 1
    k_hi = min(int(math.floor(f_high * T)), n_samples // 2 - 1)
    if k_lo > k_hi:
        raise ValueError("empty band")
    return k_lo, k_hi


@dataclass
class Segment:
    n_samples: int
    fs: float
    f_low: float
    f_high: float
    k_lo: int
    k_hi: int
    sigma: np.ndarray   # (D,)   <h_c|h_c>^(1/2) per detector
    y: np.ndarray       # (D, K) complex: over-whitened data with the template norm folded in

    @property
    def df(self):
        return self.fs / self.n_samples

    @property
    def bins(self):
        return np.arange(self.k_lo, self.k_hi + 1)

    @property
    def freqs(self):
        return self.bins * self.df


def template_norms(psd, n_samples, fs, f_low, f_high):
    """sigma_i^2 = <h_c|h_c>^i = 4 df sum_B f^(-7/3) / S^i (Sec. II.D; the
    amplitude f^(-7/6) of the SPA template, Sec. II.B).  <h_s|h_s> is the same
    and <h_c|h_s> = 0 because h_s = -i h_c in the Fourier domain."""
    k_lo, k_hi = band_bins(n_samples, fs, f_low, f_high)
    df = fs / n_samples
    f = np.arange(k_lo, k_hi + 1) * df
    psd = np.atleast_2d(psd)[:, k_lo:k_hi + 1]
    return np.sqrt(4.0 * df * np.sum(f ** (-7.0 / 3.0) / psd, axis=1))


def prepare_segment(xf, psd, fs, f_low, f_high=1000.0) -> Segment:
    """Over-whiten once: y^i_k = 4 df x^i_k f_k^(-7/6) / (S^i_k sigma_i), k in B.

    xf: (D, N/2+1) one-sided data in continuum units; psd: same shape.
    """
    xf = np.atleast_2d(np.asarray(xf, dtype=np.complex128))
    psd = np.atleast_2d(np.asarray(psd, dtype=np.float64))
    n_samples = 2 * (xf.shape[1] - 1)
    k_lo, k_hi = band_bins(n_samples, fs, f_low, f_high)
    df = fs / n_samples
    sigma = template_norms(psd, n_samples, fs, f_low, f_high)
    f = np.arange(k_lo, k_hi + 1) * df
    y = 4.0 * df * xf[:, k_lo:k_hi + 1] * f ** (-7.0 / 6.0) / psd[:, k_lo:k_hi + 1] / sigma[:, None]
    return Segment(n_samples, fs, f_low, f_high, k_lo, k_hi, sigma, y)


# --------------------------------------------------------------------------
# Fitness (Sec. II.C eqs. loglikelihood, innprod, FCASdetStat, gammaSqd;
# Sec. II.D eq. data_template_innprod)
# --------------------------------------------------------------------------

def matched_filter_series(seg: Segment, pos_m, theta):
    """z^i_j for every detector i and sample j (length N each).

    z^i_j = sum_{k in B} y^i_k exp(2 pi i [Phi_k + f_k Delta^i + k j / N]).
    Its real part is <x^i(t + Delta^i) | h_c(t - j/fs)> / sigma_i and minus its
    imaginary part the same with h_s, since h_s = -i h_c (Sec. II.B).  The time
    shift of the data (eq. data_template_innprod) is the exact phase ramp
    exp(2 pi i f Delta^i).
    """
    alpha, delta, tau0, tau15 = (float(v) for v in theta)
    N = seg.n_samples
    f = seg.freqs
    phi = phase_cycles(f, tau0, tau15, seg.f_low)
    dl = delays(alpha, delta, pos_m)
    D = seg.y.shape[0]
    z = np.empty((D, N), dtype=np.complex128)
    for i in range(D):
        a = np.zeros(N, dtype=np.complex128)
        a[seg.k_lo:seg.k_hi + 1] = seg.y[i] * np.exp(2j * math.pi * (phi + f * dl[i]))
        z[i] = N * np.fft.ifft(a)
    return z


def _gram_pinv(V):
    """Pseudo-inverse of the 2x2 Gram matrix V^T V, as V+ (V+)^T with V+ the
    SVD pseudo-inverse of V (rank rule: singular values of V below 1e-10 of the
    largest are dropped, e.g. a single detector gives rank one)."""
    Vp = np.linalg.pinv(V, rcond=1e-10)
    return Vp @ Vp.T


def gamma2_series(seg: Segment, pos_m, tensors, theta, psi=0.0):
    """Gamma^2_j for every sample j: the log-likelihood ratio maximised over the
    four amplitudes A_k, times two (reading of the scale: Gamma^2 = SNR^2 at the
    true parameters of a noiseless signal).

    With c^i = Re z^i, s^i = -Im z^i and V = diag(sigma) U, the data-template
    inner products are X = (V^T c, V^T s) and the template Gram matrix is
    M = blockdiag(V^T V, V^T V) (Sec. II.D), so 2 max_A lambda = X^T M^-1 X.
    """
    alpha, delta = float(theta[0]), float(theta[1])
    z = matched_filter_series(seg, pos_m, theta)
    c, s = z.real, -z.imag
    V = seg.sigma[:, None] * template_matrix_U(alpha, delta, tensors, psi)
    Ginv = _gram_pinv(V)
    Xc = V.T @ c
    Xs = V.T @ s
    return np.einsum("an,ab,bn->n", Xc, Ginv, Xc) + np.einsum("an,ab,bn->n", Xs, Ginv, Xs)


def in_box(theta, box_lo, box_hi):
    t = np.asarray(theta, dtype=np.float64)
    return bool(np.all(np.isfinite(t)) and np.all(t >= box_lo) and np.all(t <= box_hi))


def fitness(seg: Segment, pos_m, tensors, theta, box_lo=None, box_hi=None, j_range=None):
    """Coherent fitness Gamma^2(theta) = max_j Gamma^2_j and the maximising
    sample j* (smallest j among equal maxima).  j*/fs is the coalescence time at
    the Earth's centre, modulo the segment length.  j_range = (j_lo, j_hi)
    restricts the maximum to j_lo <= j < j_hi.

    Points outside the search rectangle (or non-finite) get (-inf, -1): the
    particle is allowed to leave the rectangle but is not evaluated there.
    """
    if box_lo is not None and not in_box(theta, box_lo, box_hi):
        return -math.inf, -1
    g = gamma2_series(seg, pos_m, tensors, theta)
    lo, hi = (0, len(g)) if j_range is None else j_range
    j = lo + int(np.argmax(g[lo:hi]))
    return float(g[j]), j


def fitness_batch(seg, pos_m, tensors, thetas, box_lo=None, box_hi=None, j_range=None):
    out_f = np.empty(len(thetas))
    out_j = np.empty(len(thetas), dtype=np.int64)
    for n, th in enumerate(thetas):
        out_f[n], out_j[n] = fitness(seg, pos_m, tensors, th, box_lo, box_hi, j_range)
    return out_f, out_j


def gamma2_at(seg: Segment, pos_m, tensors, theta, j):
    """Gamma^2_j at one sample j, by a direct sum over bins (no FFT)."""
    alpha, delta, tau0, tau15 = (float(v) for v in theta)
    f = seg.freqs
    k = seg.bins
    phi = phase_cycles(f, tau0, tau15, seg.f_low)
    dl = delays(alpha, delta, pos_m)
    z = np.array([np.sum(seg.y[i] * np.exp(2j * math.pi * (phi + f * dl[i] + k * j / seg.n_samples)))
                  for i in range(seg.y.shape[0])])
    V = seg.sigma[:, None] * template_matrix_U(alpha, delta, tensors)
    Ginv = _gram_pinv(V)
    xc, xs = V.T @ z.real, V.T @ (-z.imag)
    return float(xc @ Ginv @ xc + xs @ Ginv @ xs)
