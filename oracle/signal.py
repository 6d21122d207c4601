"""Plain FP64 oracle of the signal model and of the log-likelihood ratio as
literally defined, without the efficient-evaluation rearrangements.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the CPU-baseline leg of
the benchmark may use it; the HIP library never).

  * injection(): the strain response of eq. detresponse with the SPA
    polarisation waveforms of Sec. II.B, scaled to a network SNR (eq.
    optimalSNR).
  * loglikelihood(): lambda^(D) of eq. loglikelihood with the inner product of
    eq. innprod, for explicit amplitudes A_k and coalescence time t_c, with the
    template waveforms h_1..h_4 of Sec. II.C each delayed by Delta^i.
"""
from __future__ import annotations

import math

import numpy as np

from .fitness import antenna_patterns, band_bins, delays, phase_cycles, template_matrix_U


def inner_product(p, q, psd_row, df, k_lo, k_hi):
    """<p|q> = 4 Re int p q* / S df, as a sum over the in-band bins (eq. innprod);
    templates vanish outside the band."""
    sl = slice(k_lo, k_hi + 1)
    return 4.0 * df * float(np.real(np.sum(p[sl] * np.conj(q[sl]) / psd_row[sl])))


def spa_polarisations(n_samples, fs, f_low, f_high, tau0, tau15, t_c, phi_c, a_plus, a_cross):
    """h_plus(f), h_cross(f) on the one-sided grid (zero outside the band), Sec. II.B:
    h+ = A+ f^-7/6 e^{-i Psi},  hx = Ax f^-7/6 e^{-i (Psi + pi/2)},
    Psi = 2 pi f t_c - phi_c - pi/4 + 2 pi Phi(f)."""
    k_lo, k_hi = band_bins(n_samples, fs, f_low, f_high)
    df = fs / n_samples
    f = np.arange(k_lo, k_hi + 1) * df
    Psi = 2.0 * math.pi * (f * t_c + phase_cycles(f, tau0, tau15, f_low)) - phi_c - math.pi / 4.0
    hp = np.zeros(n_samples // 2 + 1, dtype=np.complex128)
    hc = np.zeros_like(hp)
    hp[k_lo:k_hi + 1] = a_plus * f ** (-7.0 / 6.0) * np.exp(-1j * Psi)
    hc[k_lo:k_hi + 1] = a_cross * f ** (-7.0 / 6.0) * np.exp(-1j * (Psi + math.pi / 2.0))
    return hp, hc


def shift(hf, n_samples, fs, dt):
    """Fourier transform of h(t - dt)."""
    f = np.arange(hf.size) * (fs / n_samples)
    return hf * np.exp(-2j * math.pi * f * dt)


def injection(n_samples, fs, f_low, f_high, pos_m, tensors, psd, theta0, psi, phi_c, cos_iota,
              tc_sample, snr=None):
    """Detector responses h^i(f), (D, N/2+1), for a source at theta0 = (alpha,
    delta, tau0, tau1.5) with polarisation psi, phase phi_c, inclination cos_iota
    and coalescence at sample tc_sample at the Earth's centre.

    h^i(t + Delta^i) = F+^i h+(t) + Fx^i hx(t)  (eq. detresponse), so
    h^i(f) = [F+^i h+(f) + Fx^i hx(f)] e^{-2 pi i f Delta^i}.
    Amplitudes: A+ = (1 + cos^2 iota)/2, Ax = cos iota (the reading taken for the
    unspecified overall amplitude).  If snr is given, the responses are scaled
    so that sum_i <h^i|h^i> = snr^2 (eq. optimalSNR).
    """
    alpha, delta, tau0, tau15 = (float(v) for v in theta0)
    psd = np.atleast_2d(psd)
    t_c = tc_sample / fs
    hp, hc = spa_polarisations(n_samples, fs, f_low, f_high, tau0, tau15, t_c, phi_c,
                               0.5 * (1.0 + cos_iota ** 2), cos_iota)
    fp, fc = antenna_patterns(alpha, delta, psi, tensors)
    dl = delays(alpha, delta, pos_m)
    h = np.array([shift(fp[i] * hp + fc[i] * hc, n_samples, fs, dl[i]) for i in range(len(fp))])
    if snr is not None:
        h *= snr / network_snr(h, psd, n_samples, fs, f_low, f_high)
    return h


def network_snr(h, psd, n_samples, fs, f_low, f_high):
    """[sum_i <h^i|h^i>^i]^(1/2) (eq. optimalSNR)."""
    k_lo, k_hi = band_bins(n_samples, fs, f_low, f_high)
    df = fs / n_samples
    psd = np.atleast_2d(psd)
    return math.sqrt(sum(inner_product(h[i], h[i], psd[i], df, k_lo, k_hi) for i in range(h.shape[0])))


def templates(n_samples, fs, f_low, f_high, tensors, pos_m, theta, t_c):
    """The four template waveforms h_k^i(t - Delta^i), (4, D, N/2+1), Sec. II.C:
    h1 = U+ h_c, h2 = Ux h_c, h3 = U+ h_s, h4 = Ux h_s with h_c = h+ and
    h_s = hx at phi_c = 0, A+ = Ax = 1."""
    alpha, delta, tau0, tau15 = (float(v) for v in theta)
    h_c, h_s = spa_polarisations(n_samples, fs, f_low, f_high, tau0, tau15, t_c, 0.0, 1.0, 1.0)
    U = template_matrix_U(alpha, delta, tensors)
    dl = delays(alpha, delta, pos_m)
    D = U.shape[0]
    out = np.empty((4, D, h_c.size), dtype=np.complex128)
    for i in range(D):
        hc_i = shift(h_c, n_samples, fs, dl[i])
        hs_i = shift(h_s, n_samples, fs, dl[i])
        out[0, i] = U[i, 0] * hc_i
        out[1, i] = U[i, 1] * hc_i
        out[2, i] = U[i, 0] * hs_i
        out[3, i] = U[i, 1] * hs_i
    return out


def loglikelihood(xf, psd, fs, f_low, f_high, tensors, pos_m, theta, amps, t_c):
    """lambda^(D) = sum_i [<x^i|h^i> - <h^i|h^i>/2], h^i = sum_k A_k h_k^i(t - Delta^i)."""
    xf = np.atleast_2d(xf)
    psd = np.atleast_2d(psd)
    n_samples = 2 * (xf.shape[1] - 1)
    k_lo, k_hi = band_bins(n_samples, fs, f_low, f_high)
    df = fs / n_samples
    H = templates(n_samples, fs, f_low, f_high, tensors, pos_m, theta, t_c)
    lam = 0.0
    for i in range(xf.shape[0]):
        h_i = np.tensordot(np.asarray(amps, dtype=np.float64), H[:, i], axes=1)
        lam += inner_product(xf[i], h_i, psd[i], df, k_lo, k_hi) - 0.5 * inner_product(h_i, h_i, psd[i], df, k_lo, k_hi)
    return lam


def amplitude_normal_equations(xf, psd, fs, f_low, f_high, tensors, pos_m, theta, t_c):
    """b_k = sum_i <x^i|h_k^i>, M_kl = sum_i <h_k^i|h_l^i>: lambda = A.b - A.M.A/2,
    so max_A lambda = b.M^-1.b / 2 at A* = M^-1 b."""
    xf = np.atleast_2d(xf)
    psd = np.atleast_2d(psd)
    n_samples = 2 * (xf.shape[1] - 1)
    k_lo, k_hi = band_bins(n_samples, fs, f_low, f_high)
    df = fs / n_samples
    H = templates(n_samples, fs, f_low, f_high, tensors, pos_m, theta, t_c)
    b = np.zeros(4)
    M = np.zeros((4, 4))
    for i in range(xf.shape[0]):
        for a in range(4):
            b[a] += inner_product(xf[i], H[a, i], psd[i], df, k_lo, k_hi)
            for c in range(4):
                M[a, c] += inner_product(H[a, i], H[c, i], psd[i], df, k_lo, k_hi)
    return b, M
