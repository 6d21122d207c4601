"""Plain FP64 oracle of the fitness gradient at a fixed time sample.

TEST INFRASTRUCTURE ONLY (same rule as oracle.fitness: tests, the smoke check
and the CPU-baseline leg of the benchmark may use it; the HIP library never).

The paper does not differentiate the fitness; this is the derivative of the
statistic it defines (Sec. II.C eqs. loglikelihood, gammaSqd), holding the
maximising coalescence sample j* fixed:

  Gamma^2_{j*} = Xc^T G^-1 Xc + Xs^T G^-1 Xs,
  Xc = V^T c,  Xs = V^T s,  G = V^T V,  c - i s = z_{j*},

  d Gamma^2 = 2 Xc^T G^-1 dXc - Xc^T G^-1 dG G^-1 Xc   (+ same for s)
  dXc = dV^T c + V^T dc,  dG = dV^T V + V^T dV,
  dz^i = 2 pi i sum_k y^i_k e^{2 pi i (Phi_k + f_k Delta^i + k j*/N)}
                       (dPhi_k + f_k dDelta^i).

The derivatives of the real scalar maps theta -> (phase coefficients, U,
Delta) are taken by the complex-step method (derivative = Im f(x + i h) / h
with h = 1e-30), which is exact to rounding for these analytic maps.  Only
full-rank V (two independent antenna columns) is supported.
"""
from __future__ import annotations

import math

import numpy as np

from .fitness import C_MPS, Segment, fitness

_H = 1e-30


def _phase_coefficients(tau0, tau15, f_star):
    """(c5, c3, c2, c1) with Phi(f) = c5 x^-5/3 + c3 x^-1 + c2 x^-2/3 + c1 x^-1/3,
    x = f/f*, written with numpy so that complex arguments pass through."""
    v0 = (5.0 * tau15 / (32.0 * np.pi * tau0)) ** (1.0 / 3.0)
    eta = 1.0 / (8.0 * f_star * tau15 * v0 * v0)
    tau1 = 5.0 / (192.0 * np.pi * f_star * eta * v0 ** 3) * (743.0 / 336.0 + 11.0 * eta / 4.0)
    tau2 = 5.0 / (128.0 * np.pi * f_star * eta * v0) * (
        3058673.0 / 1016064.0 + 5429.0 * eta / 1008.0 + 617.0 * eta * eta / 144.0)
    return np.array([0.6 * tau0, tau1, -1.5 * tau15, 3.0 * tau2]) * f_star


def _sky_maps(alpha, delta, tensors, pos_m):
    """U (D x 2, psi = 0) and delays (D,), complex-step safe."""
    ca, sa, cd, sd = np.cos(alpha), np.sin(alpha), np.cos(delta), np.sin(delta)
    ex = -np.array([-sa, ca, 0.0 * ca])
    ey = np.array([-sd * ca, -sd * sa, cd])
    e_plus = np.outer(ex, ex) - np.outer(ey, ey)
    e_cross = np.outer(ex, ey) + np.outer(ey, ex)
    U = np.stack([np.einsum("iab,ab->i", tensors, e_plus),
                  np.einsum("iab,ab->i", tensors, e_cross)], axis=1)
    n = np.array([cd * ca, cd * sa, sd])
    dl = -(np.asarray(pos_m) @ n) / C_MPS
    return U, dl


def fitness_gradient(seg: Segment, pos_m, tensors, theta, j=None):
    """Returns (Gamma^2_{j*}, j*, grad[4]) with grad = d Gamma^2 / d theta at fixed j*.

    If j is None the maximising sample of oracle.fitness is used.
    """
    theta = np.asarray(theta, dtype=np.float64)
    if j is None:
        _, j = fitness(seg, pos_m, tensors, theta)
    alpha, delta, tau0, tau15 = theta
    f_star = seg.f_low
    N = seg.n_samples
    k = seg.bins
    f = seg.freqs
    x = f / f_star
    basis = np.stack([x ** (-5.0 / 3.0), x ** -1.0, x ** (-2.0 / 3.0), x ** (-1.0 / 3.0)])   # (4, K)

    coef = _phase_coefficients(tau0, tau15, f_star)
    U, dl = _sky_maps(alpha, delta, tensors, pos_m)
    V = seg.sigma[:, None] * U
    phi = coef @ basis

    # complex-step derivatives of the scalar maps
    dcoef = np.zeros((4, 4))       # [param, coefficient]
    dV = np.zeros((4,) + V.shape)  # [param, D, 2]
    ddl = np.zeros((4, dl.size))   # [param, D]
    dcoef[2] = np.imag(_phase_coefficients(tau0 + 1j * _H, tau15, f_star)) / _H
    dcoef[3] = np.imag(_phase_coefficients(tau0, tau15 + 1j * _H, f_star)) / _H
    for q, (a, d) in ((0, (alpha + 1j * _H, delta)), (1, (alpha, delta + 1j * _H))):
        Uq, dlq = _sky_maps(a, d, tensors, pos_m)
        dV[q] = seg.sigma[:, None] * np.imag(Uq) / _H
        ddl[q] = np.imag(dlq) / _H

    D = seg.y.shape[0]
    z = np.empty(D, dtype=np.complex128)
    dz = np.zeros((4, D), dtype=np.complex128)
    for i in range(D):
        a_i = seg.y[i] * np.exp(2j * math.pi * (phi + f * dl[i] + k * j / N))
        z[i] = np.sum(a_i)
        for q in range(4):
            dphase = dcoef[q] @ basis + f * ddl[q, i]
            dz[q, i] = 2j * math.pi * np.sum(a_i * dphase)

    c, s = z.real, -z.imag
    G = V.T @ V
    Gi = np.linalg.inv(G)
    Xc, Xs = V.T @ c, V.T @ s
    g2 = float(Xc @ Gi @ Xc + Xs @ Gi @ Xs)
    grad = np.zeros(4)
    for q in range(4):
        dc, ds = dz[q].real, -dz[q].imag
        dG = dV[q].T @ V + V.T @ dV[q]
        dXc = dV[q].T @ c + V.T @ dc
        dXs = dV[q].T @ s + V.T @ ds
        grad[q] = (2.0 * Xc @ Gi @ dXc - Xc @ Gi @ dG @ Gi @ Xc
                   + 2.0 * Xs @ Gi @ dXs - Xs @ Gi @ dG @ Gi @ Xs)
    return g2, int(j), grad
