"""Seeded test cases built from synth (inputs) and, for injections, the oracle's
signal model.  Test-side only."""
from __future__ import annotations

import math

import numpy as np

import synth
from oracle import fitness as F
from oracle import signal as S


class Case:
    def __init__(self, names, n_samples, fs, f_low=30.0, f_high=1000.0, snr=None, noise=True,
                 cfg=0, realization=0, inj_seed=None, s0=1.0, psd="same"):
        self.net = synth.network(names)
        self.n_samples, self.fs, self.f_low, self.f_high = n_samples, fs, f_low, f_high
        D = self.net.n_det
        # "same": one analytic curve for every detector; "network": a distinct
        # curve per detector (synth.psd_network)
        self.psd = synth.psd_matrix(D, n_samples, fs, s0) if psd == "same" else synth.psd_network(D, n_samples, fs)
        xf = np.zeros((D, n_samples // 2 + 1), dtype=np.complex128)
        if noise:
            xf += synth.noise_matrix(cfg, realization, self.psd, n_samples, fs)
        self.inj = None
        self.theta0 = None
        if snr is not None:
            rng = np.random.default_rng(synth.seed_sequence(cfg, realization, 1000 if inj_seed is None else inj_seed))
            inj = synth.draw_injection(rng, n_samples)
            t0, t15 = F.chirp_times_from_masses(inj["m1"], inj["m2"], f_low)
            self.theta0 = np.array([inj["alpha"], inj["delta"], t0, t15])
            self.hf = S.injection(n_samples, fs, f_low, f_high, self.net.pos_m, self.net.tensor, self.psd,
                                  self.theta0, inj["psi"], inj["phi_c"], inj["cos_iota"], inj["tc_sample"],
                                  snr=snr)
            xf += self.hf
            self.inj = inj
        self.xf = xf
        self.seg = F.prepare_segment(xf, self.psd, fs, f_low, f_high)

    @property
    def box(self):
        return np.array(synth.SEARCH_BOX_30HZ_LO), np.array(synth.SEARCH_BOX_30HZ_HI)

    def fitness(self, theta):
        return F.fitness(self.seg, self.net.pos_m, self.net.tensor, theta)

    def series(self, theta, psi=0.0):
        return F.gamma2_series(self.seg, self.net.pos_m, self.net.tensor, theta, psi)


def random_thetas(rng, n, lo=None, hi=None):
    lo = synth.SEARCH_BOX_30HZ_LO if lo is None else lo
    hi = synth.SEARCH_BOX_30HZ_HI if hi is None else hi
    return synth.uniform_in_box(rng, n, lo, hi)


def two_pi():
    return 2.0 * math.pi
