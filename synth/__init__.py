"""Seeded synthetic inputs shared by the oracle-side tests and the GPU-side runs.

This module draws random numbers and describes the measurement set-up (detector
sites, the noise spectrum, the search rectangle).  It holds none of the fitness
arithmetic: no template phase, no antenna contraction, no inner product.  Both
the CPU oracle and the HIP library receive what it produces as plain arrays.

Recipe (data model of Sec. II, noise model of Sec. II.A):
  * one-sided PSD  S(f) = S0 [x^-4.14 - 5 x^-2 + 111 (1 - x^2 + x^4/2)/(1 + x^2/2)],
    x = f / 215 Hz, S0 = 1 (an analytic aLIGO-like curve, used for every detector
    because the per-detector design curves of Fig. 1 are not available);
  * frequency-domain Gaussian noise with E|n(f_k)|^2 = T S(f_k) / 2 in
    continuum Fourier units (dt times the DFT), independent per detector;
  * detector sites and arm directions for H, L, V, K (approximate published
    values; the fitness only ever sees the resulting vertex positions and
    response tensors);
  * injection parameters: masses U[1,3] Msun, isotropic sky, uniform
    polarisation / phase / cos(inclination), integer coalescence sample.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

ROOT_SEED = 20020215

# WGS-84 ellipsoid
_WGS84_A = 6378137.0
_WGS84_E2 = 0.00669437999014

# name: (geodetic latitude deg, longitude deg (east +), elevation m,
#        x-arm azimuth deg clockwise from north, y-arm azimuth deg)
# Approximate site values; good to a fraction of a degree, which is all a
# synthetic benchmark needs.
DETECTOR_SITES = {
    "H": (46.4551, -119.4077, 142.6, 324.0, 234.0),
    "L": (30.5629, -90.7742, -6.6, 252.3, 162.3),
    "V": (43.6314, 10.5045, 51.9, 19.4, 289.4),
    "K": (36.4119, 137.3060, 414.2, 60.4, 150.4),
}


@dataclass(frozen=True)
class Network:
    """Detector vertices (ECEF, metres) and response tensors D = (a a^T - b b^T)/2."""
    names: tuple
    pos_m: np.ndarray      # (D, 3) float64
    tensor: np.ndarray     # (D, 3, 3) float64

    @property
    def n_det(self) -> int:
        return len(self.names)


def _site_vectors(lat_deg, lon_deg, elev_m, xaz_deg, yaz_deg):
    lat, lon = math.radians(lat_deg), math.radians(lon_deg)
    sl, cl, so, co = math.sin(lat), math.cos(lat), math.sin(lon), math.cos(lon)
    nrad = _WGS84_A / math.sqrt(1.0 - _WGS84_E2 * sl * sl)
    pos = np.array([(nrad + elev_m) * cl * co,
                    (nrad + elev_m) * cl * so,
                    (nrad * (1.0 - _WGS84_E2) + elev_m) * sl])
    east = np.array([-so, co, 0.0])
    north = np.array([-sl * co, -sl * so, cl])

    def arm(az_deg):
        z = math.radians(az_deg)
        return math.sin(z) * east + math.cos(z) * north

    return pos, arm(xaz_deg), arm(yaz_deg)


def network(names="HLVK") -> Network:
    """Vertices and response tensors for the named sites, in the given order."""
    pos, ten = [], []
    for n in names:
        p, a, b = _site_vectors(*DETECTOR_SITES[n])
        pos.append(p)
        ten.append(0.5 * (np.outer(a, a) - np.outer(b, b)))
    return Network(tuple(names), np.array(pos), np.array(ten))


def custom_network(pos_m, arms_a, arms_b, names=None) -> Network:
    """A network from explicit vertices and unit arm vectors (tests use this)."""
    pos_m = np.asarray(pos_m, dtype=np.float64).reshape(-1, 3)
    a = np.asarray(arms_a, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(arms_b, dtype=np.float64).reshape(-1, 3)
    ten = 0.5 * (np.einsum("ia,ib->iab", a, a) - np.einsum("ia,ib->iab", b, b))
    if names is None:
        names = tuple(f"D{i}" for i in range(len(pos_m)))
    return Network(tuple(names), pos_m, ten)


def psd_analytic(f, s0: float = 1.0):
    """One-sided PSD of the aLIGO-like analytic curve; +inf at f <= 0."""
    f = np.asarray(f, dtype=np.float64)
    out = np.full(f.shape, np.inf)
    m = f > 0
    x = f[m] / 215.0
    out[m] = s0 * (x ** -4.14 - 5.0 * x ** -2 + 111.0 * (1.0 - x * x + 0.5 * x ** 4) / (1.0 + 0.5 * x * x))
    return out


# Per-detector stand-ins for the detector noise curves (which are not
# available here): the analytic curve with its knee moved and its level
# scaled, and narrow spectral lines (mains harmonics, suspension
# resonances) on some detectors.  Row i uses entry i mod 4.
NETWORK_KNEES = (215.0, 170.0, 260.0, 300.0)
NETWORK_SCALES = (1.0, 2.2, 0.6, 3.5)
NETWORK_LINES = (((60.0, 2.0, 40.0), (120.0, 2.0, 10.0)), ((500.0, 3.0, 300.0),), (), ((50.0, 1.5, 80.0),))


def psd_network(n_det: int, n_samples: int, fs: float):
    """(D, N/2+1) float64 PSD rows that differ between detectors (knee, level
    and lines; see NETWORK_*): each detector gets its own sigma_i and
    over-whitening."""
    f = np.arange(n_samples // 2 + 1) * (fs / n_samples)
    rows = []
    for i in range(n_det):
        k = i % 4
        row = psd_analytic(f * (215.0 / NETWORK_KNEES[k]), NETWORK_SCALES[k])
        for f_line, width, height in NETWORK_LINES[k]:
            row = row * (1.0 + height * np.exp(-0.5 * ((f - f_line) / width) ** 2))
        rows.append(row)
    return np.stack(rows)


def psd_matrix(n_det: int, n_samples: int, fs: float, s0: float = 1.0):
    """(D, N/2+1) float64 PSD rows, one per detector (all the same curve)."""
    f = np.arange(n_samples // 2 + 1) * (fs / n_samples)
    row = psd_analytic(f, s0)
    return np.tile(row, (n_det, 1))


def seed_sequence(cfg: int, realization: int, det: int = 0) -> np.random.SeedSequence:
    return np.random.SeedSequence([ROOT_SEED, cfg, realization, det])


def fd_noise(rng: np.random.Generator, psd_row, n_samples: int, fs: float):
    """One-sided FD Gaussian noise, continuum units: n_k = sqrt(T S_k / 4) (g + i g').

    DC and Nyquist (and any bin with an infinite PSD) are set to zero.
    """
    T = n_samples / fs
    psd_row = np.asarray(psd_row, dtype=np.float64)
    g = rng.standard_normal((2, psd_row.size))
    amp = np.zeros_like(psd_row)
    ok = np.isfinite(psd_row)
    amp[ok] = np.sqrt(T * psd_row[ok] / 4.0)
    out = amp * (g[0] + 1j * g[1])
    out[0] = 0.0
    if n_samples % 2 == 0:
        out[-1] = 0.0
    return out


def noise_matrix(cfg: int, realization: int, psd, n_samples: int, fs: float):
    """(D, N/2+1) complex128 noise, detector i drawn from seed (cfg, realization, i)."""
    psd = np.atleast_2d(psd)
    rows = [fd_noise(np.random.default_rng(seed_sequence(cfg, realization, i)), psd[i], n_samples, fs)
            for i in range(psd.shape[0])]
    return np.array(rows)


def draw_injection(rng: np.random.Generator, n_samples: int, m_lo=1.0, m_hi=3.0):
    """Random source: component masses, sky, polarisation, phase, inclination, on-grid t_c."""
    m1, m2 = rng.uniform(m_lo, m_hi, size=2)
    return dict(
        m1=float(m1), m2=float(m2),
        alpha=float(rng.uniform(0.0, 2.0 * math.pi)),
        delta=float(math.asin(rng.uniform(-1.0, 1.0))),
        psi=float(rng.uniform(0.0, math.pi)),
        phi_c=float(rng.uniform(0.0, 2.0 * math.pi)),
        cos_iota=float(rng.uniform(-1.0, 1.0)),
        tc_sample=int(rng.integers(0, n_samples)),
    )


def uniform_in_box(rng: np.random.Generator, n: int, lo, hi):
    """n points uniform in the rectangle [lo, hi] (4 coordinates each), float64."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return lo + rng.random((n, lo.size)) * (hi - lo)


def near_point(rng: np.random.Generator, n: int, centre, lo, hi, frac=0.01):
    """n points centre + frac * (box width) * U[-1, 1]^4."""
    centre = np.asarray(centre, dtype=np.float64)
    w = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    return centre + frac * w * rng.uniform(-1.0, 1.0, size=(n, centre.size))


# Search rectangle in (alpha, delta, tau0, tau1.5) at f_* = 30 Hz covering
# component masses in [1, 3] Msun.  The chirp-time corners were written by
# tests/golden/make_golden.py from the oracle's mass-to-chirp-time map.
# Rounded outwards to 6 significant digits.
SEARCH_BOX_30HZ_LO = (0.0, -math.pi / 2, 15.0336, 0.841913)
SEARCH_BOX_30HZ_HI = (2.0 * math.pi, math.pi / 2, 93.8141, 1.75126)


def td_noise(rng: np.random.Generator, n_samples: int, fs: float, f_min: float = 20.0, s0: float = 1.0):
    """Real Gaussian time series of n_samples at fs whose one-sided PSD is the
    analytic curve above f_min and zero below it (no power far below the band,
    so cutting segments out of the series leaks none into it).

    Drawn in the frequency domain in continuum units, n_k = sqrt(T S_k / 4)
    (g + i g'), then x = fs * irfft(n) (continuum units are dt times the DFT)."""
    f = np.arange(n_samples // 2 + 1) * (fs / n_samples)
    psd = psd_analytic(f, s0)
    psd[f < f_min] = np.inf            # fd_noise leaves those bins at zero
    return fs * np.fft.irfft(fd_noise(rng, psd, n_samples, fs), n=n_samples)


def segment_fd(x, start: int, n_samples: int, fs: float):
    """One-sided Fourier data (continuum units, dt times the DFT) of the
    rectangular window x[start : start + n_samples]."""
    return np.fft.rfft(x[start:start + n_samples]) / fs


# Source locations of the paper's simulated signals (Sec. V): sky position in
# degrees (alpha, delta) and the polarisation angle psi in degrees; both use
# equal component masses of 1.5 Msun.  L4 and L5 are the best and the worst
# conditioned antenna-pattern matrices of the HLVK network among the
# locations of the earlier work the paper draws them from.
PAPER_SOURCES = {"L4": (32.09, -53.86), "L5": (150.11, -60.16)}
PAPER_PSI_DEG = 30.0
PAPER_MASSES = (1.5, 1.5)


def paper_source(name: str, rng: np.random.Generator, tc_sample: int):
    """An injection at the paper's location `name` (L4 or L5), psi = 30 deg,
    1.5 + 1.5 Msun; the paper leaves the coalescence phase and the inclination
    unstated, so they are drawn uniformly (phi_c in [0, 2 pi), cos iota in
    [-1, 1])."""
    a, d = PAPER_SOURCES[name]
    return dict(m1=PAPER_MASSES[0], m2=PAPER_MASSES[1], alpha=math.radians(a), delta=math.radians(d),
                psi=math.radians(PAPER_PSI_DEG), phi_c=float(rng.uniform(0.0, 2.0 * math.pi)),
                cos_iota=float(rng.uniform(-1.0, 1.0)), tc_sample=int(tc_sample))
