"""Pins of the FP64 oracle to things other than itself: numbers the paper prints,
textbook closed forms, brute force on tiny inputs, invariances and statistics.

Each test names the part of the oracle it pins and the mistake it would catch.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import fitness as F
from oracle import gradient as G
from oracle import signal as S
from tests._cases import Case, random_thetas

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- chirp times

def test_paper_duration_of_1p5_1p5_binary():
    """Sec. V: 1.5+1.5 Msun from f* = 10 Hz lasts 15.1 min.  The time to
    coalescence from f* in the chirp-time family is tau0 + tau1 - tau1.5 + tau2,
    so this pins the tau0/tau1.5 definitions and the 1PN / 2PN constants of
    tau1 and tau2 (a wrong constant moves the duration by seconds)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_chirp_example.json")))
    t0, t15 = F.chirp_times_from_masses(g["m1_msun"], g["m2_msun"], g["f_star_hz"])
    t1, t2 = F.higher_chirp_times(t0, t15, g["f_star_hz"])
    dur_min = (t0 + t1 - t15 + t2) / 60.0
    assert round(dur_min, g["duration_printed_digits"]) == pytest.approx(g["duration_min"])
    # the same injection lies inside the paper's PSO search rectangle
    assert g["tau0_box_s"][0] < t0 < g["tau0_box_s"][1]
    assert g["tau15_box_s"][0] < t15 < g["tau15_box_s"][1]


def test_chirp_time_roundtrip_recovers_masses():
    """tau -> (v0, eta) -> masses -> tau is the identity (catches a wrong inverse)."""
    for m1, m2 in [(1.0, 1.0), (1.4, 2.7), (3.0, 1.1)]:
        t0, t15 = F.chirp_times_from_masses(m1, m2, 30.0)
        v0, eta = F.mass_params_from_chirp_times(t0, t15, 30.0)
        M = v0 ** 3 / (math.pi * 30.0) / F.GM_SUN_S
        assert M == pytest.approx(m1 + m2, rel=1e-12)
        assert eta == pytest.approx(m1 * m2 / (m1 + m2) ** 2, rel=1e-12)


def _taylorf2_phase_rad(f, m1, m2):
    """Textbook restricted-2PN TaylorF2 phase in the (M, eta, v) form, without
    the t_c / phi_c terms: 3/(128 eta v^5) [1 + 20/9 (743/336 + 11 eta/4) v^2
    - 16 pi v^3 + 10 (3058673/1016064 + 5429 eta/1008 + 617 eta^2/144) v^4],
    v = (pi G M f / c^3)^(1/3)."""
    M = (m1 + m2) * F.GM_SUN_S
    eta = m1 * m2 / (m1 + m2) ** 2
    v = (math.pi * M * f) ** (1.0 / 3.0)
    return 3.0 / (128.0 * eta * v ** 5) * (
        1.0 + 20.0 / 9.0 * (743.0 / 336.0 + 11.0 * eta / 4.0) * v ** 2 - 16.0 * math.pi * v ** 3
        + 10.0 * (3058673.0 / 1016064.0 + 5429.0 * eta / 1008.0 + 617.0 * eta ** 2 / 144.0) * v ** 4)


@pytest.mark.parametrize("m1,m2,fstar", [(1.5, 1.5, 10.0), (1.0, 3.0, 30.0), (2.2, 1.3, 30.0)])
def test_phase_equals_textbook_taylorf2(m1, m2, fstar):
    """The chirp-time phase equals the (M, eta) TaylorF2 2PN phase term by term
    (catches a wrong coefficient 3/5, 1, -3/2, 3 or a wrong power of x)."""
    f = np.linspace(fstar * 1.01, 1000.0, 2001)
    t0, t15 = F.chirp_times_from_masses(m1, m2, fstar)
    ours = 2.0 * math.pi * F.phase_cycles(f, t0, t15, fstar)
    ref = _taylorf2_phase_rad(f, m1, m2)
    assert np.max(np.abs(ours - ref)) < 1e-9 * np.max(np.abs(ref)) + 1e-9


# ---------------------------------------------------------------- geometry

def test_antenna_pattern_textbook_closed_form():
    """Detector at the north pole with arms along the Earth-fixed x and y axes:
    F+^2 + Fx^2 = [(1 + cos^2 t)/2]^2 cos^2 2p + cos^2 t sin^2 2p with t the
    source's polar angle and p its azimuth (textbook L-shaped detector
    response).  Catches a transposed or sign-flipped polarisation tensor."""
    net = synth.custom_network([[0.0, 0.0, 6.4e6]], [[1.0, 0.0, 0.0]], [[0.0, 1.0, 0.0]])
    rng = np.random.default_rng(5)
    for _ in range(50):
        alpha = rng.uniform(0, 2 * math.pi)
        delta = math.asin(rng.uniform(-1, 1))
        psi = rng.uniform(0, math.pi)
        fp, fc = F.antenna_patterns(alpha, delta, psi, net.tensor)
        th, ph = math.pi / 2 - delta, alpha
        ref = (0.5 * (1 + math.cos(th) ** 2)) ** 2 * math.cos(2 * ph) ** 2 + math.cos(th) ** 2 * math.sin(2 * ph) ** 2
        assert fp[0] ** 2 + fc[0] ** 2 == pytest.approx(ref, abs=1e-12)
        # zenith source, psi = 0: F+ = cos 2p-type response is maximal, |F| = 1
    fp, fc = F.antenna_patterns(0.0, math.pi / 2, 0.0, net.tensor)
    assert fp[0] ** 2 + fc[0] ** 2 == pytest.approx(1.0, abs=1e-12)


def test_polarisation_rotation_is_spin_two():
    """F(psi) = U R(2 psi): the pair rotates by twice the polarisation angle."""
    net = synth.network("HLV")
    a, d, psi = 1.1, -0.4, 0.37
    U = F.template_matrix_U(a, d, net.tensor)
    fp, fc = F.antenna_patterns(a, d, psi, net.tensor)
    c, s = math.cos(2 * psi), math.sin(2 * psi)
    assert np.allclose(fp, U[:, 0] * c + U[:, 1] * s, atol=1e-12)
    assert np.allclose(fc, -U[:, 0] * s + U[:, 1] * c, atol=1e-12)


def test_delay_arrival_order():
    """A source straight above a detector reaches it before the Earth's centre
    (negative delay of |r|/c), and the antipodal source reverses every delay."""
    net = synth.network("HLVK")
    for i in range(4):
        r = net.pos_m[i]
        alpha = math.atan2(r[1], r[0])
        delta = math.asin(r[2] / np.linalg.norm(r))
        dl = F.delays(alpha, delta, net.pos_m)
        assert dl[i] == pytest.approx(-np.linalg.norm(r) / F.C_MPS, rel=1e-12)
        assert np.argmin(dl) == i
        anti = F.delays(alpha + math.pi, -delta, net.pos_m)
        assert np.allclose(anti, -dl, atol=1e-15)


# ---------------------------------------------------------------- inner products

def test_template_norms_orthonormal():
    """<h_c|h_c> = <h_s|h_s> = sigma^2 and <h_c|h_s> = 0 (Sec. II.D) with the
    literal inner product of eq. innprod; catches a wrong f^-7/3 or 4 df."""
    n, fs = 8192, 1024.0
    psd = synth.psd_matrix(1, n, fs)[0]
    k_lo, k_hi = F.band_bins(n, fs, 30.0, 1000.0)
    df = fs / n
    hc, hs = S.spa_polarisations(n, fs, 30.0, 1000.0, 40.0, 1.3, 0.7, 0.0, 1.0, 1.0)
    sig = F.template_norms(psd, n, fs, 30.0, 1000.0)[0]
    assert S.inner_product(hc, hc, psd, df, k_lo, k_hi) == pytest.approx(sig ** 2, rel=1e-13)
    assert S.inner_product(hs, hs, psd, df, k_lo, k_hi) == pytest.approx(sig ** 2, rel=1e-13)
    assert abs(S.inner_product(hc, hs, psd, df, k_lo, k_hi)) < 1e-13 * sig ** 2


def test_band_edges_config_sizes():
    """Band bins at the benchmark sizes (30 < f <= min(1000, fs/2), DC and
    Nyquist out)."""
    assert F.band_bins(8192, 1024.0, 30.0, 1000.0) == (241, 4095)
    assert F.band_bins(131072, 2048.0, 30.0, 1000.0) == (1921, 64000)
    k_lo, k_hi = F.band_bins(262144, 2048.0, 30.0, 1000.0)
    assert k_hi - k_lo + 1 == 124160


@pytest.mark.parametrize("n", [256, 512])
def test_matched_filter_equals_naive_dft(n):
    """z^i_j from the FFT equals the defining double sum on tiny inputs."""
    case = Case("HL", n, 512.0, f_low=30.0, f_high=200.0, cfg=90, realization=n)
    theta = np.array([0.3, -0.2, 40.0, 1.2])
    z = F.matched_filter_series(case.seg, case.net.pos_m, theta)
    f = case.seg.freqs
    k = case.seg.bins
    phi = F.phase_cycles(f, theta[2], theta[3], case.f_low)
    dl = F.delays(theta[0], theta[1], case.net.pos_m)
    for i in range(2):
        for j in range(n):
            ref = 0.0j
            for kk in range(k.size):
                ref += case.seg.y[i, kk] * complex(math.cos(2 * math.pi * (phi[kk] + f[kk] * dl[i] + k[kk] * j / n)),
                                                    math.sin(2 * math.pi * (phi[kk] + f[kk] * dl[i] + k[kk] * j / n)))
            assert abs(z[i, j] - ref) < 1e-10 * (1 + abs(ref))


# ---------------------------------------------------------------- projection

def test_two_detectors_full_rank_is_sum_of_powers():
    """D = 2 with independent antenna rows: the projector is the identity and
    Gamma^2_j = |z^1_j|^2 + |z^2_j|^2 (special case of the analytic maximum)."""
    case = Case("HV", 4096, 1024.0, cfg=91)
    theta = np.array([2.0, 0.5, 30.0, 1.0])
    z = F.matched_filter_series(case.seg, case.net.pos_m, theta)
    g = case.series(theta)
    assert np.allclose(g, np.sum(np.abs(z) ** 2, axis=0), rtol=1e-10, atol=1e-10)


def test_single_detector_is_quadrature_power():
    """D = 1: rank-one projector, Gamma^2_j = |z_j|^2 (single-detector matched filter)."""
    case = Case("L", 4096, 1024.0, cfg=92)
    theta = np.array([0.1, 0.2, 50.0, 1.4])
    z = F.matched_filter_series(case.seg, case.net.pos_m, theta)
    assert np.allclose(case.series(theta), np.abs(z[0]) ** 2, rtol=1e-9, atol=1e-9)


def test_polarisation_invariance():
    """Replacing U = F(psi=0) by F(psi) for any psi leaves Gamma^2 unchanged."""
    case = Case("HLVK", 4096, 1024.0, cfg=93)
    theta = np.array([4.0, -0.9, 60.0, 1.6])
    g0 = case.series(theta)
    for psi in (0.3, 1.2, 2.9):
        assert np.allclose(case.series(theta, psi), g0, rtol=1e-10, atol=1e-10)


def test_literal_likelihood_maximised_over_amplitudes():
    """Gamma^2_j equals twice the log-likelihood ratio of eq. loglikelihood,
    built literally from the four delayed templates and the inner product of
    eq. innprod, at the amplitudes that maximise it (reading of the scale of
    Gamma^2); and those amplitudes are a maximum.  This pins over-whitening,
    the template norm, the delay ramp and the projection together."""
    case = Case("HLV", 2048, 1024.0, snr=15, cfg=94, noise=True)
    rng = np.random.default_rng(3)
    theta = case.theta0 + np.array([0.05, -0.03, 0.1, 0.01])
    g = case.series(theta)
    for j in list(rng.integers(0, case.n_samples, 3)) + [int(np.argmax(g))]:
        t_c = j / case.fs
        b, M = S.amplitude_normal_equations(case.xf, case.psd, case.fs, case.f_low, case.f_high,
                                            case.net.tensor, case.net.pos_m, theta, t_c)
        A = np.linalg.solve(M, b)
        lam = S.loglikelihood(case.xf, case.psd, case.fs, case.f_low, case.f_high,
                              case.net.tensor, case.net.pos_m, theta, A, t_c)
        assert 2.0 * lam == pytest.approx(g[j], rel=1e-9, abs=1e-9)
        for _ in range(3):
            dA = rng.normal(size=4) * 0.05 * np.linalg.norm(A)
            lam2 = S.loglikelihood(case.xf, case.psd, case.fs, case.f_low, case.f_high,
                                   case.net.tensor, case.net.pos_m, theta, A + dA, t_c)
            assert lam2 < lam


# ---------------------------------------------------------------- end to end

@pytest.mark.parametrize("names,n,fs,psd", [("HL", 8192, 1024.0, "same"), ("HLV", 4096, 2048.0, "same"),
                                            ("HLVK", 8192, 2048.0, "same"), ("HLVK", 8192, 2048.0, "network"),
                                            ("HL", 4096, 2048.0, "network")])
def test_noiseless_injection_identity(names, n, fs, psd):
    """Noiseless signal at the true parameters: Gamma^2 = SNR^2 and the maximum
    sits at the injected coalescence sample, for random sky, polarisation,
    phase and inclination, with one noise curve or a different one per
    detector."""
    for r in range(3):
        case = Case(names, n, fs, snr=11.0, noise=False, cfg=95, realization=r, psd=psd)
        g, j = case.fitness(case.theta0)
        assert g == pytest.approx(121.0, rel=1e-10)
        assert j == case.inj["tc_sample"]


def test_injection_network_snr_definition():
    """The injection is scaled by eq. optimalSNR."""
    case = Case("HLVK", 4096, 2048.0, snr=9.0, noise=False, cfg=96)
    assert S.network_snr(case.hf, case.psd, 4096, 2048.0, 30.0, 1000.0) == pytest.approx(9.0, rel=1e-13)


def test_symmetries_roll_scale_phase():
    """Cyclic roll of the data by m samples moves j* by m with Gamma^2 unchanged;
    x -> a x scales Gamma^2 by a^2; a common complex phase changes nothing."""
    case = Case("HLV", 4096, 1024.0, snr=12.0, cfg=97)
    theta = case.theta0
    g0, j0 = case.fitness(theta)
    n = case.n_samples
    k = np.arange(n // 2 + 1)
    m = 777
    rolled = case.xf * np.exp(-2j * math.pi * k * m / n)
    seg = F.prepare_segment(rolled, case.psd, case.fs, case.f_low, case.f_high)
    g1, j1 = F.fitness(seg, case.net.pos_m, case.net.tensor, theta)
    assert g1 == pytest.approx(g0, rel=1e-10)
    assert j1 == (j0 + m) % n
    seg = F.prepare_segment(2.5 * np.exp(0.7j) * case.xf, case.psd, case.fs, case.f_low, case.f_high)
    g2, j2 = F.fitness(seg, case.net.pos_m, case.net.tensor, theta)
    assert g2 == pytest.approx(6.25 * g0, rel=1e-10)
    assert j2 == j0


@pytest.mark.parametrize("kind", ["same", "network"])
def test_noise_only_statistics_chi2(kind):
    """Under noise only, at fixed theta and j, Gamma^2_j is chi^2 with 4 degrees
    of freedom for a rank-2 network (mean 4, variance 8) and E|z^i_j|^2 = 2:
    pins the normalisation sigma and the factor 4 df of over-whitening, also
    when every detector has its own noise curve (its own sigma_i)."""
    n, fs = 1024, 512.0
    net = synth.network("HLV")
    psd = synth.psd_matrix(3, n, fs) if kind == "same" else synth.psd_network(3, n, fs)
    theta = np.array([1.0, 0.3, 40.0, 1.2])
    vals, zp = [], []
    for r in range(3000):
        xf = synth.noise_matrix(98, r, psd, n, fs)
        seg = F.prepare_segment(xf, psd, fs, 30.0, 1000.0)
        j = r % n
        vals.append(F.gamma2_at(seg, net.pos_m, net.tensor, theta, j))
        z = F.matched_filter_series(seg, net.pos_m, theta)[:, j]
        zp.append(np.abs(z) ** 2)
    vals = np.array(vals)
    m = len(vals)
    assert abs(vals.mean() - 4.0) < 3.0 * math.sqrt(8.0 / m)
    # variance of the sample variance: (mu4 - sigma^4)/m = (384 - 64)/m for chi^2_4
    assert abs(vals.var() - 8.0) < 4.0 * math.sqrt(320.0 / m)
    assert abs(np.mean(zp) - 2.0) < 3.0 * 2.0 / math.sqrt(3 * m)


# ---------------------------------------------------------------- gradient

def _fd(case, theta, j, q, h):
    """Fourth-order central difference of Gamma^2_j along coordinate q."""
    e = np.zeros(4)
    e[q] = h

    def g(t):
        return F.gamma2_at(case.seg, case.net.pos_m, case.net.tensor, t, j)

    return (8.0 * (g(theta + e) - g(theta - e)) - (g(theta + 2 * e) - g(theta - 2 * e))) / (12.0 * h)


def test_gradient_matches_central_differences():
    """Analytic dGamma^2/dtheta at fixed j* equals FP64 fourth-order central
    differences (step 1e-6 of the box width) to 1e-6 relative."""
    case = Case("HLVK", 4096, 2048.0, snr=12.0, cfg=99)
    lo, hi = case.box
    w = hi - lo
    rng = np.random.default_rng(11)
    for theta in synth.near_point(rng, 3, case.theta0, lo, hi, frac=0.01):
        g2, j, grad = G.fitness_gradient(case.seg, case.net.pos_m, case.net.tensor, theta)
        assert g2 == pytest.approx(case.fitness(theta)[0], rel=1e-12)
        fd = np.array([_fd(case, theta, j, q, 1e-6 * w[q]) for q in range(4)])
        scale = np.abs(grad) + 1e-3 * np.max(np.abs(grad * w)) / w
        assert np.all(np.abs(grad - fd) <= 1e-6 * scale), (grad, fd)


def test_gradient_vanishes_at_truth_without_noise():
    """The true parameters of a noiseless signal maximise Gamma^2_{j0}: the
    gradient there is zero (relative to the gradient scale a small step away)."""
    case = Case("HLVK", 8192, 2048.0, snr=12.0, noise=False, cfg=100)
    lo, hi = case.box
    w = hi - lo
    _, j, g_true = G.fitness_gradient(case.seg, case.net.pos_m, case.net.tensor, case.theta0)
    assert j == case.inj["tc_sample"]
    _, _, g_off = G.fitness_gradient(case.seg, case.net.pos_m, case.net.tensor, case.theta0 + 1e-3 * w, j)
    assert np.all(np.abs(g_true * w) < 1e-6 * np.max(np.abs(g_off * w)))


# ---------------------------------------------------------------- search box

def test_search_box_covers_mass_square():
    g = json.load(open(os.path.join(GOLDEN, "search_box_30hz.json")))
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    assert lo[2] <= g["tau0_s"][0] and hi[2] >= g["tau0_s"][1]
    assert lo[3] <= g["tau15_s"][0] and hi[3] >= g["tau15_s"][1]
    assert hi[2] - g["tau0_s"][1] < 1e-3 and g["tau0_s"][0] - lo[2] < 1e-3


def test_restricted_coalescence_range():
    """The maximum over a sample range is the maximum of that part of the series,
    never above the unrestricted one and equal to it when the range holds j*."""
    case = Case("HLV", 4096, 1024.0, snr=12.0, cfg=101)
    th = case.theta0
    g = case.series(th)
    f_all, j_all = case.fitness(th)
    for lo, hi in ((0, 100), (1000, 3000), (j_all, j_all + 1), (max(j_all - 7, 0), min(j_all + 9, 4096))):
        f, j = F.fitness(case.seg, case.net.pos_m, case.net.tensor, th, j_range=(lo, hi))
        assert lo <= j < hi and f == pytest.approx(np.max(g[lo:hi]), rel=1e-15)
        assert f <= f_all
        if lo <= j_all < hi:
            assert j == j_all and f == f_all
