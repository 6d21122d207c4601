"""Host-side statistics of the campaign modules (no GPU)."""
import numpy as np
import pytest


def test_lognormal_threshold_closed_form():
    """The detection threshold of a lognormal fit: for values whose logarithms
    have sample mean mu and standard deviation sigma, eta = exp(mu + sigma z)
    with z the standard normal quantile at 1 - p (exact for any sample)."""
    import math
    from scipy import stats
    from paper_2002_02150_amd.detection import lognormal_threshold
    rng = np.random.default_rng(5)
    vals = np.exp(rng.normal(2.1, 0.03, 500))
    p = 1.14e-4
    eta, mu, sd, _ = lognormal_threshold(vals, p)
    lv = np.log(vals)
    assert mu == pytest.approx(lv.mean(), rel=1e-14) and sd == pytest.approx(lv.std(), rel=1e-14)
    assert eta == pytest.approx(math.exp(lv.mean() + lv.std() * stats.norm.ppf(1 - p)), rel=1e-12)


def test_h1_table_counts():
    """Detection probability P(rho' >= eta) and the loss L_DP = P(rho' <= eta |
    rho0 >= eta) are counted per SNR over the segments of several runs."""
    from paper_2002_02150_amd.detection import h1_table
    a = {"snr": 10.0, "values": {0: {"rho": 9.5, "rho0": 9.6}, 1: {"rho": 9.0, "rho0": 9.4}}}
    b = {"snr": 10.0, "values": {2: {"rho": 9.8, "rho0": 9.7}, 3: {"rho": 8.0, "rho0": 8.5}}}
    c = {"snr": 12.0, "values": {0: {"rho": 12.0, "rho0": 11.9}}}
    t = h1_table(9.2, [a, b, c])["table"]
    assert [r["snr"] for r in t] == [10.0, 12.0]
    assert t[0]["segments"] == 4 and t[0]["detection_probability"] == 0.5
    assert t[0]["truth_above_eta"] == 3 and t[0]["l_dp"] == pytest.approx(1 / 3)
    assert t[1]["detection_probability"] == 1.0 and t[1]["l_dp"] == 0.0
