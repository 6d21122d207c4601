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
