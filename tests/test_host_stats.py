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


def test_h1_table_rejects_duplicate_segments():
    """Two outputs holding the same segment of one SNR (e.g. a rerun) are an
    error, not a silent overwrite that would shrink the sample."""
    from paper_2002_02150_amd.detection import h1_table
    a = {"snr": 10.0, "values": {0: {"rho": 9.5, "rho0": 9.6}, 1: {"rho": 9.0, "rho0": 9.4}}}
    b = {"snr": 10.0, "values": {1: {"rho": 9.8, "rho0": 9.7}}}
    with pytest.raises(ValueError):
        h1_table(9.2, [a, b])


def test_chirp_duration_of_the_papers_binary():
    """The search modules place the paper's signals by the time from f_* to
    coalescence: 1.5 + 1.5 Msun from f_* = 10 Hz lasts 15.1 min (Sec. V), and
    it agrees with the oracle's chirp-time sum."""
    import json
    import os
    from oracle import fitness as F
    from paper_2002_02150_amd.params import chirp_duration
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_chirp_example.json")))
    d = chirp_duration(g["m1_msun"], g["m2_msun"], g["f_star_hz"])
    assert round(d / 60.0, g["duration_printed_digits"]) == g["duration_min"]
    t0, t15 = F.chirp_times_from_masses(1.4, 1.7, 30.0)
    t1, t2 = F.higher_chirp_times(t0, t15, 30.0)
    assert chirp_duration(1.4, 1.7, 30.0) == pytest.approx(t0 + t1 - t15 + t2, rel=1e-12)


def test_paper_sources_are_the_printed_locations():
    """L4 and L5 of Sec. V: alpha, delta in degrees, psi = 30 deg, 1.5 + 1.5 Msun."""
    import math
    import synth
    rng = np.random.default_rng(0)
    for name, (a, d) in (("L4", (32.09, -53.86)), ("L5", (150.11, -60.16))):
        inj = synth.paper_source(name, rng, 123)
        assert inj["alpha"] == pytest.approx(math.radians(a)) and inj["delta"] == pytest.approx(math.radians(d))
        assert inj["psi"] == pytest.approx(math.radians(30.0)) and (inj["m1"], inj["m2"]) == (1.5, 1.5)
        assert inj["tc_sample"] == 123 and -1 <= inj["cos_iota"] <= 1 and 0 <= inj["phi_c"] < 2 * math.pi


def test_detection_rows_by_location():
    """Per-location detection probabilities and losses (the paper's detection
    table separates L4 and L5)."""
    from paper_2002_02150_amd.detection import h1_rows
    r1 = [9.6, 9.0, 9.7, 8.0]
    r0 = [9.7, 9.6, 9.4, 9.55]
    row = h1_rows(10.0, r1, r0, ["L4", "L4", "L5", "L5"], 9.5)
    assert row["segments"] == 4 and row["detection_probability"] == 0.5
    assert row["l_dp"] == pytest.approx(2 / 3)
    assert row["by_location"]["L4"]["detection_probability"] == 0.5 and row["by_location"]["L4"]["l_dp"] == 0.5
    assert row["by_location"]["L5"]["detection_probability"] == 0.5 and row["by_location"]["L5"]["l_dp"] == 1.0


def _ks_perm_pvalue(a, b):
    """Exact two-sample KS p-value by enumeration: the fraction of the splits
    of the pooled sample into groups of len(a) and len(b) whose statistic is at
    least the observed one (distinct values, so the split fixes the ranks)."""
    import itertools
    pool = sorted(a + b)

    def d(x, y):
        return max(abs(sum(v <= t for v in x) / len(x) - sum(v <= t for v in y) / len(y)) for t in pool)
    d0 = d(a, b)
    splits = list(itertools.combinations(range(len(pool)), len(a)))
    hits = sum(d([pool[i] for i in c], [pool[i] for i in range(len(pool)) if i not in c]) >= d0 - 1e-12
               for c in splits)
    return hits / len(splits)


def test_detection_rows_location_ks_test():
    """The two-sample KS test between the locations' rho' samples (Sec. V),
    on all values and on those above 9.0, against the exact permutation
    p-value by enumeration."""
    from paper_2002_02150_amd.detection import h1_rows
    a, b = [8.0, 9.1, 9.2, 9.3], [8.5, 9.4, 9.5, 9.6]
    row = h1_rows(9.0, a + b, [10.0] * 8, ["L4"] * 4 + ["L5"] * 4, 9.5)
    assert row["ks_pvalue_locations"] == pytest.approx(_ks_perm_pvalue(a, b), rel=1e-9)
    assert row["ks_pvalue_locations_above_9"] == pytest.approx(_ks_perm_pvalue(a[1:], b[1:]), rel=1e-9)
    assert row["ks_pvalue_locations_above_9"] == pytest.approx(0.1)      # 2 of the 20 splits of 3 + 3 separate fully


def test_hour_h0_combine_checks():
    """The hour-long H0 outputs combine into one lognormal fit only when they
    share a band and no slide appears twice."""
    from paper_2002_02150_amd.detection import combine
    rng = np.random.default_rng(3)
    a = dict(rho={str(s): float(v) for s, v in zip(range(1, 9), rng.lognormal(2.1, 0.03, 8))}, iterations=500,
             runs=12, f_low=10.0)
    b = dict(rho={str(s): float(v) for s, v in zip(range(9, 17), rng.lognormal(2.1, 0.03, 8))}, iterations=500,
             runs=12, f_low=10.0)
    c = combine([a, b])
    assert c["segments_h0"] == 16 and c["f_low"] == 10.0 and c["eta"] > max(max(a["rho"].values()), 8.0)
    with pytest.raises(ValueError):
        combine([a, a])
    with pytest.raises(ValueError):
        combine([a, dict(b, f_low=30.0)])


def test_tuning_metric_bootstrap():
    """The bootstrap of M(N_runs, N_iter) (Sec. V.A): all runs above the truth
    give 0, all below give 1; with one realization whose two runs straddle the
    truth, a draw of N_runs runs with replacement ends below it with
    probability 2^-N_runs, which the bootstrap mean reproduces."""
    from paper_2002_02150_amd.tuning_metric import bootstrap_metric
    above = [dict(rho0_sq=100.0, run_best={"500": [101.0, 120.0, 100.5]}) for _ in range(5)]
    below = [dict(rho0_sq=100.0, run_best={"500": [90.0, 99.0, 80.0]}) for _ in range(5)]
    assert bootstrap_metric(above, 2, 500, n_boot=200) == ([0.0, 0.0], 0.0)
    assert bootstrap_metric(below, 2, 500, n_boot=200) == ([1.0, 1.0], 1.0)
    mixed = [dict(rho0_sq=100.0, run_best={"500": [90.0, 110.0]})]
    for m in (1, 2, 3):
        _, mean = bootstrap_metric(mixed, m, 500, n_boot=20000, seed=m)
        assert mean == pytest.approx(0.5 ** m, abs=0.015)
    (p1, p99), _ = bootstrap_metric(above[:3] + below[:2], 1, 500, n_boot=4000)
    assert 0.0 <= p1 < 0.4 < p99 <= 1.0


def test_full_search_layout_tiles_the_data():
    """The overlapping segments of the full-length search cover the data up to
    its last sample, and their searched coalescence ranges tile [0, total)
    with no gap or overlap, for the hour's 56 segments and other counts."""
    from paper_2002_02150_amd.full_search import SEG, layout
    for total, n in ((7372800, 56), (491520, 3), (2 * SEG, 2), (1000003, 7), (SEG + 5, 2)):
        starts, stride, ranges = layout(total, n)
        assert len(starts) == len(ranges) == n
        assert starts[0] == 0 and starts[-1] + SEG == total
        assert all(0 < b - a <= stride + n - 2 for a, b in zip(starts, starts[1:]))
        end = 0
        for s, (lo, hi) in zip(starts, ranges):
            assert 0 <= lo < hi <= SEG
            assert s + lo == end
            end = s + hi
        assert end == total
    with pytest.raises(ValueError):
        layout(10 * SEG, 3)          # windows too far apart to overlap
    with pytest.raises(ValueError):
        layout(SEG - 1, 2)
