"""End-to-end runs of the searches built on the library (tuning metric,
full-length search, detection statistics), each small, with every reported
result re-evaluated by the FP64 oracle: the fitness the search reports at the
point it reports (within 1e-4 relative), its coalescence sample (within one
sample, or a sample where the oracle's series is within 1e-4 of its maximum),
and the fitness at the injected parameters."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

import synth
from oracle import fitness as F
from tests._gpu import assert_parity, require_gpu

pytestmark = pytest.mark.gpu

FS, F_HIGH = 2048.0, 1000.0


def _check(xf, net, theta, rho_sq, argmax, f_low=30.0, box=None, j_range=None, rtol=1e-4):
    """The oracle's fitness and sample at theta against a reported (rho_sq, argmax)."""
    lo, hi = box if box is not None else (synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI)
    n = 2 * (xf.shape[1] - 1)
    psd = synth.psd_matrix(net.n_det, n, FS)
    seg = F.prepare_segment(xf, psd, FS, f_low, F_HIGH)
    th = np.asarray(theta, dtype=np.float64)[None, :]
    fo, jo = F.fitness_batch(seg, net.pos_m, net.tensor, th, np.array(lo), np.array(hi), j_range)
    case = SimpleNamespace(n_samples=n, seg=seg, net=net)
    assert_parity(case, th, np.array([rho_sq]), np.array([argmax]), fo, jo, rtol)
    return fo[0]


def test_tuning_metric_small_matches_oracle():
    """The tuning metric at the paper's location L4 (two realizations, two
    iteration counts, best of the first 2 and 4 of 12 runs): rho0^2 at the
    injected parameters and every best-of-runs rho'^2 match the oracle at the
    same points, the table is the fraction of realizations below the truth,
    and more runs never end lower."""
    require_gpu()
    from paper_2002_02150_amd import tuning_metric as T
    net = synth.network("HLVK")
    out = T.run(realizations=2, snr=12.0, n_iters=(20, 30), n_runs_list=(2, 4), source="L4", batch=2,
                keep_data=True, log=lambda s: None)
    assert out["realizations"] == 2 and set(out["table"]) == {"2x20", "4x20", "2x30", "4x30"}
    a, d = synth.PAPER_SOURCES["L4"]
    for rec in out["records"]:
        assert rec["theta0"][0] == pytest.approx(math.radians(a)) and rec["theta0"][1] == pytest.approx(math.radians(d))
        f0 = _check(rec["xf"], net, rec["theta0"], rec["rho0_sq"], _oracle_argmax(rec["xf"], net, rec["theta0"]))
        assert f0 > 100.0          # an SNR-12 signal at its true parameters
        for key, b in rec["best"].items():
            _check(rec["xf"], net, b["theta"], b["rho_sq"], b["argmax"])
        for it in (20, 30):
            assert rec["best"][f"4x{it}"]["rho_sq"] >= rec["best"][f"2x{it}"]["rho_sq"]
            # the recorded run bests (used by the bootstrap) give the same best of the first m runs
            for m in (2, 4):
                assert max(rec["run_best"][str(it)][:m]) == rec["best"][f"{m}x{it}"]["rho_sq"]
    for key, v in out["table"].items():
        assert v == np.mean([r["best"][key]["rho_sq"] < r["rho0_sq"] for r in out["records"]])


def _oracle_value(xf, net, theta, f_low=30.0, j_range=None):
    n = 2 * (xf.shape[1] - 1)
    seg = F.prepare_segment(xf, synth.psd_matrix(net.n_det, n, FS), FS, f_low, F_HIGH)
    return F.fitness(seg, net.pos_m, net.tensor, theta, j_range=j_range)[0]


def _oracle_argmax(xf, net, theta, f_low=30.0):
    n = 2 * (xf.shape[1] - 1)
    seg = F.prepare_segment(xf, synth.psd_matrix(net.n_det, n, FS), FS, f_low, F_HIGH)
    return F.fitness(seg, net.pos_m, net.tensor, theta)[1]


def test_full_search_small_matches_oracle():
    """The full-length search on a 4-minute stretch: three overlapping 128-s
    segments with per-segment coalescence ranges, one injection synthesised
    over the whole stretch and added in the time domain before the segments
    are cut.  Every segment's reported best point, fitness and sample match
    the oracle under the segment's range; the injection's rho0^2 matches the
    oracle on the segment that holds it; the polish never lowers a segment's
    best."""
    require_gpu()
    from paper_2002_02150_amd.full_search import layout, run
    net = synth.network("HLVK")
    out = run(minutes=4.0, n_seg=3, iters=30, n_inj=1, polish_steps=3, keep_data=True, log=lambda s: None)
    assert out["segments"] == 3 and out["iterations"] == 30 and out["evaluated_points"] > 0
    sd = out["segment_data"]
    starts, stride, ranges = layout(int(4 * 60 * 2048), 3)
    assert stride == out["stride_samples"] and list(sd["starts"]) == starts
    for s in range(3):
        assert sd["rho_sq"][s] >= sd["rho_sq_pso"][s] - 1e-9
        _check(sd["xf"][s], net, sd["theta"][s], sd["rho_sq"][s], sd["argmax"][s], j_range=ranges[s])
    for d in out["injections"]:
        s = d["segment"]
        assert starts[s] + ranges[s][0] <= d["tc_sample"] < starts[s] + ranges[s][1]
        assert _oracle_value(sd["xf"][s], net, d["theta0"], j_range=ranges[s]) == pytest.approx(d["rho0_sq"], rel=1e-4)
        assert d["rho0_sq"] > 64.0      # SNR 10-12, most of the chirp inside the segment


def test_detection_study_small_matches_oracle():
    """The detection study with the paper's sources: one slide of 4 noise-only
    64-s segments and one SNR-12 segment at each of L4 and L5; every segment's
    reported rho'^2, point and sample match the oracle, so do rho0^2 at the
    injected parameters, and the table reports both locations."""
    require_gpu()
    from paper_2002_02150_amd.detection import run
    net = synth.network("HLVK")
    out = run(slides=1, per_snr=1, snrs=(12.0,), iters=20, n_per_slide=4, source="paper", keep_data=True,
              log=lambda s: None)
    assert out["segments_h0"] == 4 and out["segments_h1"] == 2
    sd = out["segment_data"]
    for s in range(6):
        _check(sd["xf"][s], net, sd["theta"][s], sd["rho_sq"][s], sd["argmax"][s])
    for k in range(2):
        xf = sd["xf"][4 + k]
        _check(xf, net, sd["theta0"][k], sd["rho0_sq"][k], _oracle_argmax(xf, net, sd["theta0"][k]))
    row = out["table"][0]
    assert set(row["by_location"]) == {"L4", "L5"} and row["segments"] == 2
    assert out["eta"] > out["h0_rho_quantiles"][0.5] > 0


def test_hour_h1_paper_band_matches_oracle():
    """One hour-long segment with an SNR-12 signal at L4 in the paper's band
    and rectangle (f_* = 10 Hz, tau0 in [500, 1500] s, tau1.5 in [5, 15] s,
    arrival 20 min into the hour): the reported rho'^2, point and sample and
    rho0^2 at the injected parameters match the oracle."""
    require_gpu()
    from paper_2002_02150_amd.detection import PAPER_BOX_HI, PAPER_BOX_LO, hour_h1
    net = synth.network("HLVK")
    out = hour_h1(12.0, 0, 0, iters=6, runs=1, polish_steps=1, source="L4", f_low=10.0, keep_data=True,
                  log=lambda s: None)
    v = out["values"][0]
    box = (PAPER_BOX_LO, PAPER_BOX_HI)
    _check(v["xf"], net, v["theta"], v["rho_sq"], v["argmax"], f_low=10.0, box=box)
    _check(v["xf"], net, v["theta0"], v["rho0_sq"], _oracle_argmax(v["xf"], net, v["theta0"], 10.0), f_low=10.0,
           box=box)
    assert v["rho0"] > 10.0 and out["f_low"] == 10.0
