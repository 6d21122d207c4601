"""Detection statistics of the PSO search (Sec. V): the distribution of the
coherent search statistic rho' under H0 from time slides, its lognormal fit
and the detection threshold eta for a false-alarm rate, and under H1 the
detection probability P(rho' >= eta) and the loss in detection probability
L_DP = P(rho' <= eta | rho0 >= eta) (eq. loss_detprob), rho0 being the
statistic at the true parameters.

    python -m paper_2002_02150_amd.detection [--slides 4] [--per-snr 64] [--iters 1000]
    python -m paper_2002_02150_amd.detection --hour --slides 1-24 [--iters 500] [--runs 12]
    python -m paper_2002_02150_amd.detection --combine a.json b.json ...
    python -m paper_2002_02150_amd.detection --hour-h1 --snr 10 --segments 0-7 [--iters 1500]
    python -m paper_2002_02150_amd.detection --h1-table ETA h1a.json h1b.json ...

Data: 4 detectors (H, L, V, K), 64-s segments at 2048 Hz, analytic PSD.
- H0: an hour of seeded Gaussian noise per detector, cut into 56 consecutive
  64-s segments; each time slide s = 1..S shifts detector i circularly by
  10 s * s * i, so every slide gives 56 more noise-only network segments with
  the detectors' noise offset by at least 10 s.
- H1: per SNR, independent noise segments with one SPA injection each at that
  network SNR.  source="paper" (the default): the paper's two locations L4
  and L5 (Sec. V: sky position, psi = 30 deg, 1.5 + 1.5 Msun; phase and
  inclination drawn), per_snr segments each, the signal's frequency crossing
  f_* 8 s into the segment; source="random": component masses U[1, 3] Msun,
  isotropic sky and orientation, coalescence uniform over the middle half of
  the segment.
Search: 8 PSO runs x 40 particles x N_iter iterations per segment, all
segments of both sets one batch (campaign.search_segments), then the polish.
The threshold is taken at a false-alarm probability per segment of
FAR x T_seg (FAR = 1 per year by default) on the lognormal fitted to rho' by
maximum likelihood (mean and standard deviation of log rho').

--hour takes the paper's own segment length (Sec. V: one 60-min segment per
search, false-alarm probability 1.14e-4 per segment for 1 per year): one hour
of noise per detector, slide s = a..b shifting detector i circularly by
10 s * s * i, each slide one hour-long noise-only network segment searched
with the three-pass FFT plan (`group` segments per batch).  It prints the H0
values rho' of its slides; --combine fits the lognormal to the values of
several such runs and gives eta.  --hour-h1 searches hour-long segments of
independent noise with one SPA injection each at a network SNR and prints rho'
and rho0 (the statistic at the true parameters); --h1-table gives, for a
threshold eta, the detection probability and L_DP per SNR.
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np
import torch

from . import Context
from .campaign import search_segments
from .params import chirp_duration, chirp_times

FS, F_LOW, F_HIGH = 2048.0, 30.0, 1000.0
SEG = 131072                    # 64 s
SLIDE_S = 10.0
YEAR_S = 365.25 * 86400.0


def h0_segments(series, n_per_slide, slides):
    """Fourier data of the time-slid noise-only segments: (slide, segment) pairs."""
    import synth
    D = series.shape[0]
    out = []
    for s in range(1, slides + 1):
        slid = [np.roll(series[i], -int(round(SLIDE_S * FS)) * s * i) for i in range(D)]
        for k in range(n_per_slide):
            out.append(np.stack([synth.segment_fd(slid[i], k * SEG, SEG, FS) for i in range(D)]))
    return out


def lognormal_threshold(rho, p_fa):
    """eta with P(rho' > eta) = p_fa under the lognormal fitted to rho' (ML)."""
    from scipy import stats
    lr = np.log(np.asarray(rho, dtype=np.float64))
    mu, sd = float(lr.mean()), float(lr.std())
    eta = math.exp(mu + sd * stats.norm.isf(p_fa))
    ks = stats.kstest(lr, "norm", args=(mu, sd))
    return eta, mu, sd, float(ks.pvalue)


ARRIVAL_S = 8.0     # paper sources: the frequency crosses f_* this long after the segment's start


def h1_injections(rng, snr, per_snr, source, n_samples, f_low, arrival_s):
    """Injection parameters of the H1 segments of one SNR: the paper's
    locations L4 and L5 (per_snr each; the frequency crossing f_* arrival_s
    after the segment's start) or per_snr random sources (coalescence in the
    middle half of the segment)."""
    import synth
    out = []
    for loc in (("L4", "L5") if source == "paper" else ("random",)):
        for _ in range(per_snr):
            if loc == "random":
                inj = synth.draw_injection(rng, n_samples)
                inj["tc_sample"] = int(rng.integers(n_samples // 4, 3 * n_samples // 4))
            else:
                inj = synth.paper_source(loc, rng, 0)
                inj["tc_sample"] = int(round((arrival_s + chirp_duration(inj["m1"], inj["m2"], f_low)) * FS))
            inj["tau0"], inj["tau15"] = chirp_times(inj["m1"], inj["m2"], f_low)
            inj["snr"] = snr
            inj["location"] = loc
            out.append(inj)
    return out


def h1_rows(snr, r1, r0, loc, eta):
    """Detection probability P(rho' >= eta) and L_DP = P(rho' <= eta | rho0 >=
    eta) of one SNR, overall and per location."""
    r1, r0, loc = np.asarray(r1), np.asarray(r0), np.asarray(loc)

    def stats(m):
        above0 = r0[m] >= eta
        return dict(segments=int(m.sum()), detection_probability=float(np.mean(r1[m] >= eta)),
                    l_dp=float(np.mean(r1[m][above0] <= eta)) if above0.any() else None,
                    truth_above_eta=int(above0.sum()), pso_below_truth=float(np.mean(r1[m] < r0[m])),
                    median_rho=float(np.median(r1[m])), median_rho0=float(np.median(r0[m])))
    row = dict(snr=snr, **stats(np.ones(len(r1), dtype=bool)))
    locs = sorted(set(loc.tolist()))
    if len(locs) > 1:
        row["by_location"] = {l: stats(loc == l) for l in locs}
    if len(locs) == 2:
        # Sec. V: two-sample Kolmogorov-Smirnov test of the two locations' rho'
        # samples, on all of them and on those above 9.0 only
        from scipy.stats import ks_2samp
        a, b = r1[loc == locs[0]], r1[loc == locs[1]]
        row["ks_pvalue_locations"] = float(ks_2samp(a, b).pvalue)
        a9, b9 = a[a > 9.0], b[b > 9.0]
        row["ks_pvalue_locations_above_9"] = float(ks_2samp(a9, b9).pvalue) if len(a9) and len(b9) else None
    return row


def run(slides=4, per_snr=64, snrs=(9.0, 10.0, 12.0, 15.0), iters=1000, runs=8, far_per_year=1.0, seed=6,
        n_per_slide=56, source="paper", keep_data=False, log=print):
    import synth
    dev = torch.device("cuda", 0)
    net = synth.network("HLVK")
    D = net.n_det
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    total = n_per_slide * SEG
    series = np.stack([synth.td_noise(np.random.default_rng(synth.seed_sequence(seed, 0, i)), total, FS)
                       for i in range(D)])
    h0 = h0_segments(series, n_per_slide, slides)
    psd_np = synth.psd_matrix(D, SEG, FS)
    rng = np.random.default_rng(synth.seed_sequence(seed, 1, 1000))
    h1 = []
    for snr in snrs:
        for inj in h1_injections(rng, snr, per_snr, source, SEG, F_LOW, ARRIVAL_S):
            xf = synth.noise_matrix(seed, 1 + len(h1), psd_np, SEG, FS)
            h1.append((xf, inj))
    n_seg = len(h0) + len(h1)
    ctx = Context.from_network(net, fs=FS, f_low=F_LOW, f_high=F_HIGH, box_lo=lo, box_hi=hi,
                               max_batch=n_seg * runs * 40, max_segments=n_seg, max_samples=SEG)
    psd = torch.from_numpy(psd_np).to(dev)
    for s, xf in enumerate(h0):
        ctx.set_segment(s, torch.from_numpy(xf).to(dev), psd)
    truth = []
    kept = [xf for xf in h0] if keep_data else None
    for k, (xf, inj) in enumerate(h1):
        x = torch.from_numpy(xf).to(dev)
        ctx.inject(x, psd, inj["alpha"], inj["delta"], inj["tau0"], inj["tau15"], inj["psi"], inj["phi_c"],
                   inj["cos_iota"], inj["tc_sample"] / FS, inj["snr"])
        ctx.set_segment(len(h0) + k, x, psd)
        truth.append([inj["alpha"], inj["delta"], inj["tau0"], inj["tau15"]])
        if keep_data:
            kept.append(x.cpu().numpy())
    torch.cuda.synchronize()
    log(f"{len(h0)} noise-only and {len(h1)} signal segments registered; searching")
    res = search_segments(ctx, n_seg, runs, 40, iters, seed=20020215 + seed, log=log)
    th0 = torch.tensor(truth, dtype=torch.float64, device=dev)
    seg1 = torch.arange(len(h0), n_seg, dtype=torch.int32, device=dev)
    rho0_sq = ctx.eval(th0, seg1)[0].cpu().numpy()
    rho0 = np.sqrt(np.maximum(rho0_sq, 0.0))
    rho = np.sqrt(np.maximum(res["rho_sq"].cpu().numpy(), 0.0))
    ctx.close()

    rho_h0, rho_h1 = rho[:len(h0)], rho[len(h0):]
    p_fa = far_per_year * SEG / FS / YEAR_S
    eta, mu, sd, ks_p = lognormal_threshold(rho_h0, p_fa)
    table = []
    loc = np.array([inj["location"] for _, inj in h1])
    snr_of = np.array([inj["snr"] for _, inj in h1])
    for snr in snrs:
        m = snr_of == snr
        table.append(h1_rows(snr, rho_h1[m], rho0[m], loc[m], eta))
        log(f"SNR {snr:g}: detection probability {table[-1]['detection_probability']:.3f}, "
            f"L_DP {table[-1]['l_dp']}, rho' < rho0 in {table[-1]['pso_below_truth']:.3f}")
    out = dict(segments_h0=len(h0), segments_h1=len(h1), slides=slides, source=source, seconds_search=res["seconds"],
               iterations=iters, runs=runs, far_per_year=far_per_year, p_false_alarm_per_segment=p_fa,
               h0_lognormal=dict(mu=mu, sigma=sd, ks_pvalue=ks_p),
               h0_rho_quantiles={q: float(np.quantile(rho_h0, q)) for q in (0.05, 0.5, 0.95, 1.0)},
               eta=eta, table=table)
    if keep_data:
        out["segment_data"] = dict(xf=kept, theta=res["theta"].cpu().numpy(), rho_sq=res["rho_sq"].cpu().numpy(),
                                   argmax=res["argmax"].cpu().numpy(), theta0=np.array(truth), rho0_sq=rho0_sq)
    return out


HOUR = 7372800


def hour_h0(first=1, last=24, iters=500, runs=12, group=8, seed=8, polish_steps=20, f_low=F_LOW, log=print):
    """H0 values rho' of the time-slid hour-long noise-only segments first..last
    (f_low = 10: the paper's band and rectangle, as hour_h1)."""
    import synth
    dev = torch.device("cuda", 0)
    net = synth.network("HLVK")
    D = net.n_det
    if f_low == PAPER_F_LOW:
        lo, hi = PAPER_BOX_LO, PAPER_BOX_HI
    else:
        lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    series = np.stack([synth.td_noise(np.random.default_rng(synth.seed_sequence(seed, 0, i)), HOUR, FS)
                       for i in range(D)])
    psd = torch.from_numpy(synth.psd_matrix(D, HOUR, FS)).to(dev)
    rho, seconds = {}, 0.0
    for g0 in range(first, last + 1, group):
        slides = list(range(g0, min(g0 + group, last + 1)))
        n = len(slides) * runs * 40
        ctx = Context.from_network(net, fs=FS, f_low=f_low, f_high=F_HIGH, box_lo=lo, box_hi=hi, max_batch=n,
                                   max_segments=len(slides), max_samples=HOUR,
                                   workspace_bytes=min(16 << 30, n * 2 * HOUR * 8))
        for k, s in enumerate(slides):
            xf = np.stack([synth.segment_fd(np.roll(series[i], -int(round(SLIDE_S * FS)) * s * i), 0, HOUR, FS)
                           for i in range(D)])
            ctx.set_segment(k, torch.from_numpy(xf).to(dev), psd)
        torch.cuda.synchronize()
        res = search_segments(ctx, len(slides), runs, 40, iters, seed=20020215 + seed + g0,
                              polish_steps=polish_steps, log=log)
        seconds += res["seconds"]
        for k, s in enumerate(slides):
            rho[s] = float(np.sqrt(max(res["rho_sq"][k].item(), 0.0)))
        ctx.close()
        log(f"slides {slides[0]}-{slides[-1]}: rho' " + " ".join(f"{rho[s]:.3f}" for s in slides))
    return dict(segment_samples=HOUR, slides=[first, last], iterations=iters, runs=runs, f_low=f_low,
                seconds_search=seconds, rho=rho)


# The paper's own search rectangle and band (Sec. II.B, Sec. V): f_* = 10 Hz,
# tau0 in [500, 1500] s, tau1.5 in [5, 15] s, the whole sky.
PAPER_F_LOW = 10.0
PAPER_BOX_LO = (0.0, -math.pi / 2, 500.0, 5.0)
PAPER_BOX_HI = (2.0 * math.pi, math.pi / 2, 1500.0, 15.0)
PAPER_ARRIVAL_S = 20.0 * 60.0   # the paper's signals arrive 20 min into the hour


def hour_h1(snr, first=0, last=7, iters=1500, runs=12, group=8, seed=9, polish_steps=20, source="random",
            f_low=F_LOW, keep_data=False, log=print):
    """rho' and rho0 of hour-long segments first..last: independent Gaussian
    noise (seeded per segment) with one SPA injection at network SNR `snr`.
    source="random": masses U[1, 3] Msun, isotropic sky and orientation,
    coalescence in the middle half of the hour.  source="L4" / "L5": the
    paper's location, psi = 30 deg, 1.5 + 1.5 Msun, the frequency crossing f_*
    20 min into the hour.  f_low = 10 takes the paper's band and rectangle
    (f_* = 10 Hz, tau0 in [500, 1500] s, tau1.5 in [5, 15] s); 30 the band and
    rectangle of the other workloads (masses in [1, 3] Msun at 30 Hz)."""
    import synth
    dev = torch.device("cuda", 0)
    net = synth.network("HLVK")
    D = net.n_det
    if f_low == PAPER_F_LOW:
        lo, hi = PAPER_BOX_LO, PAPER_BOX_HI
    else:
        lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    psd_np = synth.psd_matrix(D, HOUR, FS)
    psd = torch.from_numpy(psd_np).to(dev)
    out, seconds, kept = {}, 0.0, {}
    sidx = int(round(10 * snr)) + (100 if f_low == PAPER_F_LOW else 0) + {"random": 0, "L4": 1000, "L5": 2000}[source]
    for g0 in range(first, last + 1, group):
        idx = list(range(g0, min(g0 + group, last + 1)))
        n = len(idx) * runs * 40
        ctx = Context.from_network(net, fs=FS, f_low=f_low, f_high=F_HIGH, box_lo=lo, box_hi=hi, max_batch=n,
                                   max_segments=len(idx), max_samples=HOUR,
                                   workspace_bytes=min(16 << 30, n * 2 * HOUR * 8))
        truth = []
        for k, r in enumerate(idx):
            rng = np.random.default_rng(synth.seed_sequence(seed, sidx, 5000 + r))
            if source == "random":
                inj = synth.draw_injection(rng, HOUR)
                inj["tc_sample"] = int(rng.integers(HOUR // 4, 3 * HOUR // 4))
            else:
                inj = synth.paper_source(source, rng, 0)
                inj["tc_sample"] = int(round((PAPER_ARRIVAL_S + chirp_duration(inj["m1"], inj["m2"], f_low)) * FS))
            t0, t15 = chirp_times(inj["m1"], inj["m2"], f_low)
            x = torch.from_numpy(synth.noise_matrix(seed, 1000 * sidx + r, psd_np, HOUR, FS)).to(dev)
            ctx.inject(x, psd, inj["alpha"], inj["delta"], t0, t15, inj["psi"], inj["phi_c"], inj["cos_iota"],
                       inj["tc_sample"] / FS, snr)
            ctx.set_segment(k, x, psd)
            truth.append([inj["alpha"], inj["delta"], t0, t15])
            if keep_data:
                kept[r] = x.cpu().numpy()
        torch.cuda.synchronize()
        res = search_segments(ctx, len(idx), runs, 40, iters, seed=20020215 + seed + 7 * g0,
                              polish_steps=polish_steps, log=log)
        seconds += res["seconds"]
        th0 = torch.tensor(truth, dtype=torch.float64, device=dev)
        f0 = ctx.eval(th0, torch.arange(len(idx), dtype=torch.int32, device=dev))[0].cpu().numpy()
        for k, r in enumerate(idx):
            out[r] = dict(rho=float(np.sqrt(max(res["rho_sq"][k].item(), 0.0))), rho0=float(np.sqrt(max(f0[k], 0.0))),
                          location=source)
            if keep_data:
                out[r].update(theta=res["theta"][k].cpu().numpy(), rho_sq=float(res["rho_sq"][k].item()),
                              argmax=int(res["argmax"][k].item()), theta0=truth[k], rho0_sq=float(f0[k]),
                              xf=kept[r])
        ctx.close()
        log(f"SNR {snr:g} segments {idx[0]}-{idx[-1]}: " + " ".join(f"{out[r]['rho']:.2f}/{out[r]['rho0']:.2f}" for r in idx))
    return dict(segment_samples=HOUR, snr=snr, segments=[first, last], iterations=iters, runs=runs, source=source,
                f_low=f_low, seconds_search=seconds, values=out)


def h1_table(eta, outs):
    """Detection probability P(rho' >= eta) and L_DP = P(rho' <= eta | rho0 >= eta) per SNR."""
    by = {}
    for o in outs:
        loc = o.get("source", "random")
        d = by.setdefault(o["snr"], {})
        vals = {(loc, int(k)): v for k, v in o["values"].items()}
        dup = sorted(set(d) & set(vals))
        if dup:
            raise ValueError(f"SNR {o['snr']:g}: segments {dup} appear in more than one output")
        d.update(vals)
    table = []
    for snr in sorted(by):
        keys = sorted(by[snr])
        r1 = np.array([by[snr][k]["rho"] for k in keys])
        r0 = np.array([by[snr][k]["rho0"] for k in keys])
        loc = np.array([k[0] for k in keys])
        table.append(h1_rows(snr, r1, r0, loc, eta))
    return dict(eta=eta, table=table)


def combine(outs, far_per_year=1.0):
    """Lognormal fit of the H0 values of several hour_h0 runs and the threshold."""
    rho = {}
    bands = {o.get("f_low", F_LOW) for o in outs}
    if len(bands) > 1:
        raise ValueError(f"H0 runs of different bands (f_low {sorted(bands)}) cannot share a threshold")
    for o in outs:
        dup = sorted(set(rho) & {int(k) for k in o["rho"]})
        if dup:
            raise ValueError(f"slides {dup} appear in more than one output")
        rho.update({int(k): v for k, v in o["rho"].items()})
    vals = np.array([rho[k] for k in sorted(rho)])
    p_fa = far_per_year * HOUR / FS / YEAR_S
    eta, mu, sd, ks_p = lognormal_threshold(vals, p_fa)
    return dict(segments_h0=len(vals), p_false_alarm_per_segment=p_fa, eta=eta,
                h0_lognormal=dict(mu=mu, sigma=sd, ks_pvalue=ks_p),
                h0_rho_quantiles={q: float(np.quantile(vals, q)) for q in (0.05, 0.5, 0.95, 1.0)},
                iterations=sorted({o["iterations"] for o in outs}), runs=sorted({o["runs"] for o in outs}),
                f_low=bands.pop())


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--slides", default="4", help="time slides (an int), or a-b with --hour")
    ap.add_argument("--per-snr", type=int, default=64)
    ap.add_argument("--iters", type=int, default=None, help="PSO iterations (1000; 500 with --hour)")
    ap.add_argument("--snrs", default="9,10,12,15")
    ap.add_argument("--hour", action="store_true", help="H0 of time-slid hour-long segments (slides a-b)")
    ap.add_argument("--runs", type=int, default=None)
    ap.add_argument("--combine", nargs="+", default=None, help="JSON outputs of --hour runs to fit together")
    ap.add_argument("--hour-h1", action="store_true", help="hour-long segments with an injection at --snr")
    ap.add_argument("--snr", type=float, default=10.0)
    ap.add_argument("--segments", default="0-7", help="--hour-h1: segment indices a-b")
    ap.add_argument("--h1-table", nargs="+", default=None, help="ETA, then JSON outputs of --hour-h1 runs")
    ap.add_argument("--source", default=None,
                    help="H1 sources: paper (L4 and L5; default) or random for the 64-s study; random, L4 or L5 "
                         "with --hour-h1")
    ap.add_argument("--f-low", type=float, default=F_LOW,
                    help="--hour and --hour-h1: 10 takes the paper's band and rectangle (f_* = 10 Hz, tau0 in [500, 1500] s, "
                         "tau1.5 in [5, 15] s)")
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    if a.h1_table:
        outs = []
        for path in a.h1_table[1:]:
            with open(path) as fh:
                outs.append(json.loads([l for l in fh if l.startswith("{")][-1]))
        print(json.dumps(h1_table(float(a.h1_table[0]), outs)))
        return 0
    if a.hour_h1:
        first, last = (int(x) for x in a.segments.split("-"))
        out = hour_h1(a.snr, first, last, iters=a.iters or 1500, runs=a.runs or 12, source=a.source or "random",
                      f_low=a.f_low, log=log)
        print(json.dumps(out))
        return 0
    if a.combine:
        outs = []
        for path in a.combine:
            with open(path) as fh:
                outs.append(json.loads([l for l in fh if l.startswith("{")][-1]))
        print(json.dumps(combine(outs)))
        return 0
    if a.hour:
        first, last = (int(x) for x in str(a.slides).split("-"))
        out = hour_h0(first, last, iters=a.iters or 500, runs=a.runs or 12, f_low=a.f_low, log=log)
        print(json.dumps(out))
        return 0
    out = run(int(a.slides), a.per_snr, tuple(float(x) for x in a.snrs.split(",")), a.iters or 1000,
              runs=a.runs or 8, source=a.source or "paper", log=log)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
