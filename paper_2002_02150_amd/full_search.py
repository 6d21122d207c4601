"""Full-length search of an hour of 4-detector data, timed against the data
duration (Sec. IV: the search's runtime over the duration of the data it
covers).

    python -m paper_2002_02150_amd.full_search [--minutes 60] [--segments 56] [--iters 2000]
    python -m paper_2002_02150_amd.full_search --single-segment [--minutes 60] [--iters 1000]

Data: a seeded Gaussian time series per detector (H, L, V, K) at 2048 Hz with
the analytic PSD above 20 Hz, cut into overlapping 128-s segments (262144
samples) at a common stride, the last one ending with the data; 8
double-neutron-star injections (component masses U[1.2, 1.6] Msun, isotropic
sky and orientation, network SNR U[10, 12], coalescence uniform over the hour
from 128 s on, so that every chirp starts inside the data).  Each injection is synthesised once over the whole stretch
(fcas_inject on the Fourier grid of the full length, network SNR over the
stretch), brought to the time domain and added to the noise series before the
segments are cut, so that every segment overlapping a chirp holds the part of
it its window sees.

Search: every segment gets 8 independent PSO runs of 40 particles and 2000
iterations; all segments' runs are one batch of 17,920 points per iteration,
launched as captured HIP graphs of 20 iterations.  Each segment's coalescence
time is searched only over the central stride of its window (the first and
last segments also over the outer ends), so the central parts tile the hour.
After the iterations the best point of each segment is polished by gradient
ascent (fitness_polish, 20 steps of 16 backtracking trials from 1e-3 of the
rectangle down to 3e-8).  T_run is the device time of the iterations and the
polish; the data preparation (host FFTs, segment registration) is reported
beside it.

--single-segment is the paper's own layout (Sec. IV): the whole stretch is one
segment (7,372,800 samples per detector for an hour at 2048 Hz, searched with
the three-pass FFT plan), with one double-neutron-star injection anywhere in
it and 8 PSO runs of 40 particles as one batch; the coalescence time is
searched over the whole hour.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import Context
from .campaign import search_segments
from .params import chirp_times

FS, F_LOW, F_HIGH = 2048.0, 30.0, 1000.0
SEG = 262144                          # 128 s
RUNS, PARTICLES = 8, 40


def layout(total: int, n_seg: int, seg: int = SEG):
    """Segment starts and the searched coalescence range of each.  The segments
    follow a common stride, except the last, which starts where it ends with
    the data (up to n_seg - 2 samples later than the stride puts it); every
    range continues where the previous one ends, so the ranges tile
    [0, total) with no gap or overlap."""
    if n_seg < 2 or total < seg:
        raise ValueError(f"need at least two segments of {seg} samples, got {n_seg} over {total}")
    stride = (total - seg) // (n_seg - 1)
    if stride > seg:
        raise ValueError(f"{n_seg} segments of {seg} samples leave gaps in {total} samples")
    starts = [k * stride for k in range(n_seg - 1)] + [total - seg]
    margin = (seg - stride) // 2
    ranges = []
    end = 0                              # where the previous range ends (absolute sample)
    for k in range(n_seg):
        lo = end - starts[k]
        hi = seg if k == n_seg - 1 else margin + stride
        ranges.append((lo, hi))
        end = starts[k] + hi
    return starts, stride, ranges


def add_injections(ctx, series, injections, dev):
    """Adds each injection to the time series (D x total, in place): its SPA
    response on the Fourier grid of the whole stretch (fcas_inject, scaled to
    its network SNR over the stretch), brought to the time domain (continuum
    units: x = fs * irfft)."""
    import synth
    D, total = series.shape
    psd_full = torch.from_numpy(synth.psd_matrix(D, total, FS)).to(dev)
    for inj in injections:
        hf = torch.zeros(D, total // 2 + 1, dtype=torch.complex128, device=dev)
        ctx.inject(hf, psd_full, inj["alpha"], inj["delta"], inj["tau0"], inj["tau15"], inj["psi"], inj["phi_c"],
                   inj["cos_iota"], inj["tc_sample"] / FS, inj["snr"])
        series += FS * np.fft.irfft(hf.cpu().numpy(), n=total, axis=1)
        del hf


def run(minutes=60.0, n_seg=56, iters=2000, n_inj=8, seed=5, polish_steps=20, keep_data=False, log=print):
    """The search of the stretch; keep_data also returns every segment's
    Fourier data (host copies; the PSD is synth.psd_matrix) and results."""
    import synth
    dev = torch.device("cuda", 0)
    total = int(round(minutes * 60.0 * FS))
    starts, stride, ranges = layout(total, n_seg)
    net = synth.network("HLVK")
    D = net.n_det
    lo_box, hi_box = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI

    n = n_seg * RUNS * PARTICLES
    ctx = Context.from_network(net, fs=FS, f_low=F_LOW, f_high=F_HIGH, box_lo=lo_box, box_hi=hi_box, max_batch=n,
                               max_segments=n_seg, max_samples=SEG)
    t0 = time.perf_counter()
    series = np.stack([synth.td_noise(np.random.default_rng(synth.seed_sequence(seed, 0, i)), total, FS)
                       for i in range(D)])
    rng = np.random.default_rng(synth.seed_sequence(seed, 0, 1000))
    injections = []
    for _ in range(n_inj):
        inj = synth.draw_injection(rng, total, m_lo=1.2, m_hi=1.6)
        inj["tc_sample"] = int(rng.integers(SEG, total - SEG // 4))
        inj["snr"] = float(rng.uniform(10.0, 12.0))
        inj["tau0"], inj["tau15"] = chirp_times(inj["m1"], inj["m2"], F_LOW)
        injections.append(inj)
    add_injections(ctx, series, injections, dev)
    t_series = time.perf_counter() - t0

    psd = torch.from_numpy(synth.psd_matrix(D, SEG, FS)).to(dev)
    t1 = time.perf_counter()
    kept = []
    for s, a in enumerate(starts):
        xf_np = np.stack([synth.segment_fd(series[i], a, SEG, FS) for i in range(D)])
        if keep_data:
            kept.append(xf_np)
        ctx.set_segment(s, torch.from_numpy(xf_np).to(dev), psd)
        ctx.set_segment_range(s, *ranges[s])
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t1

    res = search_segments(ctx, n_seg, RUNS, PARTICLES, iters, seed=20020215 + seed, polish_steps=polish_steps,
                          log=log)
    t_run = res["seconds"]
    f_pso, f_pol, j_pol, theta = res["rho_sq_pso"], res["rho_sq"], res["argmax"], res["theta"]
    evaluated = ctx.evaluated()

    f_pso, f_pol, j_pol, theta = f_pso.cpu().numpy(), f_pol.cpu().numpy(), j_pol.cpu().numpy(), theta.cpu().numpy()
    found = []
    for inj in injections:
        # the segment whose searched range holds the coalescence
        s = next(s for s in range(n_seg) if starts[s] + ranges[s][0] <= inj["tc_sample"] < starts[s] + ranges[s][1])
        th0 = torch.tensor([[inj["alpha"], inj["delta"], inj["tau0"], inj["tau15"]]], dtype=torch.float64,
                           device=dev)
        rho0_sq = ctx.eval(th0, torch.tensor([s], dtype=torch.int32, device=dev))[0].item()
        found.append(dict(segment=s, snr=inj["snr"], m1=inj["m1"], m2=inj["m2"], rho0_sq=rho0_sq,
                          tc_sample=inj["tc_sample"],
                          theta0=[inj["alpha"], inj["delta"], inj["tau0"], inj["tau15"]],
                          rho_sq_pso=float(f_pso[s]), rho_sq=float(f_pol[s]),
                          dt_c_samples=int(starts[s] + j_pol[s] - inj["tc_sample"]),
                          d_tau0=float(theta[s, 2] - inj["tau0"]), d_tau15=float(theta[s, 3] - inj["tau15"])))
        log(f"injection in segment {s}: SNR {inj['snr']:.2f} (rho0^2 {rho0_sq:.1f}), found rho^2 {f_pol[s]:.1f} "
            f"(PSO {f_pso[s]:.1f}), t_c off by {found[-1]['dt_c_samples']} samples")
    improved = int(np.sum(f_pol > f_pso))
    with_inj = {d["segment"] for d in found}
    noise_only = [float(f_pol[s]) for s in range(n_seg) if s not in with_inj]
    ctx.close()
    T = total / FS
    out = dict(data_seconds=T, segments=n_seg, stride_samples=stride, iterations=iters,
               points_per_iteration=n, evaluated_points=evaluated, t_run_s=t_run, t_run_over_t=t_run / T,
               evaluated_points_per_s=evaluated / t_run,
               data_generation_s=t_series, segment_preparation_s=t_prep, polish_improved_segments=improved,
               injections=found, noise_only_max_rho_sq=dict(
                   median=float(np.median(noise_only)) if noise_only else None,
                   max=float(np.max(noise_only)) if noise_only else None))
    if keep_data:
        out["segment_data"] = dict(xf=kept, starts=starts, ranges=ranges, theta=theta, rho_sq=f_pol,
                                   rho_sq_pso=f_pso, argmax=j_pol)
    return out


def run_single_segment(minutes=60.0, iters=1000, runs=RUNS, seed=7, snr=(10.0, 12.0), polish_steps=20, log=print):
    """One segment over the whole stretch, one injection, `runs` PSO runs of 40
    particles; T_run covers the iterations and the polish."""
    import synth
    from . import fcas
    dev = torch.device("cuda", 0)
    total = int(round(minutes * 60.0 * FS))
    if not fcas.supported_n(total):
        raise ValueError(f"{minutes} min at {FS:g} Hz = {total} samples has no FFT plan")
    net = synth.network("HLVK")
    D = net.n_det
    lo_box, hi_box = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    t0 = time.perf_counter()
    series = np.stack([synth.td_noise(np.random.default_rng(synth.seed_sequence(seed, 0, i)), total, FS)
                       for i in range(D)])
    rng = np.random.default_rng(synth.seed_sequence(seed, 0, 1000))
    inj = synth.draw_injection(rng, total, m_lo=1.2, m_hi=1.6)
    inj["tc_sample"] = int(rng.integers(0, total))
    inj["snr"] = float(rng.uniform(*snr))
    inj["tau0"], inj["tau15"] = chirp_times(inj["m1"], inj["m2"], F_LOW)
    t_series = time.perf_counter() - t0
    # a 4 GiB workspace (36 points of an hour per launch) measured fastest: the
    # later passes then find more of their input in the caches
    ctx = Context.from_network(net, fs=FS, f_low=F_LOW, f_high=F_HIGH, box_lo=lo_box, box_hi=hi_box,
                               max_batch=runs * PARTICLES, max_segments=1, max_samples=total,
                               workspace_bytes=min(4 << 30, runs * PARTICLES * 2 * total * 8))
    psd = torch.from_numpy(synth.psd_matrix(D, total, FS)).to(dev)
    t1 = time.perf_counter()
    xf = torch.from_numpy(np.stack([synth.segment_fd(series[i], 0, total, FS) for i in range(D)])).to(dev)
    del series
    ctx.inject(xf, psd, inj["alpha"], inj["delta"], inj["tau0"], inj["tau15"], inj["psi"], inj["phi_c"],
               inj["cos_iota"], inj["tc_sample"] / FS, inj["snr"])
    ctx.set_segment(0, xf, psd)
    del xf
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t1
    res = search_segments(ctx, 1, runs, PARTICLES, iters, seed=20020215 + seed, polish_steps=polish_steps, log=log)
    t_run = res["seconds"]
    th0 = torch.tensor([[inj["alpha"], inj["delta"], inj["tau0"], inj["tau15"]]], dtype=torch.float64, device=dev)
    rho0_sq = ctx.eval(th0, torch.zeros(1, dtype=torch.int32, device=dev))[0].item()
    evaluated = ctx.evaluated()
    theta = res["theta"][0].cpu().numpy()
    found = dict(snr=inj["snr"], m1=inj["m1"], m2=inj["m2"], rho0_sq=rho0_sq,
                 rho_sq_pso=float(res["rho_sq_pso"][0]), rho_sq=float(res["rho_sq"][0]),
                 dt_c_samples=int(res["argmax"][0].item() - inj["tc_sample"]),
                 d_tau0=float(theta[2] - inj["tau0"]), d_tau15=float(theta[3] - inj["tau15"]))
    log(f"injection SNR {inj['snr']:.2f} (rho0^2 {rho0_sq:.1f}): found rho^2 {found['rho_sq']:.1f} "
        f"(PSO {found['rho_sq_pso']:.1f}), t_c off by {found['dt_c_samples']} samples")
    ctx.close()
    T = total / FS
    return dict(data_seconds=T, samples=total, runs=runs, particles=PARTICLES, iterations=iters,
                points_per_iteration=runs * PARTICLES, evaluated_points=evaluated, t_run_s=t_run,
                t_run_over_t=t_run / T, evaluated_points_per_s=evaluated / t_run, data_generation_s=t_series,
                segment_preparation_s=t_prep, injection=found)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--minutes", type=float, default=60.0)
    ap.add_argument("--segments", type=int, default=56)
    ap.add_argument("--iters", type=int, default=None, help="PSO iterations (2000; 1000 with --single-segment)")
    ap.add_argument("--injections", type=int, default=8)
    ap.add_argument("--single-segment", action="store_true", help="the whole stretch as one segment")
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    if a.single_segment:
        out = run_single_segment(a.minutes, a.iters if a.iters is not None else 1000, log=log)
    else:
        out = run(a.minutes, a.segments, a.iters if a.iters is not None else 2000, a.injections, log=log)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
