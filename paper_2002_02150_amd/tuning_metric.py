"""PSO tuning metric (Sec. III, eq. tuning_metric) on synthetic injections:

    M(N_runs, N_iter) = Pr( rho'_coh(N_runs, N_iter) < rho_coh^(0) ),

with rho'_coh^2 the best-of-N_runs PSO result and rho_coh^(0)^2 the fitness at
the true parameters, estimated as the fraction of realizations where the search
ends below the truth.  Each N_iter gets its own search (the inertia schedule
depends on it); the N_runs values are the first N_runs of 12 independent runs.

    python -m paper_2002_02150_amd.tuning_metric [--realizations 32] [--snr 10]

Workload: 4 detectors (H, L, V, K), 64 s at 2048 Hz, analytic PSD, Gaussian
noise and one SPA injection per realization (masses U[1,3] Msun, isotropic
sky), 40 particles per run, one captured HIP graph per PSO iteration.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import Context, PsoConfig, Swarm
from .params import chirp_times

N_SAMPLES, FS, F_LOW, F_HIGH = 131072, 2048.0, 30.0, 1000.0
PARTICLES, MAX_RUNS = 40, 12


def search(ctx, seg, cfg: PsoConfig):
    """One best-of-runs search; returns the per-run best fitness (device tensor)."""
    sw = Swarm(ctx, cfg)
    n = sw.n
    f = torch.empty(n, dtype=torch.float64, device=ctx.device)
    j = torch.empty(n, dtype=torch.int32, device=ctx.device)
    sw.init()

    def iteration():
        ctx.eval(sw.theta, seg, f, j)
        sw.step(f, j)

    st = torch.cuda.Stream(ctx.device)
    st.wait_stream(torch.cuda.current_stream(ctx.device))
    with torch.cuda.stream(st):
        iteration()
    torch.cuda.current_stream(ctx.device).wait_stream(st)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        iteration()
    for _ in range(cfg.n_iter - 2):
        g.replay()
    ctx.eval(sw.theta, seg, f, j)   # fitness of the final positions enters the personal bests
    sw.step(f, j)
    return sw.best_f.clone()


def run(realizations=32, snr=10.0, n_iters=(250, 500, 1000), n_runs_list=(2, 4, 8, 12), seed=2002, log=print):
    import synth
    dev = torch.device("cuda", 0)
    net = synth.network("HLVK")
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    ctx = Context.from_network(net, fs=FS, f_low=F_LOW, f_high=F_HIGH, box_lo=lo, box_hi=hi,
                               max_batch=MAX_RUNS * PARTICLES, max_samples=N_SAMPLES)
    psd = torch.from_numpy(synth.psd_matrix(4, N_SAMPLES, FS)).to(dev)
    seg = torch.zeros(MAX_RUNS * PARTICLES, dtype=torch.int32, device=dev)
    below = {(m, it): 0 for m in n_runs_list for it in n_iters}
    records = []
    t_start = time.perf_counter()
    for r in range(realizations):
        xf = torch.from_numpy(synth.noise_matrix(5, r, psd.cpu().numpy(), N_SAMPLES, FS)).to(dev)
        inj = synth.draw_injection(np.random.default_rng(synth.seed_sequence(5, r, 1000)), N_SAMPLES)
        t0, t15 = chirp_times(inj["m1"], inj["m2"], F_LOW)
        ctx.inject(xf, psd, inj["alpha"], inj["delta"], t0, t15, inj["psi"], inj["phi_c"], inj["cos_iota"],
                   inj["tc_sample"] / FS, snr)
        ctx.set_segment(0, xf, psd)
        theta0 = torch.tensor([[inj["alpha"], inj["delta"], t0, t15]], dtype=torch.float64, device=dev)
        rho0_sq = ctx.eval(theta0, seg[:1])[0].item()
        rec = dict(realization=r, rho0_sq=rho0_sq, best={})
        for it in n_iters:
            best_f = search(ctx, seg, PsoConfig(n_runs=MAX_RUNS, n_particles=PARTICLES, n_iter=it,
                                                seed=seed * 1000003 + r * 101 + it)).cpu().numpy()
            for m in n_runs_list:
                rho_sq = float(np.max(best_f[:m]))
                rec["best"][f"{m}x{it}"] = rho_sq
                below[(m, it)] += rho_sq < rho0_sq
        records.append(rec)
        log(f"realization {r}: rho0^2 = {rho0_sq:.2f}, best of 12 x {n_iters[-1]} = {rec['best'][f'12x{n_iters[-1]}']:.2f}")
    elapsed = time.perf_counter() - t_start
    table = {f"{m}x{it}": below[(m, it)] / realizations for m in n_runs_list for it in n_iters}
    ctx.close()
    return dict(metric="M(N_runs, N_iter) = Pr(rho' < rho0)", snr=snr, realizations=realizations,
                n_iters=list(n_iters), n_runs=list(n_runs_list), table=table, seconds=elapsed, records=records)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--realizations", type=int, default=32)
    ap.add_argument("--snr", type=float, default=10.0)
    ap.add_argument("--iters", default="250,500,1000")
    a = ap.parse_args(argv)
    out = run(a.realizations, a.snr, tuple(int(x) for x in a.iters.split(",")),
              log=lambda s: print(s, flush=True))
    print(json.dumps({k: v for k, v in out.items() if k != "records"}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
