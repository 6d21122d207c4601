"""Throughput of the coherent-fitness hot path on one MI355X.

One step is one iteration of the PSO search of the 4-detector, 64 s, 2048 Hz
configuration (131072 samples per detector, SNR-10 injection): the fitness of
8 runs x 40 particles (320 evaluations), the swarm update, the best of the
runs, and the gradient at the best point.  value = fitness evaluations per
second over the timed steps (inputs resident in HBM).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_SAMPLES, FS, F_LOW, F_HIGH = 131072, 2048.0, 30.0, 1000.0
RUNS, PARTICLES = 8, 40
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("fft_core.hpp", "fitness_tiles.hpp", "plans.hpp", "eval_kernels.hpp", "eval_f32.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=320)
    return ap.parse_args()


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2002_02150_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def make_workload(torch, dev):
    import synth
    from paper_2002_02150_amd import Context
    from paper_2002_02150_amd.params import chirp_times
    net = synth.network("HLVK")
    psd = synth.psd_matrix(4, N_SAMPLES, FS)
    noise = synth.noise_matrix(2, 0, psd, N_SAMPLES, FS)
    inj = synth.draw_injection(np.random.default_rng(synth.seed_sequence(2, 0, 1000)), N_SAMPLES)
    t0, t15 = chirp_times(inj["m1"], inj["m2"], F_LOW)
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    ctx = Context.from_network(net, fs=FS, f_low=F_LOW, f_high=F_HIGH, box_lo=lo, box_hi=hi,
                               max_batch=RUNS * PARTICLES, max_samples=N_SAMPLES)
    xf = torch.from_numpy(noise).to(dev)
    psd_d = torch.from_numpy(np.ascontiguousarray(psd)).to(dev)
    ctx.inject(xf, psd_d, inj["alpha"], inj["delta"], t0, t15, inj["psi"], inj["phi_c"], inj["cos_iota"],
               inj["tc_sample"] / FS, 10.0)
    ctx.set_segment(0, xf, psd_d)
    return ctx, net, xf, psd_d, (inj, t0, t15)


def run_steps(torch, ctx, sw, seg, seg1, steps, it0):
    th = sw.theta
    for s in range(steps):
        f, j = ctx.eval(th, seg, *bufs(ctx, torch))
        th = sw.step(f, j, it0 + s)
        bf, bt, bj, br = sw.best()
        ctx.grad(bt.view(1, 4), seg1)
    return th


_BUFS = {}


def bufs(ctx, torch):
    key = id(ctx)
    if key not in _BUFS:
        n = RUNS * PARTICLES
        _BUFS[key] = (torch.empty(n, dtype=torch.float64, device=ctx.device),
                      torch.empty(n, dtype=torch.int32, device=ctx.device))
    return _BUFS[key]


def fp64_plain_rate(torch, net, xf, psd_d, thetas, dev):
    """Per-particle FP64 path: the same kernels in double precision, one
    evaluation per call, no batching."""
    import synth
    from paper_2002_02150_amd import FP64, Context
    ctx = Context.from_network(net, fs=FS, f_low=F_LOW, f_high=F_HIGH, box_lo=synth.SEARCH_BOX_30HZ_LO,
                               box_hi=synth.SEARCH_BOX_30HZ_HI, precision=FP64, max_batch=1, max_samples=N_SAMPLES)
    ctx.set_segment(0, xf, psd_d)
    seg = torch.zeros(1, dtype=torch.int32, device=dev)
    rows = [thetas[i:i + 1].contiguous() for i in range(thetas.shape[0])]
    for r in rows[:4]:
        ctx.eval(r, seg)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for r in rows:
        ctx.eval(r, seg)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ctx.close()
    return len(rows) / dt


def _oracle_worker(args):
    from oracle import fitness as F
    seg, pos, ten, th = args
    return [F.fitness(seg, pos, ten, t)[0] for t in th]


def cpu_baseline(xf_np, psd, net, thetas, sample):
    """The FP64 oracle on the host cores, on the first `sample` points."""
    import multiprocessing as mp
    from oracle import fitness as F
    seg = F.prepare_segment(xf_np, psd, FS, F_LOW, F_HIGH)
    th = thetas[:sample]
    cores = max(1, min(os.cpu_count() or 1, 64))
    chunks = [th[i::cores] for i in range(cores)]
    ctx = mp.get_context("fork")
    t = time.perf_counter()
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_worker, [(seg, net.pos_m, net.tensor, c) for c in chunks if len(c)])
    dt = time.perf_counter() - t
    return dict(value=len(th) / dt, unit="evals/s", cores=cores, kind="oracle",
                sample=f"{len(th)} fitness evaluations of the first PSO batch (4 det x 131072 samples), "
                       f"multiprocessing pool over {cores} host cores, {dt:.1f} s wall")


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    from paper_2002_02150_amd import PsoConfig, Swarm
    dev = torch.device("cuda", 0)
    ctx, net, xf, psd_d, inj = make_workload(torch, dev)
    sw = Swarm(ctx, PsoConfig(n_runs=RUNS, n_particles=PARTICLES, n_iter=2000, seed=20020215))
    seg = torch.zeros(RUNS * PARTICLES, dtype=torch.int32, device=dev)
    seg1 = torch.zeros(1, dtype=torch.int32, device=dev)
    first_batch = sw.init().clone()
    run_steps(torch, ctx, sw, seg, seg1, a.warmup, 0)
    torch.cuda.synchronize()
    # timed region: K steps, kernel durations recorded with HIP events on the same stream
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    run_steps(torch, ctx, sw, seg, seg1, a.steps, a.warmup)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ctx.set_timing(False)
    ms1, n1 = ctx.read_timing("pass1")
    ms2, n2 = ctx.read_timing("pass2")
    evals = a.steps * RUNS * PARTICLES
    value = evals / dt
    # dominant kernel and its algorithmic bytes per launch (320 evaluations of one segment)
    K = 64000 - 1921 + 1
    D = 4
    per_eval_p1 = 16 * N_SAMPLES
    per_launch_p1 = RUNS * PARTICLES * per_eval_p1 + 8 * K * D + 8 * K
    per_launch_p2 = RUNS * PARTICLES * 16 * N_SAMPLES
    if ms1 >= ms2:
        name, avg_ms, alg = "k_pass1", ms1 / max(n1, 1), per_launch_p1
    else:
        name, avg_ms, alg = "k_pass2", ms2 / max(n2, 1), per_launch_p2
    achieved = alg / (avg_ms * 1e-3) / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        tr = json.load(open(tf))
        if tr.get("kernel_hash") == kernel_hash() and name in tr.get("kernels", {}):
            traffic = tr["kernels"][name]["bytes_per_launch"]
    out = {
        "metric": "coherent-fitness evals/s, 4 det x 131072 samples; mixed vs FP64 plain; % HBM BW",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64phase", "data": "synthetic",
        "config": {"workload": "4 detectors (HLVK), 64 s at 2048 Hz (131072 samples), SNR-10 SPA injection, "
                               "PSO 8 runs x 40 particles: fitness batch + swarm update + best-of-runs + gradient",
                   "global_batch": RUNS * PARTICLES, "seq_len": N_SAMPLES, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_ms": avg_ms, "alg_bytes_per_launch": alg},
        "kernel_ms_per_step": {"k_pass1": ms1 / a.steps, "k_pass2": ms2 / a.steps},
    }
    if not a.no_fp64:
        rate64 = fp64_plain_rate(torch, net, xf, psd_d, first_batch[:64].contiguous(), dev)
        out["fp64_plain"] = {"value": rate64, "unit": "evals/s", "speedup": value / rate64,
                             "what": "same kernels in FP64, one evaluation per call, no graph"}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(xf.cpu().numpy(), psd_d.cpu().numpy(), net,
                                           first_batch.cpu().numpy(), a.cpu_sample)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
