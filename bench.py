"""Throughput of the coherent-fitness hot path on one MI355X.

One step is one iteration of the PSO search of the 4-detector, 64 s, 2048 Hz
configuration (131072 samples per detector, SNR-10 injection): the fitness of
8 runs x 40 particles (320 evaluations) and the swarm update, captured as HIP
graphs of 20 iterations and replayed; by default the timed region is one whole
search (2000 iterations).  value = fitness evaluations of the particles per
second over the timed region (inputs resident in HBM; particles that left the
search rectangle are not evaluated and not counted).  The best of the runs and
the gradient polish of that point, done once per search, are timed on their
own after the iterations (polish_ms).  A second
timed region launches the same steps eagerly with HIP events recorded by the
FFT pass kernels' dispatch, for the roofline figures.  The FP64 oracle evaluates the first
PSO batch on the host cores (cpu_baseline), and the library's results on the
same points are compared with it (parity: relative error of the fitness,
argmax agreement).

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Other workloads (--config): hour (the paper's own segment length: one hour at
2048 Hz, 7,372,800 samples per detector, three-pass FFT plan, the same PSO
step and polish, per-pass rooflines), batched (256 ragged segments), gradient
(4096 fitness gradients), sweep (batch sizes 320-20480).
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
KERNEL_SOURCES = ("fft_core.hpp", "fitness_tiles.hpp", "plans.hpp", "eval_kernels.hpp", "eval_f32.hip", "fcas_api.cpp")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: search 2000 = one whole search, batched 20, gradient 50)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1280,
                    help="points the oracle evaluates for cpu_baseline (the first 320 also for parity)")
    ap.add_argument("--schedule", choices=("fused", "two-pass"), default="two-pass")
    ap.add_argument("--tail", choices=("fused", "separate"), default="fused",
                    help="end of a PSO iteration in captured steps: one kernel (pso_run) or the separate finalize, "
                         "swarm-update and set-up kernels (fitness_eval_batch + pso_step)")
    ap.add_argument("--config", choices=("search", "batched", "gradient", "sweep", "hour"), default="search",
                    help="search: the benchmark configuration (default); batched: 256 ragged segments, "
                         "40 particles x 4 runs each; gradient: 4096 fitness gradients near a true source; "
                         "sweep: fitness batches of 320 to 20480 points; hour: the PSO search of one hour-long "
                         "segment (7,372,800 samples per detector, three-pass FFT)")
    ap.add_argument("--hour-workspace-gib", type=float, default=4.0,
                    help="hour: FFT workspace in GiB (0: the library default, 8 GiB = 72 points); 4 GiB = 36 "
                         "points, nine launches per pass for 320 points, measured fastest of 0.22-37.7 GB")
    ap.add_argument("--launch-counts", action="store_true",
                    help="record the points evaluated by each eager launch (adds a sync per step)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, one device-to-device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2002_02150_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


SCHEDULES = {"fused": 0, "two-pass": 1}


def make_workload(torch, dev, schedule, max_batch=RUNS * PARTICLES):
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
                               max_batch=max_batch, max_samples=N_SAMPLES, schedule=SCHEDULES[schedule])
    xf = torch.from_numpy(noise).to(dev)
    psd_d = torch.from_numpy(np.ascontiguousarray(psd)).to(dev)
    ctx.inject(xf, psd_d, inj["alpha"], inj["delta"], t0, t15, inj["psi"], inj["phi_c"], inj["cos_iota"],
               inj["tc_sample"] / FS, 10.0)
    ctx.set_segment(0, xf, psd_d)
    return ctx, net, xf, psd_d, (inj, t0, t15)


class Search:
    """The search of the benchmark configuration on preallocated buffers: one
    iteration is the fitness of all particles and the swarm update; after the
    iterations the best of the runs is taken and that point polished."""

    def __init__(self, torch, ctx, sw, fused_tail=True):
        self.torch, self.ctx, self.sw, self.fused_tail = torch, ctx, sw, fused_tail
        n = RUNS * PARTICLES
        dev = ctx.device
        self.seg = torch.zeros(n, dtype=torch.int32, device=dev)
        self.seg1 = torch.zeros(1, dtype=torch.int32, device=dev)
        self.f = torch.empty(n, dtype=torch.float64, device=dev)
        self.j = torch.empty(n, dtype=torch.int32, device=dev)
        self.pol_theta = torch.empty(1, 4, dtype=torch.float64, device=dev)
        self.pol_f = torch.empty(1, dtype=torch.float64, device=dev)
        self.pol_j = torch.empty(1, dtype=torch.int32, device=dev)
        self.graph = None

    def iteration(self, timed=False):
        self.ctx.set_timing(timed)   # kernel events bracket only the fitness launches
        self.ctx.eval(self.sw.theta, self.seg, self.f, self.j)
        self.ctx.set_timing(False)
        self.sw.step(self.f, self.j)

    def iterations(self, k):
        """k iterations: one pso_run call (the fused end of iteration), or k
        alternations of the fitness call and the swarm update."""
        if self.fused_tail:
            self.sw.run(k, self.seg, self.f, self.j)
        else:
            for _ in range(k):
                self.iteration()

    def capture(self, group):
        """Captures two HIP graphs: `group` iterations, and one iteration."""
        torch = self.torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.iterations(1)
        torch.cuda.current_stream().wait_stream(s)
        self.group = group
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.iterations(group)
        self.graph1 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph1):
            self.iterations(1)

    def run(self, steps):
        """`steps` iterations as graph replays."""
        for _ in range(steps // self.group):
            self.graph.replay()
        for _ in range(steps % self.group):
            self.graph1.replay()

    def polish(self):
        """Best of the runs (Sec. III), then the gradient polish of that point."""
        from paper_2002_02150_amd import polish
        self.sw.best()
        self.pol_theta.copy_(self.sw.out_theta.view(1, 4))
        polish(self.ctx, self.pol_theta, self.seg1, steps=POLISH_STEPS, step_frac=1e-3, trials=8,
               fitness=self.pol_f, argmax=self.pol_j)


POLISH_STEPS = 10
GRAPH_GROUP = 20   # PSO iterations per replayed HIP graph


def fp64_plain_rate(torch, net, xf, psd_d, thetas, dev, n_samples=N_SAMPLES):
    """Per-particle FP64 path: the same kernels in double precision, one
    evaluation per call, no batching."""
    import synth
    from paper_2002_02150_amd import FP64, Context
    ctx = Context.from_network(net, fs=FS, f_low=F_LOW, f_high=F_HIGH, box_lo=synth.SEARCH_BOX_30HZ_LO,
                               box_hi=synth.SEARCH_BOX_30HZ_HI, precision=FP64, max_batch=1, max_samples=n_samples)
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


_ORACLE = {}


def _oracle_init(seg, pos, ten):
    from threadpoolctl import threadpool_limits
    _ORACLE.update(seg=seg, pos=pos, ten=ten, limits=threadpool_limits(1))   # one thread per process


def _oracle_worker(th):
    from oracle import fitness as F
    return [F.fitness(_ORACLE["seg"], _ORACLE["pos"], _ORACLE["ten"], t) for t in th]


def _oracle_ready(_):
    return True


def cpu_baseline(xf_np, psd, net, thetas, sample, shape="4 det x 131072 samples"):
    """The FP64 oracle on the host cores: a pool of one process per core (the
    segment handed over once, the pool started before timing) evaluates
    `sample` points uniform in the rectangle (the first PSO batch, then more
    points drawn the same way).  Returns the rate, the oracle's segment and its
    (fitness, argmax) of the first len(thetas) points, in order."""
    import multiprocessing as mp
    import synth
    from oracle import fitness as F
    seg = F.prepare_segment(xf_np, psd, FS, F_LOW, F_HIGH)
    extra = synth.uniform_in_box(np.random.default_rng(synth.seed_sequence(2, 0, 3000)), max(0, sample - len(thetas)),
                                 synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI)
    th = np.concatenate([thetas, extra])[:sample]
    cores = max(1, min(os.cpu_count() or 1, 64))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores, initializer=_oracle_init, initargs=(seg, net.pos_m, net.tensor)) as pool:
        pool.map(_oracle_ready, range(cores))
        t = time.perf_counter()
        parts = pool.map(_oracle_worker, [th[i::cores] for i in range(cores)])
        dt = time.perf_counter() - t
    ref = [None] * len(th)
    for i, part in enumerate(parts):
        ref[i::cores] = part
    return dict(value=len(th) / dt, unit="evals/s", cores=cores, kind="oracle",
                sample=f"{len(th)} fitness evaluations uniform in the rectangle (the first PSO batch and more "
                       f"drawn alike; {shape}), one single-threaded process per host core, {dt:.1f} s wall"), \
        seg, ref[:len(thetas)]


def parity(torch, ctx, seg, net, thetas, ref, dev):
    """Error of the library's mixed path against the FP64 oracle on the same
    points: largest relative error of the fitness, and the argmax samples that
    differ (a differing sample counts as a near tie when the oracle's value
    there is within 1e-4 of its maximum)."""
    from oracle import fitness as F
    th = torch.from_numpy(np.ascontiguousarray(thetas)).to(dev)
    f, j = ctx.eval(th, torch.zeros(len(thetas), dtype=torch.int32, device=dev))
    f, j = f.cpu().numpy(), j.cpu().numpy()
    fo = np.array([r[0] for r in ref])
    jo = np.array([r[1] for r in ref])
    rel = np.abs(f - fo) / np.abs(fo)
    differ = np.nonzero(j != jo)[0]
    ties = sum(F.gamma2_at(seg, net.pos_m, net.tensor, thetas[k], int(j[k])) >= (1 - 1e-4) * fo[k] for k in differ)
    return {"points": int(len(thetas)), "max_rel_err_fitness": float(rel.max()),
            "mean_rel_err_fitness": float(rel.mean()), "argmax_differs": int(len(differ)),
            "argmax_differs_near_tie": int(ties),
            "max_argmax_delta": int(np.abs(j - jo).max()), "bar": "1e-4 relative; argmax equal or a near tie"}


def run_batched(a, torch, dev):
    """256 independent segments of 32/64/96/128 s at 2048 Hz (4 detectors), every
    second one with an SPA injection at SNR U[8, 14]; 40 particles x 4 runs per
    segment, so one PSO iteration evaluates 40,960 points of mixed segment
    lengths in one captured HIP graph."""
    import synth
    from paper_2002_02150_amd import Context, PsoConfig, Swarm
    from paper_2002_02150_amd.params import chirp_times
    n_seg, runs_per_seg = 256, 4
    lengths = (65536, 131072, 196608, 262144)
    rng = np.random.default_rng(synth.seed_sequence(3, 0, 0))
    seg_len = [lengths[i] for i in rng.integers(0, 4, n_seg)]
    net = synth.network("HLVK")
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    R = n_seg * runs_per_seg
    n = R * PARTICLES
    ctx = Context.from_network(net, fs=FS, f_low=F_LOW, f_high=F_HIGH, box_lo=lo, box_hi=hi, max_batch=n,
                               max_segments=n_seg, max_samples=max(lengths), schedule=SCHEDULES[a.schedule])
    gen = torch.Generator(device=dev).manual_seed(20020215 + 3)
    for s_id, N in enumerate(seg_len):
        half = N // 2 + 1
        psd = torch.from_numpy(synth.psd_matrix(4, N, FS)).to(dev)
        amp = torch.sqrt(torch.where(torch.isfinite(psd), psd, torch.zeros_like(psd)) * (N / FS) / 4.0)
        xf = torch.complex(torch.randn(4, half, generator=gen, device=dev, dtype=torch.float64),
                           torch.randn(4, half, generator=gen, device=dev, dtype=torch.float64)) * amp
        if s_id % 2 == 0:
            inj = synth.draw_injection(rng, N)
            t0, t15 = chirp_times(inj["m1"], inj["m2"], F_LOW)
            ctx.inject(xf, psd, inj["alpha"], inj["delta"], t0, t15, inj["psi"], inj["phi_c"], inj["cos_iota"],
                       inj["tc_sample"] / FS, float(rng.uniform(8.0, 14.0)))
        ctx.set_segment(s_id, xf, psd)
    sw = Swarm(ctx, PsoConfig(n_runs=R, n_particles=PARTICLES, n_iter=2000, seed=20020216))
    seg = torch.arange(R, device=dev, dtype=torch.int32).repeat_interleave(PARTICLES) // runs_per_seg
    f = torch.empty(n, dtype=torch.float64, device=dev)
    j = torch.empty(n, dtype=torch.int32, device=dev)
    sw.init()

    def iteration():
        if a.tail == "fused":
            sw.run(1, seg, f, j)
        else:
            ctx.eval(sw.theta, seg, f, j)
            sw.step(f, j)

    for _ in range(a.warmup):
        iteration()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        iteration()
    torch.cuda.current_stream().wait_stream(st)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        iteration()
    ev0 = ctx.evaluated()
    t = time.perf_counter()
    for _ in range(a.steps):
        g.replay()
    ev1 = ctx.evaluated()
    dt = time.perf_counter() - t
    mix = {str(N): seg_len.count(N) for N in lengths}
    out = {"metric": "coherent-fitness evals/s, 256 ragged 4-detector segments (32-128 s at 2048 Hz)",
           "value": (ev1 - ev0) / dt, "unit": "evals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64phase", "data": "synthetic",
           "config": {"workload": "256 noise realizations with segment lengths drawn from {32, 64, 96, 128} s at "
                                  "2048 Hz, 4 detectors, even segments with SPA injections at SNR U[8,14]; "
                                  "40 particles x 4 runs per segment, one PSO iteration (40,960 points) per step "
                                  "as a captured HIP graph", "segments_by_length": mix,
                      "global_batch": n, "parallelism": "single-gpu"},
           "points_per_s": a.steps * n / dt, "evaluated_fraction": (ev1 - ev0) / (a.steps * n)}
    ctx.close()
    print(json.dumps(out))


def run_gradient(a, torch, dev):
    """Fitness gradients at 4096 points within 1% (of the rectangle width) of
    the true parameters of an SNR-12 injection (4 detectors, 64 s at 2048 Hz),
    then the polish of the best of them."""
    import synth
    from paper_2002_02150_amd import Context, polish
    from paper_2002_02150_amd.params import chirp_times
    n = 4096
    net = synth.network("HLVK")
    psd = synth.psd_matrix(4, N_SAMPLES, FS)
    noise = synth.noise_matrix(4, 0, psd, N_SAMPLES, FS)
    rng = np.random.default_rng(synth.seed_sequence(4, 0, 1000))
    inj = synth.draw_injection(rng, N_SAMPLES)
    t0, t15 = chirp_times(inj["m1"], inj["m2"], F_LOW)
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    ctx = Context.from_network(net, fs=FS, f_low=F_LOW, f_high=F_HIGH, box_lo=lo, box_hi=hi, max_batch=n,
                               max_samples=N_SAMPLES, schedule=SCHEDULES[a.schedule])
    xf = torch.from_numpy(noise).to(dev)
    psd_d = torch.from_numpy(np.ascontiguousarray(psd)).to(dev)
    ctx.inject(xf, psd_d, inj["alpha"], inj["delta"], t0, t15, inj["psi"], inj["phi_c"], inj["cos_iota"],
               inj["tc_sample"] / FS, 12.0)
    ctx.set_segment(0, xf, psd_d)
    theta0 = np.array([inj["alpha"], inj["delta"], t0, t15])
    th = torch.from_numpy(synth.near_point(rng, n, theta0, lo, hi, 0.01)).to(dev)
    seg = torch.zeros(n, dtype=torch.int32, device=dev)
    f = torch.empty(n, dtype=torch.float64, device=dev)
    j = torch.empty(n, dtype=torch.int32, device=dev)
    g = torch.empty(n, 4, dtype=torch.float64, device=dev)
    for _ in range(a.warmup):
        ctx.grad(th, seg, f, j, g)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(a.steps):
        ctx.grad(th, seg, f, j, g)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    starts = th[:64].clone()
    f_start = f[:64].clone()
    f0 = ctx.eval(torch.from_numpy(theta0[None, :].copy()).to(dev), seg[:1])[0].item()
    t2 = time.perf_counter()
    _, fp, _ = polish(ctx, starts, seg[:64], steps=20, step_frac=1e-3, trials=16)
    torch.cuda.synchronize()
    dt2 = time.perf_counter() - t2
    out = {"metric": "fitness gradients/s (value, argmax and dGamma^2/dtheta), 4 det x 131072 samples",
           "value": a.steps * n / dt, "unit": "gradients/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64phase (FP64 chain rule)", "data": "synthetic",
           "config": {"workload": "4096 points within 1% of the rectangle width around the true parameters of an "
                                  "SNR-12 SPA injection, 4 detectors, 64 s at 2048 Hz; one step = one "
                                  "fitness_grad_batch call", "global_batch": n, "parallelism": "single-gpu"},
           "polish": {"starts": 64, "steps": 20, "trials": 16, "ms": dt2 * 1e3, "fitness_at_truth": f0,
                      "improved": int((fp > f_start).sum().item()),
                      "mean_gain": (fp - f_start).mean().item(), "best_after": fp.max().item(),
                      "best_before": f_start.max().item()}}
    ctx.close()
    print(json.dumps(out))


def run_sweep(a, torch, dev):
    """Fitness batches of n points uniform in the rectangle (every point
    evaluated) on the benchmark segment, n = 320 ... 20480: evals/s per batch
    size, each batch one fitness_eval_batch call replayed from a HIP graph."""
    import synth
    ctx, net, xf, psd_d, inj = make_workload(torch, dev, a.schedule, max_batch=20480)
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    rng = np.random.default_rng(synth.seed_sequence(2, 0, 2000))
    rows = []
    for n in (320, 1280, 5120, 20480):
        th = torch.from_numpy(synth.uniform_in_box(rng, n, lo, hi)).to(dev)
        seg = torch.zeros(n, dtype=torch.int32, device=dev)
        f = torch.empty(n, dtype=torch.float64, device=dev)
        j = torch.empty(n, dtype=torch.int32, device=dev)
        for _ in range(max(a.warmup, 1)):
            ctx.eval(th, seg, f, j)
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            ctx.eval(th, seg, f, j)
        torch.cuda.current_stream().wait_stream(st)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.eval(th, seg, f, j)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(a.steps):
            g.replay()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        rows.append({"batch": n, "evals_per_s": a.steps * n / dt, "ms_per_call": dt / a.steps * 1e3,
                     "hbm_alg_tb_per_s": a.steps * n * 32 * N_SAMPLES / dt / 1e12})
    ctx.close()
    out = {"metric": "coherent-fitness evals/s by batch size, 4 det x 131072 samples",
           "value": max(r["evals_per_s"] for r in rows), "unit": "evals/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64phase", "data": "synthetic",
           "config": {"workload": "batches of 320 to 20480 points uniform in the rectangle on the 4-detector, "
                                  "64-s, SNR-10 benchmark segment; one step = one fitness_eval_batch call "
                                  "(a captured HIP graph)", "parallelism": "single-gpu"},
           "sweep": rows}
    print(json.dumps(out))


HOUR_SAMPLES = 7372800
PAPER_KNL_HOUR = 40 * 1000 / (54.9 * 60)   # one PSO run (40 particles, 1000 iterations) in 54.9 min on KNL


def pass_roofline(name, avg_ms, alg_bytes):
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "avg_launch_ms": avg_ms, "alg_bytes_per_launch": alg_bytes}


def run_hour(a, torch, dev):
    """The paper's own layout (Sec. IV): one hour-long segment of 4-detector data
    at 2048 Hz (7,372,800 samples per detector, three-pass FFT plan) with an
    SNR-10 injection; PSO 8 runs x 40 particles, one step = the fitness of the
    320 particles and the swarm update, captured as HIP graphs of 20 steps; the
    best of the runs and its gradient polish are timed after the steps."""
    import synth
    from paper_2002_02150_amd import Context, PsoConfig, Swarm
    from paper_2002_02150_amd.params import chirp_times
    N, n = HOUR_SAMPLES, RUNS * PARTICLES
    net = synth.network("HLVK")
    psd = synth.psd_matrix(4, N, FS)
    noise = synth.noise_matrix(5, 0, psd, N, FS)
    inj = synth.draw_injection(np.random.default_rng(synth.seed_sequence(5, 0, 1000)), N)
    t0, t15 = chirp_times(inj["m1"], inj["m2"], F_LOW)
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    ws = int(a.hour_workspace_gib * (1 << 30))
    ctx = Context.from_network(net, fs=FS, f_low=F_LOW, f_high=F_HIGH, box_lo=lo, box_hi=hi, max_batch=n,
                               max_samples=N, workspace_bytes=ws, schedule=SCHEDULES[a.schedule])
    xf = torch.from_numpy(noise).to(dev)
    psd_d = torch.from_numpy(np.ascontiguousarray(psd)).to(dev)
    ctx.inject(xf, psd_d, inj["alpha"], inj["delta"], t0, t15, inj["psi"], inj["phi_c"], inj["cos_iota"],
               inj["tc_sample"] / FS, 10.0)
    ctx.set_segment(0, xf, psd_d)
    sw = Swarm(ctx, PsoConfig(n_runs=RUNS, n_particles=PARTICLES, n_iter=1000, seed=20020215))
    first_batch = sw.init().clone()
    search = Search(torch, ctx, sw, fused_tail=a.tail == "fused")
    for _ in range(a.warmup):
        search.iteration()
    search.capture(GRAPH_GROUP)
    torch.cuda.synchronize()
    ev0 = ctx.evaluated()
    t = time.perf_counter()
    search.run(a.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ev_mid = ctx.evaluated()
    tp = time.perf_counter()
    search.polish()
    torch.cuda.synchronize()
    dt_polish = time.perf_counter() - tp
    # eager steps with HIP events recorded by the three FFT passes' dispatch
    eager = min(a.steps, 20)
    ev2 = ctx.evaluated()
    for _ in range(eager):
        search.iteration(timed=True)
    torch.cuda.synchronize()
    ev3 = ctx.evaluated()
    timing = {k: ctx.read_timing(k) for k in ("pass1", "passm", "pass2")}
    pts = ev3 - ev2
    K = int(1000.0 * N / FS) - int(30.0 * N / FS)   # in-band bins 30 < f <= 1000 Hz
    per_point = {"pass1": 16 * N, "passm": 32 * N, "pass2": 16 * N}
    kname = {"pass1": "k_pass1", "passm": "k_passm", "pass2": "k_pass2"}
    lines = {}
    for k, (ms, cnt) in timing.items():
        alg = pts / max(cnt, 1) * per_point[k] + (8 * K * 4 + 8 * K if k == "pass1" else 0)
        lines[k] = pass_roofline(kname[k], ms / max(cnt, 1), alg)
        lines[k]["ms_per_step"] = ms / eager
    dom = max(lines, key=lambda k: lines[k]["ms_per_step"])
    # measured HBM bytes per point of each pass (rocprofv3 FETCH_SIZE / WRITE_SIZE
    # runs of this configuration, calibrated on a device copy), valid only for
    # the kernel sources they were taken on
    tf = os.path.join(ROOT, "profiles", "traffic_hour.json")
    if os.path.exists(tf):
        tr = json.load(open(tf))
        if tr.get("kernel_hash") == kernel_hash():
            for k in lines:
                bpp = tr.get("kernels", {}).get(kname[k], {}).get("bytes_per_point")
                if bpp is not None:
                    lines[k]["traffic"] = bpp * pts / max(timing[k][1], 1)
    value = (ev_mid - ev0) / dt
    out = {
        "metric": "coherent-fitness evals/s, 4 det x 7,372,800 samples (one hour at 2048 Hz)",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64phase", "data": "synthetic",
        "config": {"workload": "4 detectors (HLVK), one 60-min segment at 2048 Hz (7,372,800 samples), SNR-10 SPA "
                               "injection; PSO 8 runs x 40 particles, one step = fitness of the 320 particles + "
                               "swarm update (captured HIP graphs of 20 steps); the best of the runs and a "
                               f"{POLISH_STEPS}-step gradient polish of that point follow the timed steps "
                               "(polish_ms)",
                   "global_batch": n, "seq_len": N, "parallelism": "single-gpu",
                   "workspace_bytes": ctx.workspace_bytes},
        "roofline": dict(lines[dom], traffic=lines[dom].get("traffic")),
        "passes": lines,
        "paper_context": {"value": PAPER_KNL_HOUR, "unit": "evals/s",
                          "what": "one PSO run (40 particles, 1000 iterations) on 60 min of data took 54.9 min "
                                  "(median) on one KNL node; other hardware, shown for context"},
        "kernel_hash": kernel_hash(),
        "points_per_s": a.steps * n / dt, "evaluated_fraction": (ev_mid - ev0) / (a.steps * n),
        "best": {"fitness": search.pol_f.item(), "argmax": search.pol_j.item()},
        "polish_ms": dt_polish * 1e3,
    }
    if not a.no_fp64:
        rate64 = fp64_plain_rate(torch, net, xf, psd_d, first_batch[:8].contiguous(), dev, n_samples=N)
        out["fp64_plain"] = {"value": rate64, "unit": "evals/s", "speedup": value / rate64,
                             "what": "same kernels in FP64, one evaluation per call, no graph"}
    if not a.no_cpu_baseline:
        sample = first_batch[:32].cpu().numpy()
        out["cpu_baseline"], oseg, ref = cpu_baseline(xf.cpu().numpy(), psd_d.cpu().numpy(), net, sample, 32,
                                                      shape="4 det x 7,372,800 samples")
        out["parity"] = parity(torch, ctx, oseg, net, sample, ref, dev)
    out["evaluated_total"] = ctx.evaluated()   # every point the float passes processed in this process
    ctx.close()
    calib_copy(a, torch, dev, out)
    print(json.dumps(out))


def calib_copy(a, torch, dev, out):
    """One device-to-device copy of --calib-copy-mib MiB (HBM counter calibration)."""
    if a.calib_copy_mib:
        src = torch.ones(a.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = src.numel() * 4


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    from paper_2002_02150_amd import PsoConfig, Swarm
    dev = torch.device("cuda", 0)
    if a.steps is None:
        a.steps = {"search": 2000, "batched": 20, "gradient": 50, "sweep": 20, "hour": 200}[a.config]
    if a.config == "batched":
        return run_batched(a, torch, dev)
    if a.config == "gradient":
        return run_gradient(a, torch, dev)
    if a.config == "sweep":
        return run_sweep(a, torch, dev)
    if a.config == "hour":
        return run_hour(a, torch, dev)
    ctx, net, xf, psd_d, inj = make_workload(torch, dev, a.schedule)
    sw = Swarm(ctx, PsoConfig(n_runs=RUNS, n_particles=PARTICLES, n_iter=2000, seed=20020215))
    first_batch = sw.init().clone()
    search = Search(torch, ctx, sw, fused_tail=a.tail == "fused")
    for _ in range(a.warmup):
        search.iteration()
    search.capture(GRAPH_GROUP)   # one more iteration, then graphs of GRAPH_GROUP and 1 iterations
    torch.cuda.synchronize()
    # timed region 1: K iterations (graph replays)
    ev0 = ctx.evaluated()
    t = time.perf_counter()
    search.run(a.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ev_mid = ctx.evaluated()
    # once per search: the best of the runs and its gradient polish, timed apart
    tp = time.perf_counter()
    search.polish()
    torch.cuda.synchronize()
    dt_polish = time.perf_counter() - tp
    iterations_done = sw.iteration.item()
    # timed region 2: K iterations launched eagerly, HIP events recorded by the
    # FFT passes' dispatch
    ev2 = ctx.evaluated()
    t2 = time.perf_counter()
    per_launch = []
    prev = ev2
    for _ in range(a.steps):
        search.iteration(timed=True)
        if a.launch_counts:      # synchronises every step: only for pairing with counter runs
            cur = ctx.evaluated()
            per_launch.append(cur - prev)
            prev = cur
    torch.cuda.synchronize()
    dt2 = time.perf_counter() - t2
    ev3 = ctx.evaluated()
    ms1, n1 = ctx.read_timing("pass1")
    ms2, n2 = ctx.read_timing("pass2")
    msf, nf = ctx.read_timing("fused")
    evals = a.steps * RUNS * PARTICLES
    # value counts the fitness evaluations performed for the particles inside the
    # rectangle (points that flew out are not evaluated)
    particle_evals = ev_mid - ev0
    value = particle_evals / dt
    # dominant kernel and its algorithmic bytes per launch: the points evaluated
    # per fitness launch (inside the rectangle) times the bytes per point, plus
    # one read of the segment's data (y, 8 B per bin and detector, and the
    # FP64 basis table, 8 B per bin)
    pts = (ev3 - ev2) / a.steps
    K = 64000 - 1921 + 1
    D = 4
    per_launch_p1 = pts * 16 * N_SAMPLES + 8 * K * D + 8 * K
    per_launch_p2 = pts * 16 * N_SAMPLES
    avg1, avg2, avgf = ms1 / max(n1, 1), ms2 / max(n2, 1), msf / max(nf, 1)
    if nf:
        name, avg_ms, alg = "k_fused", avgf, per_launch_p1 + per_launch_p2
    elif avg1 >= avg2:
        name, avg_ms, alg = "k_pass1", avg1, per_launch_p1
    else:
        name, avg_ms, alg = "k_pass2", avg2, per_launch_p2
    achieved = alg / (avg_ms * 1e-3) / 1e9
    # measured HBM bytes of this kernel per launch: FETCH_SIZE (x2.0) + WRITE_SIZE
    # (x1.0) from rocprofv3 counter runs, fitted per evaluated point; valid only
    # for the kernel sources the counters were taken on
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        tr = json.load(open(tf))
        if tr.get("kernel_hash") == kernel_hash() and name in tr.get("kernels", {}):
            k = tr["kernels"][name]
            traffic = k["bytes_per_point"] * pts + k["bytes_fixed"]
    out = {
        "metric": "coherent-fitness evals/s, 4 det x 131072 samples; mixed vs FP64 plain; % HBM BW",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64phase", "data": "synthetic",
        "config": {"workload": "4 detectors (HLVK), 64 s at 2048 Hz (131072 samples), SNR-10 SPA injection; "
                               "PSO 8 runs x 40 particles, one step = fitness of the 320 particles + swarm update "
                               "(captured HIP graphs of 20 steps); the best of the runs and a "
                               f"{POLISH_STEPS}-step gradient polish of that point follow the timed steps "
                               "(polish_ms)",
                   "global_batch": RUNS * PARTICLES, "seq_len": N_SAMPLES, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_ms": avg_ms, "alg_bytes_per_launch": alg},
        "kernel_ms_per_step": {"k_pass1": avg1, "k_pass2": avg2, "k_fused": avgf},
        "schedule": a.schedule, "tail": a.tail,
        "eager_value": (ev3 - ev2) / dt2, "points_per_launch": pts,
        "kernel_hash": kernel_hash(),
        "points_per_s": evals / dt, "evaluated_fraction": particle_evals / evals,
        "best": {"fitness": search.pol_f.item(), "argmax": search.pol_j.item(), "iterations": iterations_done},
        "polish_ms": dt_polish * 1e3,
    }
    if not a.no_fp64:
        rate64 = fp64_plain_rate(torch, net, xf, psd_d, first_batch[:64].contiguous(), dev)
        out["fp64_plain"] = {"value": rate64, "unit": "evals/s", "speedup": value / rate64,
                             "what": "same kernels in FP64, one evaluation per call, no graph"}
    if not a.no_cpu_baseline:
        sample = first_batch.cpu().numpy()
        out["cpu_baseline"], oseg, ref = cpu_baseline(xf.cpu().numpy(), psd_d.cpu().numpy(), net, sample,
                                                      a.cpu_sample)
        out["parity"] = parity(torch, ctx, oseg, net, sample, ref, dev)
        from oracle import fitness as F
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            t1 = time.perf_counter()
            for t_ in sample[:8]:
                F.fitness(oseg, net.pos_m, net.tensor, t_)
            out["cpu_baseline_1core"] = {"value": 8 / (time.perf_counter() - t1), "unit": "evals/s", "cores": 1,
                                         "kind": "oracle", "sample": "8 points of the first PSO batch, one thread"}
    ctx.close()
    if per_launch:
        out["eager_launch_points"] = per_launch
    calib_copy(a, torch, dev, out)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
