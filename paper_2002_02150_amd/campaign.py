"""Searches of many registered segments at once: every segment gets its own
PSO runs, all runs of all segments are one batch per iteration (captured HIP
graphs of up to 20 iterations), then the best run of each segment is polished
by gradient ascent (fitness_polish).  Used by the full-length search and the
detection-statistics study."""
from __future__ import annotations

import time

import torch

from . import PsoConfig, Swarm, polish


def search_segments(ctx, n_seg, runs=8, particles=40, iters=2000, seed=20020215, polish_steps=20, trials=16,
                    log=None):
    """PSO search of segments 0..n_seg-1 of `ctx` (its max_batch must hold
    n_seg * runs * particles points).  Returns a dict of per-segment device
    tensors: rho_sq_pso (best of the runs), rho_sq, theta [n_seg][4], argmax
    (after the polish), and the seconds the device took."""
    dev = ctx.device
    R = n_seg * runs
    n = R * particles
    sw = Swarm(ctx, PsoConfig(n_runs=R, n_particles=particles, n_iter=iters, seed=seed))
    seg = (torch.arange(R, device=dev, dtype=torch.int32) // runs).repeat_interleave(particles)
    f = torch.empty(n, dtype=torch.float64, device=dev)
    j = torch.empty(n, dtype=torch.int32, device=dev)

    def iterations(k):
        # k iterations (fitness, then swarm update) in one pso_run call
        sw.run(k, seg, f, j)

    group = min(20, iters)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    sw.init()
    st = torch.cuda.Stream(dev)
    st.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(st):
        iterations(1)                     # iteration 1, eagerly, before the capture
    torch.cuda.current_stream(dev).wait_stream(st)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        iterations(group)
    graph1 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph1):
        iterations(1)
    rest = iters - 1
    for g in range(rest // group):
        graph.replay()
        if log is not None and (g + 1) % 20 == 0:     # progress (waits for the device)
            torch.cuda.synchronize(dev)
            log(f"iteration {1 + (g + 1) * group}: {time.perf_counter() - t0:.1f} s")
    for _ in range(rest % group):
        graph1.replay()
    # best of each segment's runs, in the library (pso_best_segments)
    f_pso, theta, _, _ = sw.best_segments(runs)
    seg_best = torch.arange(n_seg, device=dev, dtype=torch.int32)
    if polish_steps > 0:
        theta, f_pol, j_pol = polish(ctx, theta, seg_best, steps=polish_steps, step_frac=1e-3, trials=trials)
    else:
        f_pol, j_pol = ctx.eval(theta, seg_best)
    torch.cuda.synchronize(dev)
    return dict(rho_sq_pso=f_pso, rho_sq=f_pol, theta=theta, argmax=j_pol, seconds=time.perf_counter() - t0)
