"""FFT plan autotuner: times every plan of each segment length on this device,
over a grid of persistent work-group counts for the two passes, and writes the
fastest choice per length to tuning.json (applied by Context by default).

    python -m paper_2002_02150_amd.autotune [--lengths 131072,262144] [--out PATH]

Timing: fitness batches of `batch` points spread over the search rectangle
(every point evaluated; 256 by default, between the 192 points a 320-particle
swarm keeps inside the rectangle early in a search and the 311 it keeps at the
end), HIP events around `reps` back-to-back calls, best of three such runs.  The data are random: the cost of an evaluation does not depend
on the data values.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import torch

from . import fcas

DEFAULT_LENGTHS = (8192, 65536, 131072, 196608, 262144, 460800, 3686400, 7372800)
GRIDS = (1024, 2048, 4096)
# rectangle of component masses in [1, 3] Msun at f_low = 30 Hz
BOX_LO = (0.0, -math.pi / 2, 15.0336, 0.841913)
BOX_HI = (2.0 * math.pi, math.pi / 2, 93.8141, 1.75126)


def _network(n_det, device):
    """A generic network: detectors spread over the globe with crossed arms."""
    pos, ten = [], []
    for i in range(n_det):
        lat, lon = 0.7 * math.sin(1.3 * i + 0.2), 2.1 * i + 0.4
        r = 6.37e6
        p = (r * math.cos(lat) * math.cos(lon), r * math.cos(lat) * math.sin(lon), r * math.sin(lat))
        east = (-math.sin(lon), math.cos(lon), 0.0)
        north = (-math.sin(lat) * math.cos(lon), -math.sin(lat) * math.sin(lon), math.cos(lat))
        a = [(math.cos(0.3 * i) * e + math.sin(0.3 * i) * n) for e, n in zip(east, north)]
        b = [(-math.sin(0.3 * i) * e + math.cos(0.3 * i) * n) for e, n in zip(east, north)]
        pos.append(p)
        ten.append([[0.5 * (a[x] * a[y] - b[x] * b[y]) for y in range(3)] for x in range(3)])
    return pos, ten


def time_plan(ctx, plan, g1, g2, xf, psd, theta, seg, reps):
    """Mean device time (ms) of one fitness call, over `reps` back-to-back calls."""
    ctx.select_plan(plan, g1, g2)
    ctx.set_segment(0, xf, psd)
    f = torch.empty(theta.shape[0], dtype=torch.float64, device=ctx.device)
    j = torch.empty(theta.shape[0], dtype=torch.int32, device=ctx.device)
    for _ in range(3):
        ctx.eval(theta, seg, f, j)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    samples = []
    for _ in range(3):
        e0.record()
        for _ in range(reps):
            ctx.eval(theta, seg, f, j)
        e1.record()
        torch.cuda.synchronize(ctx.device)
        samples.append(e0.elapsed_time(e1) / reps)
    return min(samples)


def autotune(lengths=DEFAULT_LENGTHS, n_det=4, fs=2048.0, batch=256, reps=10, grids=GRIDS, out=fcas.TUNING_PATH,
             device=0, log=print):
    dev = torch.device("cuda", device)
    pos, ten = _network(n_det, dev)
    gen = torch.Generator(device="cpu").manual_seed(1234)
    results, choices = [], {}
    for n in lengths:
        cands = [p for p, d in fcas.plans() if d["n"] == n]
        if not cands:
            continue
        half = n // 2 + 1
        xf = torch.complex(torch.randn(n_det, half, generator=gen, dtype=torch.float64),
                           torch.randn(n_det, half, generator=gen, dtype=torch.float64)).to(dev)
        psd = torch.ones(n_det, half, dtype=torch.float64, device=dev)
        u = torch.rand(batch, 4, generator=gen, dtype=torch.float64)
        lo, hi = torch.tensor(BOX_LO, dtype=torch.float64), torch.tensor(BOX_HI, dtype=torch.float64)
        theta = (lo + u * (hi - lo)).to(dev)
        seg = torch.zeros(batch, dtype=torch.int32, device=dev)
        # the long three-pass lengths are timed with the 4 GiB workspace their
        # searches use (36 hour-long points per launch, measured fastest)
        ws = min(4 << 30, batch * 2 * n * 8) if n > 262144 else 0
        ctx = fcas.Context(pos, ten, fs=fs, f_low=30.0, f_high=1000.0, box_lo=BOX_LO, box_hi=BOX_HI,
                           max_batch=batch, max_samples=n, device=device, tuning=None, workspace_bytes=ws)
        best = None
        for p in cands:
            for g1 in grids:
                for g2 in grids:
                    ms = time_plan(ctx, p, g1, g2, xf, psd, theta, seg, reps)
                    results.append(dict(n=n, plan=p, grid1=g1, grid2=g2, ms=ms))
                    if best is None or ms < best["ms"]:
                        best = dict(plan=p, grid1=g1, grid2=g2, ms=ms)
            log(f"N={n} plan {p}: best so far {best}")
        ctx.close()
        choices[str(n)] = best
        log(f"N={n}: chose {best}")
    doc = dict(device=torch.cuda.get_device_name(dev), n_det=n_det, batch=batch, reps=reps,
               what="mean device time of one fitness call (set-up, passes, finalize)",
               written=time.strftime("%Y-%m-%d %H:%M:%S"), choices=choices, measurements=results)
    if out:
        with open(out, "w") as fh:
            json.dump(doc, fh, indent=1)
            fh.write("\n")
    return doc


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--lengths", default=",".join(str(n) for n in DEFAULT_LENGTHS))
    ap.add_argument("--out", default=fcas.TUNING_PATH)
    ap.add_argument("--reps", type=int, default=10)
    a = ap.parse_args(argv)
    autotune(tuple(int(x) for x in a.lengths.split(",")), reps=a.reps, out=a.out,
             log=lambda s: print(s, flush=True))


if __name__ == "__main__":
    sys.exit(main())
