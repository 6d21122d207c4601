"""pso_run (whole PSO iterations with the fused tail kernel: finalize, swarm
update and the next set-up in one launch) against the separate calls it
replaces: n iterations of fitness_eval_batch + pso_step on the same swarm give
the same swarm state, points, fitness and samples bit for bit, and the same
count of evaluated points."""
import numpy as np
import pytest
import torch

from tests._cases import Case
from tests._gpu import dev, make_ctx, require_gpu, upload

pytestmark = pytest.mark.gpu

STATE = ("x", "v", "pbest_x", "pbest_f", "pbest_j", "best_x", "best_f", "best_j", "theta")


def _pair(ctx, runs, particles, n_iter, seed):
    from paper_2002_02150_amd import PsoConfig, Swarm
    cfg = PsoConfig(n_runs=runs, n_particles=particles, n_iter=n_iter, seed=seed)
    a, b = Swarm(ctx, cfg), Swarm(ctx, cfg)
    a.init()
    b.init()
    return a, b


def _alternate(ctx, sw, seg, k):
    """k iterations as separate calls; returns the last fitness and samples."""
    f = j = None
    for _ in range(k):
        f, j = ctx.eval(sw.theta, seg)
        sw.step(f, j)
    return f, j


def _assert_same(a, b):
    for name in STATE:
        assert torch.equal(getattr(a, name), getattr(b, name)), name
    assert a.iteration.item() == b.iteration.item()


def _run_and_compare(ctx, a, b, seg, k):
    n = a.n
    f = torch.empty(n, dtype=torch.float64, device=dev())
    j = torch.empty(n, dtype=torch.int32, device=dev())
    e0 = ctx.evaluated()
    fa, ja = _alternate(ctx, a, seg, k)
    e1 = ctx.evaluated()
    b.run(k, seg, f, j)
    e2 = ctx.evaluated()
    _assert_same(a, b)
    assert torch.equal(fa, f) and torch.equal(ja, j)
    assert e2 - e1 == e1 - e0 > 0
    return f, j


def test_pso_run_single_segment_bitwise():
    """One segment, 4 runs x 40 particles (the fused tail): 25 iterations in one
    call, then 12 more, each equal to the separate calls; an ordinary
    fitness call afterwards still sees empty work lists."""
    require_gpu()
    case = Case("HL", 8192, 1024.0, snr=12.0, cfg=1, realization=3)
    ctx = make_ctx(case, 0, max_batch=160)
    upload(ctx, 0, case)
    a, b = _pair(ctx, 4, 40, 300, 2024)
    seg = torch.zeros(160, dtype=torch.int32, device=dev())
    _run_and_compare(ctx, a, b, seg, 25)
    _run_and_compare(ctx, a, b, seg, 12)
    f1, j1 = ctx.eval(b.theta, seg)
    f2, j2 = ctx.eval(a.theta, seg)
    assert torch.equal(f1, f2) and torch.equal(j1, j2)
    ctx.close()


def test_pso_run_ragged_segments_bitwise():
    """Three segments of different lengths (three FFT plans in one iteration),
    two runs each, 20 particles per run (work-groups with idle lanes), in
    single and double precision."""
    require_gpu()
    cases = [Case("HLV", n, 2048.0, snr=12.0, cfg=12, realization=i) for i, n in enumerate((8192, 24576, 16384))]
    for prec in (0, 1):
        ctx = make_ctx(cases[0], prec, max_batch=120, max_segments=3, max_samples=24576)
        for i, c in enumerate(cases):
            upload(ctx, i, c)
        a, b = _pair(ctx, 6, 20, 40, 99 + prec)
        seg = (torch.arange(6, dtype=torch.int32, device=dev()) // 2).repeat_interleave(20)
        _run_and_compare(ctx, a, b, seg, 7 if prec else 15)
        ctx.close()


def test_pso_run_large_runs_take_separate_kernels():
    """Runs of more than 128 particles take the separate launches, with the
    same results."""
    require_gpu()
    case = Case("HL", 2048, 1024.0, snr=12.0, cfg=23, realization=1)
    ctx = make_ctx(case, 0, max_batch=260)
    upload(ctx, 0, case)
    a, b = _pair(ctx, 2, 130, 10, 5)
    seg = torch.zeros(260, dtype=torch.int32, device=dev())
    _run_and_compare(ctx, a, b, seg, 4)
    ctx.close()


def test_pso_run_captured_graph_replays():
    """A captured pso_run of 10 iterations replayed three times, with eager
    fitness calls and synchronisation between the replays, follows the
    separate calls bit for bit (the iteration count and the work-list sets
    live on the device and in the launch order, so every replay continues the
    search)."""
    require_gpu()
    case = Case("HL", 8192, 1024.0, snr=12.0, cfg=1, realization=4)
    ctx = make_ctx(case, 0, max_batch=160)
    upload(ctx, 0, case)
    a, b = _pair(ctx, 4, 40, 100, 31337)
    seg = torch.zeros(160, dtype=torch.int32, device=dev())
    f = torch.empty(160, dtype=torch.float64, device=dev())
    j = torch.empty(160, dtype=torch.int32, device=dev())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run(1, seg, f, j)      # warm-up iteration on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    _alternate(ctx, a, seg, 1)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run(10, seg, f, j)
    probe = torch.from_numpy(case.theta0[None, :].copy()).to(dev())
    for r in range(3):
        g.replay()
        torch.cuda.synchronize()
        fa, ja = _alternate(ctx, a, seg, 10)
        _assert_same(a, b)
        assert torch.equal(fa, f) and torch.equal(ja, j)
        assert b.iteration.item() == 1 + 10 * (r + 1)
        ctx.eval(probe, torch.zeros(1, dtype=torch.int32, device=dev()))
    ctx.close()


def test_pso_run_errors():
    """Capacity and argument checks of pso_run."""
    require_gpu()
    from paper_2002_02150_amd import FcasError
    case = Case("HL", 2048, 1024.0, snr=None, cfg=23)
    ctx = make_ctx(case, 0, max_batch=80)
    upload(ctx, 0, case)
    from paper_2002_02150_amd import PsoConfig, Swarm
    sw = Swarm(ctx, PsoConfig(n_runs=3, n_particles=40, n_iter=5, seed=1))
    sw.init()
    seg = torch.zeros(120, dtype=torch.int32, device=dev())
    f = torch.empty(120, dtype=torch.float64, device=dev())
    j = torch.empty(120, dtype=torch.int32, device=dev())
    with pytest.raises(FcasError):
        sw.run(2, seg, f, j)          # 120 points > max_batch 80
    ok = Swarm(ctx, PsoConfig(n_runs=2, n_particles=40, n_iter=5, seed=1))
    ok.init()
    with pytest.raises(FcasError):
        ok.run(-1, seg[:80], f[:80], j[:80])
    ok.run(0, seg[:80], f[:80], j[:80])
    assert ok.iteration.item() == 0
    ctx.close()
