"""GPU parity of fitness_grad_batch (fixed-sample adjoint) and of the swarm
kernels (pso_init / pso_step / pso_best) against the oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import gradient as G
from oracle import pso as OP
from tests._cases import Case
from tests._gpu import dev, make_ctx, require_gpu, upload

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol,rtol", [(0, 1e-5, 1e-4), (1, 1e-10, 1e-9)], ids=["mixed", "fp64"])
def test_gradient_matches_oracle(prec, tol, rtol):
    """dGamma^2/dtheta at the GPU's maximising sample vs the oracle's analytic
    gradient at the same sample (itself pinned to finite differences): every
    component within tol of the gradient's scale in rectangle-width units, and
    every component above 1e-3 of that scale within rtol of itself."""
    require_gpu()
    case = Case("HLVK", 16384, 2048.0, snr=12.0, cfg=20)
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    rng = np.random.default_rng(21)
    th = synth.near_point(rng, 12, case.theta0, lo, hi, 0.01)
    ctx = make_ctx(case, prec, max_batch=len(th))
    upload(ctx, 0, case)
    f, j, g = ctx.grad(torch.from_numpy(th).to(dev()), torch.zeros(len(th), dtype=torch.int32, device=dev()))
    f, j, g = f.cpu().numpy(), j.cpu().numpy(), g.cpu().numpy()
    w = np.array(hi) - np.array(lo)
    worst_abs = worst_rel = 0.0
    for k in range(len(th)):
        g2, _, go = G.fitness_gradient(case.seg, case.net.pos_m, case.net.tensor, th[k], int(j[k]))
        scale = np.max(np.abs(go * w))     # gradient scale in box-width units
        err = np.abs((g[k] - go) * w)
        assert np.all(err <= tol * scale), (k, g[k], go)
        big = np.abs(go * w) > 1e-3 * scale
        assert np.all(err[big] <= rtol * np.abs(go * w)[big]), (k, g[k], go)
        worst_abs = max(worst_abs, float(np.max(err) / scale))
        worst_rel = max(worst_rel, float(np.max(err[big] / np.abs(go * w)[big])))
    print(f"gradient 16384 prec={prec}: max |dg w|/s {worst_abs:.3e}, max per-component rel {worst_rel:.3e}")
    ctx.close()


def test_fitnessfn_backward_and_polish():
    require_gpu()
    from paper_2002_02150_amd import FitnessFn, polish
    case = Case("HLVK", 16384, 2048.0, snr=15.0, cfg=22)
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    rng = np.random.default_rng(5)
    th = synth.near_point(rng, 4, case.theta0, lo, hi, 0.002)
    ctx = make_ctx(case, 0, max_batch=32)
    upload(ctx, 0, case)
    t = torch.from_numpy(th).to(dev()).requires_grad_(True)
    seg = torch.zeros(4, dtype=torch.int32, device=dev())
    f, j = FitnessFn.apply(t, seg, ctx)
    (f * torch.arange(1, 5, device=dev(), dtype=torch.float64)).sum().backward()
    _, _, g = ctx.grad(t.detach(), seg)
    assert torch.allclose(t.grad, g * torch.arange(1, 5, device=dev(), dtype=torch.float64)[:, None])
    th2, f2, j2 = polish(ctx, t.detach().clone(), seg, steps=10)
    assert torch.all(f2 >= f.detach())
    # the polished points are what they claim: re-evaluate them
    f3, j3 = ctx.eval(th2, seg)
    assert torch.equal(f3, f2) and torch.equal(j3, j2)
    ctx.close()
    # On noiseless data the global maximum is SNR^2 at the true parameters:
    # the polish must raise every point strictly, never pass SNR^2, and close
    # most of the gap to it.
    clean = Case("HLVK", 16384, 2048.0, snr=15.0, noise=False, cfg=22)
    ctx = make_ctx(clean, 0, max_batch=32)
    upload(ctx, 0, clean)
    th = torch.from_numpy(synth.near_point(rng, 4, clean.theta0, lo, hi, 0.002)).to(dev())
    fs, _ = ctx.eval(th, seg)
    fs = fs.clone()
    _, fp, _ = polish(ctx, th.clone(), seg, steps=10)
    assert torch.all(fp > fs), (fs, fp)
    assert torch.all(fp <= 225.0 * (1 + 1e-4)), fp
    assert (225.0 - fp).sum() < 0.5 * (225.0 - fs).sum(), (fs, fp)
    ctx.close()


def _gpu_state_to_numpy(sw):
    return {k: getattr(sw, k).cpu().numpy() for k in ("x", "v", "pbest_x", "pbest_f", "pbest_j", "best_x", "best_f", "best_j")}


def test_pso_trajectory_bitwise_equal_to_oracle():
    """Given the same fitness values, the device swarm follows the oracle's
    trajectory bit for bit (same Philox stream, same FP64 operation order)."""
    require_gpu()
    from paper_2002_02150_amd import PsoConfig, Swarm
    case = Case("HL", 2048, 1024.0, snr=None, cfg=23)
    ctx = make_ctx(case, 0, max_batch=120)
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    cfg = PsoConfig(n_runs=3, n_particles=40, n_iter=6, seed=0x1234_5678_9ABC)
    sw = Swarm(ctx, cfg)
    th_gpu = sw.init().cpu().numpy()
    p = OP.PsoParams(n_runs=3, n_particles=40, n_iter=6, seed=cfg.seed)
    st, th_ora = OP.init(p, lo, hi)
    assert np.array_equal(th_gpu, th_ora)
    rng = np.random.default_rng(9)
    for it in range(6):
        fit = rng.normal(50.0, 10.0, 120)
        fit[rng.random(120) < 0.2] = -np.inf
        fit[5] = fit[6]  # a tie
        am = rng.integers(0, 2048, 120).astype(np.int32)
        th_g = sw.step(torch.from_numpy(fit).to(dev()), torch.from_numpy(am).to(dev())).cpu().numpy()
        th_o = OP.step(p, st, fit, am, it, lo, hi)
        assert np.array_equal(th_g, th_o), it
        s = _gpu_state_to_numpy(sw)
        assert np.array_equal(s["x"], st.x) and np.array_equal(s["v"], st.v)
        assert np.array_equal(s["pbest_x"], st.pbest_x) and np.array_equal(s["pbest_f"], st.pbest_f)
        assert np.array_equal(s["pbest_j"], st.pbest_j) and np.array_equal(s["best_f"], st.best_f)
        assert np.array_equal(s["best_x"], st.best_x) and np.array_equal(s["best_j"], st.best_j)
        assert sw.iteration.item() == it + 1
    bf, bt, bj, br = sw.best()
    of, ot, oj, orun = OP.best_of_runs(st, lo, hi)
    assert bf.item() == of and np.array_equal(bt.cpu().numpy(), ot) and bj.item() == oj and br.item() == orun
    ctx.close()


def test_pso_best_segments_bitwise_equal_to_oracle():
    """Best of the runs of each segment (runs grouped by segment, the layout of
    the multi-segment searches; optionally of only the first runs of each
    group, as the tuning metric compares), on the device, equals the oracle's
    best of runs applied to each group bit for bit: fitness, theta, sample and
    run index (lowest run on ties, which the fitness values force here)."""
    require_gpu()
    from types import SimpleNamespace
    from paper_2002_02150_amd import PsoConfig, Swarm
    case = Case("HL", 2048, 1024.0, snr=None, cfg=24)
    ctx = make_ctx(case, 0, max_batch=240)
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    R, P, m = 6, 40, 2
    cfg = PsoConfig(n_runs=R, n_particles=P, n_iter=4, seed=99)
    sw = Swarm(ctx, cfg)
    sw.init()
    p = OP.PsoParams(n_runs=R, n_particles=P, n_iter=4, seed=cfg.seed)
    st, _ = OP.init(p, lo, hi)
    rng = np.random.default_rng(12)
    for it in range(4):
        fit = rng.normal(50.0, 10.0, R * P)
        fit[rng.random(R * P) < 0.2] = -np.inf
        fit[P:2 * P] = fit[:P]          # runs 0 and 1 (segment 0) tie
        am = rng.integers(0, 2048, R * P).astype(np.int32)
        sw.step(torch.from_numpy(fit).to(dev()), torch.from_numpy(am).to(dev()))
        OP.step(p, st, fit, am, it, lo, hi)
    for m, u in ((2, 2), (3, 2), (6, 4), (1, 1)):
        f, th, j, run = (t.cpu().numpy() for t in sw.best_segments(m, u))
        assert len(f) == R // m
        for g in range(R // m):
            sl = slice(g * m, g * m + u)
            sub = SimpleNamespace(best_f=st.best_f[sl], best_x=st.best_x[sl], best_j=st.best_j[sl])
            of, ot, oj, orun = OP.best_of_runs(sub, lo, hi)
            assert f[g] == of and np.array_equal(th[g], ot) and j[g] == oj and run[g] == g * m + orun, (m, u, g)
        if m == 2:
            assert run[0] == 0
    from paper_2002_02150_amd import FcasError
    for m, u in ((4, 4), (2, 3), (2, 0)):      # m must divide the 6 runs, 1 <= u <= m
        with pytest.raises(FcasError):
            sw.best_segments(m, u)
    ctx.close()


def test_pso_search_recovers_injection():
    """A best-of-4-runs search on a config-1 style segment (2 detectors, 8 s at
    1024 Hz, SNR 12) reaches the fitness at the true parameters (the tuning
    criterion of Sec. III, with a 5% margin).  The search runs twice: eagerly,
    and as one captured HIP graph of an iteration (fitness batch + swarm
    update) replayed, with eager work and synchronisation between replays;
    both must give bit-identical swarms."""
    require_gpu()
    from paper_2002_02150_amd import PsoConfig, Swarm
    case = Case("HL", 8192, 1024.0, snr=12.0, cfg=1, realization=0)
    ctx = make_ctx(case, 0, max_batch=160)
    upload(ctx, 0, case)
    f0, _ = ctx.eval(torch.from_numpy(case.theta0[None, :].copy()).to(dev()),
                     torch.zeros(1, dtype=torch.int32, device=dev()))
    seg = torch.zeros(160, dtype=torch.int32, device=dev())
    cfg = PsoConfig(n_runs=4, n_particles=40, n_iter=300, seed=77)
    eager = Swarm(ctx, cfg)
    th = eager.init()
    for it in range(300):
        f, j = ctx.eval(th, seg)
        th = eager.step(f, j)
    graph = Swarm(ctx, cfg)
    th = graph.init()
    f_buf = torch.empty(160, dtype=torch.float64, device=dev())
    j_buf = torch.empty(160, dtype=torch.int32, device=dev())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx.eval(th, seg, f_buf, j_buf)   # first iteration eagerly, on the capture stream
        graph.step(f_buf, j_buf)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.eval(th, seg, f_buf, j_buf)
        graph.step(f_buf, j_buf)
    for it in range(299):
        g.replay()
        if it % 50 == 0:
            torch.cuda.synchronize()
            assert graph.iteration.item() == it + 2
            ctx.eval(torch.from_numpy(case.theta0[None, :].copy()).to(dev()),
                     torch.zeros(1, dtype=torch.int32, device=dev()))
    torch.cuda.synchronize()
    assert graph.iteration.item() == 300 and eager.iteration.item() == 300
    for name in ("x", "v", "pbest_x", "pbest_f", "pbest_j", "best_x", "best_f", "best_j"):
        assert torch.equal(getattr(eager, name), getattr(graph, name)), name
    bf, bt, bj, br = graph.best()
    assert bf.item() >= 0.95 * f0.item(), (bf.item(), f0.item())
    ctx.close()


def test_single_segment_search_small():
    """The paper's layout (the whole stretch one segment, three-pass FFT plan,
    one injection, batched runs, polish) end to end on a 225-s stretch."""
    require_gpu()
    from paper_2002_02150_amd.full_search import run_single_segment
    out = run_single_segment(minutes=3.75, iters=40, runs=2, polish_steps=3, log=lambda s: None)
    assert out["samples"] == 460800 and out["points_per_iteration"] == 80
    assert out["evaluated_points"] > 0 and out["t_run_s"] > 0
    d = out["injection"]
    assert d["rho_sq"] >= d["rho_sq_pso"] - 1e-9 and d["rho0_sq"] > 0
    assert abs(d["rho0_sq"] / d["snr"] ** 2 - 1.0) < 0.5


def test_hour_h0_small():
    """The hour-long H0 mode (time-slid 7,372,800-sample noise segments,
    three-pass FFT) runs end to end for two slides and its values combine into
    a threshold."""
    require_gpu()
    from paper_2002_02150_amd.detection import combine, hour_h0
    out = hour_h0(1, 2, iters=6, runs=1, group=2, polish_steps=1, log=lambda s: None)
    assert sorted(out["rho"]) == [1, 2] and all(v > 0 for v in out["rho"].values())
    c = combine([out])
    assert c["segments_h0"] == 2 and c["eta"] > max(out["rho"].values())
