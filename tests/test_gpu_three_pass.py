"""GPU parity of the three-pass lengths (N = N1 * 225 * N2: 225 s, 30 min and
one hour at 2048 Hz) against the FP64 oracle, through the C ABI.

The hour-long segment is the paper's own search length (Sec. IV: one segment
of 7,372,800 samples per detector).  Bars as for the two-pass plans: mixed
path within 1e-4 relative in fitness, FP64 path within 1e-9, argmax within one
sample or an equally good sample; results bitwise independent of grids and
workspace chunking.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import gradient as G
from tests._cases import Case
from tests._gpu import assert_parity, dev, make_ctx, oracle_eval, require_gpu, thetas_for, upload

pytestmark = pytest.mark.gpu

HOUR = 7372800


def _plan_of(n):
    from paper_2002_02150_amd.fcas import plans
    return next(p for p, d in plans() if d["n"] == n)


def _eval(ctx, th, seg=0):
    f, j = ctx.eval(torch.from_numpy(th).to(dev()), torch.full((len(th),), seg, dtype=torch.int32, device=dev()))
    return f.cpu().numpy(), j.cpu().numpy()


@pytest.mark.parametrize("names,prec", [("HLVK", 0), ("HLVK", 1), ("L", 0), ("HLVKHL", 0)],
                         ids=["HLVK-mixed", "HLVK-fp64", "L-mixed", "HLVKHL-mixed"])
def test_three_pass_225s_matches_oracle(names, prec):
    """460,800 samples: every point of a batch with near, uniform, corner and
    outside-the-rectangle points, for one to six detectors."""
    require_gpu()
    case = Case(names, 460800, 2048.0, snr=12.0, cfg=30, realization=prec)
    rng = np.random.default_rng(250 + prec)
    th = thetas_for(case, rng, n_near=6, n_uniform=6)
    ctx = make_ctx(case, prec, max_batch=len(th))
    upload(ctx, 0, case)
    f, j = _eval(ctx, th)
    fo, jo = oracle_eval(case, th)
    assert_parity(case, th, f, j, fo, jo, 1e-4 if prec == 0 else 1e-9)
    assert f[-3] == -np.inf and j[-3] == -1
    ctx.close()


@pytest.mark.parametrize("n,prec", [(3686400, 0), (HOUR, 0), (HOUR, 1)], ids=["30min-mixed", "1h-mixed", "1h-fp64"])
def test_three_pass_long_segments_sampled(n, prec):
    """30-minute and one-hour segments: a batch of near and uniform points,
    the oracle checking the first, the last and one in between."""
    require_gpu()
    case = Case("HLVK", n, 2048.0, snr=12.0, cfg=31, realization=n % 97)
    rng = np.random.default_rng(n % 1000 + prec)
    th = thetas_for(case, rng, n_near=5, n_uniform=5, extras=False)
    ctx = make_ctx(case, prec, max_batch=len(th))
    upload(ctx, 0, case)
    f, j = _eval(ctx, th)
    assert np.all(np.isfinite(f)) and np.all((j >= 0) & (j < n))
    idx = np.array([0, 4, len(th) - 1])
    fo, jo = oracle_eval(case, th[idx])
    assert_parity(case, th[idx], f[idx], j[idx], fo, jo, 1e-4 if prec == 0 else 1e-9)
    ctx.close()


def test_hour_noiseless_identity():
    """Gamma^2 at the true parameters of a noiseless hour-long signal equals
    SNR^2 and its maximum sits on the injected coalescence sample."""
    require_gpu()
    case = Case("HLVK", HOUR, 2048.0, snr=11.0, noise=False, cfg=32)
    ctx = make_ctx(case, 0, max_batch=1)
    upload(ctx, 0, case)
    f, j = _eval(ctx, case.theta0[None, :].copy())
    assert f[0] == pytest.approx(121.0, rel=1e-4)
    assert j[0] == case.inj["tc_sample"]
    ctx.close()


def test_hour_pso_batch_grids_and_chunks_bitwise():
    """The benchmark's launch shape on the hour-long segment (a 320-point PSO
    batch): the same results bit for bit for other grids of all three passes
    and for a workspace of three evaluations (the batch then runs in 107
    chunks); the oracle checks sampled points, the rest must be finite with
    their samples in range."""
    require_gpu()
    case = Case("HLVK", HOUR, 2048.0, snr=10.0, cfg=33)
    rng = np.random.default_rng(33)
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    th = np.concatenate([synth.uniform_in_box(rng, 300, lo, hi), synth.near_point(rng, 20, case.theta0, lo, hi, 0.01)])
    plan = _plan_of(HOUR)
    ctx = make_ctx(case, 0, max_batch=len(th))
    upload(ctx, 0, case)
    f0, j0 = _eval(ctx, th)
    assert np.all(np.isfinite(f0)) and np.all((j0 >= 0) & (j0 < HOUR))
    ctx.select_plan(plan, 97, 333)
    upload(ctx, 0, case)
    f1, j1 = _eval(ctx, th)
    assert np.array_equal(f0, f1) and np.array_equal(j0, j1)
    ctx.close()
    slot = 2 * HOUR * 8
    ctx = make_ctx(case, 0, max_batch=len(th), workspace_bytes=3 * slot)
    upload(ctx, 0, case)
    f2, j2 = _eval(ctx, th)
    assert np.array_equal(f0, f2) and np.array_equal(j0, j2)
    ctx.close()
    idx = np.array([0, 150, 319])
    fo, jo = oracle_eval(case, th[idx])
    assert_parity(case, th[idx], f0[idx], j0[idx], fo, jo, 1e-4)


def test_hour_gradient_matches_oracle():
    """The fixed-sample adjoint on the hour-long segment (the gradient runs
    over the 3.5 million in-band bins, indices past 2^31 in k j*)."""
    require_gpu()
    case = Case("HLVK", HOUR, 2048.0, snr=12.0, cfg=34)
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    rng = np.random.default_rng(34)
    th = synth.near_point(rng, 3, case.theta0, lo, hi, 0.01)
    ctx = make_ctx(case, 0, max_batch=len(th))
    upload(ctx, 0, case)
    f, j, g = ctx.grad(torch.from_numpy(th).to(dev()), torch.zeros(len(th), dtype=torch.int32, device=dev()))
    f, j, g = f.cpu().numpy(), j.cpu().numpy(), g.cpu().numpy()
    w = np.array(hi) - np.array(lo)
    for k in range(len(th)):
        _, _, go = G.fitness_gradient(case.seg, case.net.pos_m, case.net.tensor, th[k], int(j[k]))
        scale = np.max(np.abs(go * w))
        assert np.all(np.abs((g[k] - go) * w) <= 2e-4 * scale), (k, g[k], go)
    ctx.close()


def test_mixed_lengths_with_a_three_pass_plan():
    """A 225-s segment (three passes) and a 64-s segment (two passes) in one
    batch, interleaved; the fused schedule runs the three-pass plan as separate
    launches and gives the same results as the two-pass schedule."""
    require_gpu()
    cases = [Case("HLV", 460800, 2048.0, snr=12.0, cfg=35, realization=0),
             Case("HLV", 131072, 2048.0, snr=12.0, cfg=35, realization=1)]
    rng = np.random.default_rng(35)
    ths, segs = [], []
    for i, c in enumerate(cases):
        t = thetas_for(c, rng, n_near=3, n_uniform=3, extras=False)
        ths.append(t)
        segs.append(np.full(len(t), i, dtype=np.int32))
    order = rng.permutation(sum(len(t) for t in ths))
    th = np.concatenate(ths)[order]
    sg = np.concatenate(segs)[order]
    out = []
    for schedule in (1, 0):
        ctx = make_ctx(cases[0], 0, max_batch=len(th), max_segments=2, max_samples=460800, schedule=schedule)
        for i, c in enumerate(cases):
            upload(ctx, i, c)
        f, j = ctx.eval(torch.from_numpy(th).to(dev()), torch.from_numpy(sg).to(dev()))
        out.append((f.cpu().numpy(), j.cpu().numpy()))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    f, j = out[0]
    for i, c in enumerate(cases):
        m = sg == i
        fo, jo = oracle_eval(c, th[m])
        assert_parity(c, th[m], f[m], j[m], fo, jo, 1e-4)
