"""GPU parity of the hot path against the FP64 oracle at the sizes and launch
shapes of the benchmark workloads, through the C ABI: every point of every
batch is checked.

  * the FP64 context at 131072 samples (the plain FP64 path whose rate is the
    denominator of the benchmark's speed-up), 1e-9 relative;
  * the mixed path at 65536 samples through the autotuned plan (the 32-s
    segments of the ragged workload);
  * one ragged call over the four segment lengths of the ragged workload
    (32, 64, 96 and 128 s at 2048 Hz) with the autotuned plans;
  * the fixed-sample gradient at 131072 samples for 16 points within 1% of the
    rectangle width of a source, with a bar on every component that is not
    negligible next to the largest;
  * re-registration of a segment that fails leaves the id unregistered.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import gradient as G
from tests._cases import Case
from tests._gpu import assert_parity, dev, make_ctx, oracle_eval, require_gpu, thetas_for, upload

pytestmark = pytest.mark.gpu

CONFIG3_LENGTHS = (65536, 131072, 196608, 262144)


def _eval(ctx, th, seg):
    f, j = ctx.eval(torch.from_numpy(np.ascontiguousarray(th)).to(dev()), torch.from_numpy(seg).to(dev()))
    return f.cpu().numpy(), j.cpu().numpy()


def test_fp64_context_131072_every_point():
    """The FP64 instantiation at 4 x 131072 samples (its default plan: the
    autotuner's choices apply to mixed contexts only): 24 points near the
    source and uniform in the rectangle, two corners and three points outside
    it, all within 1e-9 of the oracle."""
    require_gpu()
    from paper_2002_02150_amd.fcas import load_tuning
    case = Case("HLVK", 131072, 2048.0, snr=10.0, cfg=2, realization=0)
    rng = np.random.default_rng(131)
    th = thetas_for(case, rng, n_near=12, n_uniform=12)
    ctx = make_ctx(case, 1, max_batch=len(th))
    upload(ctx, 0, case)
    f, j = _eval(ctx, th, np.zeros(len(th), dtype=np.int32))
    fo, jo = oracle_eval(case, th)
    assert_parity(case, th, f, j, fo, jo, 1e-9)
    rel = np.abs(f - fo)[np.isfinite(fo)] / fo[np.isfinite(fo)]
    print(f"fp64 131072: max rel err {rel.max():.3e} over {len(rel)} points")
    assert 131072 in load_tuning()   # the mixed contexts of the same length take another plan
    ctx.close()


def test_mixed_65536_tuned_plan_every_point():
    """4 x 65536 samples (32 s at 2048 Hz) through the plan the autotuner
    chose for that length, every point of the batch checked."""
    require_gpu()
    from paper_2002_02150_amd.fcas import load_tuning, plans
    tuned = load_tuning()[65536]["plan"]
    assert dict(plans())[tuned]["n"] == 65536
    case = Case("HLVK", 65536, 2048.0, snr=11.0, cfg=3, realization=65)
    rng = np.random.default_rng(65)
    th = thetas_for(case, rng, n_near=16, n_uniform=16)
    ctx = make_ctx(case, 0, max_batch=len(th))
    upload(ctx, 0, case)
    f, j = _eval(ctx, th, np.zeros(len(th), dtype=np.int32))
    fo, jo = oracle_eval(case, th)
    assert_parity(case, th, f, j, fo, jo, 1e-4)
    ctx.close()


def test_ragged_config3_lengths_one_call():
    """Segments of 32, 64, 96 and 128 s (65536 to 262144 samples, four plans,
    the tuned grids) interleaved at random in one call, injections at SNR
    U[8, 14] in every other segment as in the ragged workload; every point
    (near the source, uniform, corners, outside) matches the oracle."""
    require_gpu()
    rng = np.random.default_rng(2003)
    cases = []
    for i, n in enumerate(CONFIG3_LENGTHS):
        snr = float(rng.uniform(8.0, 14.0)) if i % 2 == 0 else None
        cases.append(Case("HLVK", n, 2048.0, snr=snr, cfg=3, realization=100 + i))
    ths, segs = [], []
    for i, c in enumerate(cases):
        t = thetas_for(c, rng, n_near=6 if c.theta0 is not None else 0, n_uniform=8)
        ths.append(t)
        segs.append(np.full(len(t), i, dtype=np.int32))
    order = rng.permutation(sum(len(t) for t in ths))
    th = np.concatenate(ths)[order]
    sg = np.concatenate(segs)[order]
    ctx = make_ctx(cases[0], 0, max_batch=len(th), max_segments=len(cases), max_samples=max(CONFIG3_LENGTHS))
    for i, c in enumerate(cases):
        upload(ctx, i, c)
    f, j = _eval(ctx, th, sg)
    for i, c in enumerate(cases):
        m = sg == i
        fo, jo = oracle_eval(c, th[m])
        assert_parity(c, th[m], f[m], j[m], fo, jo, 1e-4)
    ctx.close()


@pytest.mark.parametrize("prec,rtol,atol", [(0, 1e-4, 1e-5), (1, 1e-9, 1e-9)], ids=["mixed", "fp64"])
def test_gradient_131072_per_component(prec, rtol, atol):
    """dGamma^2/dtheta at 4 x 131072 samples for 16 points within 1% of the
    rectangle width of an SNR-12 source, against the oracle's analytic
    gradient at the GPU's maximising sample.  With w the rectangle widths and
    s = max_q |g_q w_q|, every component satisfies |dg_q w_q| <= atol s, and
    every component with |g_q w_q| > 1e-3 s is also within rtol of itself.

    Mixed path: the sums over the 62,080 bins are FP32, an error of a few
    1e-7 of the sum of the terms' magnitudes; measured 4.9e-7 of s at worst
    and 1.7e-6 of a component (FP64: 4.4e-11), so the bars hold the measured
    errors with a margin of 20 or more."""
    require_gpu()
    case = Case("HLVK", 131072, 2048.0, snr=12.0, cfg=4, realization=0)
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    rng = np.random.default_rng(404)
    th = synth.near_point(rng, 16, case.theta0, lo, hi, 0.01)
    ctx = make_ctx(case, prec, max_batch=len(th))
    upload(ctx, 0, case)
    f, j, g = ctx.grad(torch.from_numpy(th).to(dev()), torch.zeros(len(th), dtype=torch.int32, device=dev()))
    f, j, g = f.cpu().numpy(), j.cpu().numpy(), g.cpu().numpy()
    w = np.array(hi) - np.array(lo)
    worst_abs, worst_rel, checked = 0.0, 0.0, 0
    for k in range(len(th)):
        g2, _, go = G.fitness_gradient(case.seg, case.net.pos_m, case.net.tensor, th[k], int(j[k]))
        assert f[k] == pytest.approx(g2, rel=1e-4 if prec == 0 else 1e-9)
        gw, gow = g[k] * w, go * w
        s = np.max(np.abs(gow))
        err = np.abs(gw - gow)
        assert np.all(err <= atol * s), (k, g[k], go)
        big = np.abs(gow) > 1e-3 * s
        assert np.all(err[big] <= rtol * np.abs(gow[big])), (k, g[k], go)
        worst_abs = max(worst_abs, float(np.max(err) / s))
        worst_rel = max(worst_rel, float(np.max(err[big] / np.abs(gow[big]))))
        checked += int(big.sum())
    print(f"gradient 131072 prec={prec}: max |dg w|/s {worst_abs:.3e}, max per-component rel {worst_rel:.3e} "
          f"({checked} components)")
    ctx.close()


def test_failed_reregistration_leaves_segment_unregistered():
    """Re-registering a segment with a PSD that is zero in band fails with
    FCAS_EINVAL; the id is then unregistered (NaN, -2, device error flag),
    and a later valid registration works again."""
    require_gpu()
    from paper_2002_02150_amd import FcasError
    case = Case("HLV", 8192, 2048.0, snr=12.0, cfg=40)
    ctx = make_ctx(case, 0, max_batch=4)
    upload(ctx, 0, case)
    th = torch.from_numpy(np.tile(case.theta0, (4, 1))).to(dev())
    seg = torch.zeros(4, dtype=torch.int32, device=dev())
    f_ok, j_ok = ctx.eval(th, seg)
    f_ok, j_ok = f_ok.cpu().numpy().copy(), j_ok.cpu().numpy().copy()
    assert np.all(np.isfinite(f_ok))
    bad_psd = case.psd.copy()
    bad_psd[:, 1000] = 0.0                        # in band (bin 1000 = 250 Hz)
    with pytest.raises(FcasError) as ei:
        ctx.set_segment(0, torch.from_numpy(np.ascontiguousarray(case.xf)).to(dev()),
                        torch.from_numpy(np.ascontiguousarray(bad_psd)).to(dev()))
    assert ei.value.code == -1
    f, j = ctx.eval(th, seg)
    assert np.all(np.isnan(f.cpu().numpy())) and np.all(j.cpu().numpy() == -2)
    assert ctx.device_error() == 1
    upload(ctx, 0, case)
    f, j = ctx.eval(th, seg)
    assert np.array_equal(f.cpu().numpy(), f_ok) and np.array_equal(j.cpu().numpy(), j_ok)
    assert ctx.device_error() == 0
    ctx.close()
