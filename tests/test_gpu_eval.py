"""GPU parity of fitness_eval_batch against the FP64 oracle, through the C ABI.

Bars: mixed path (FP64 phase, FP32 data / FFT / projection) within 1e-4
relative in fitness; the FP64 path within 1e-9; argmax within one sample or an
equally good sample (near-tie rule).  Sizes span several tiles of every
plan, ragged segment mixes, chunked workspaces and the benchmark's full size.
"""
import numpy as np
import pytest
import torch

from oracle import fitness as F
from tests._cases import Case
from tests._gpu import assert_parity, dev, make_ctx, oracle_eval, require_gpu, thetas_for, upload

pytestmark = pytest.mark.gpu

SMALL = [  # (N, fs, detectors)
    (2048, 1024.0, "HL"), (4096, 2048.0, "HLV"), (8192, 1024.0, "HL"), (16384, 2048.0, "HLVK"),
    (32768, 2048.0, "L"), (24576, 2048.0, "HLV"), (49152, 2048.0, "HLVK"),
    # five and six detectors (a repeated site is a co-located pair with independent
    # noise): the kernels' run-time detector loop
    (16384, 2048.0, "HLVKH"), (8192, 1024.0, "HLVKHL"),
]


@pytest.mark.parametrize("prec", [0, 1], ids=["mixed", "fp64"])
@pytest.mark.parametrize("n,fs,names", SMALL, ids=[f"N{n}-{d}" for n, _, d in SMALL])
def test_eval_matches_oracle(n, fs, names, prec):
    require_gpu()
    case = Case(names, n, fs, snr=12.0, cfg=10, realization=n)
    rng = np.random.default_rng(n + prec)
    th = thetas_for(case, rng)
    ctx = make_ctx(case, prec, max_batch=len(th))
    upload(ctx, 0, case)
    f, j = ctx.eval(torch.from_numpy(th).to(dev()), torch.zeros(len(th), dtype=torch.int32, device=dev()))
    f, j = f.cpu().numpy(), j.cpu().numpy()
    fo, jo = oracle_eval(case, th)
    assert_parity(case, th, f, j, fo, jo, 1e-4 if prec == 0 else 1e-9)
    assert np.isnan(th[-3, 0]) and f[-3] == -np.inf and j[-3] == -1
    ctx.close()


@pytest.mark.parametrize("n,names,batch,n_check", [(131072, "HLVK", 320, None), (8192, "HL", 40, None),
                                                   (262144, "HLVK", 16, 3), (196608, "HLVK", 16, 3)],
                         ids=["N131072-cfg2", "N8192-cfg1", "N262144", "N196608"])
def test_eval_full_size_sampled(n, names, batch, n_check):
    """Full benchmark sizes and launch shape: the 320-point batch of the 64-s
    search and the 40-point batch of the 8-s search are checked point by point
    against the oracle, the longer segments on a sample of points."""
    require_gpu()
    fs = 1024.0 if n == 8192 else 2048.0
    case = Case(names, n, fs, snr=10.0, cfg=2, realization=0)
    rng = np.random.default_rng(7)
    th = thetas_for(case, rng, n_near=batch // 2, n_uniform=batch - batch // 2, extras=False)
    ctx = make_ctx(case, 0, max_batch=batch)
    upload(ctx, 0, case)
    f, j = ctx.eval(torch.from_numpy(th).to(dev()), torch.zeros(batch, dtype=torch.int32, device=dev()))
    f, j = f.cpu().numpy(), j.cpu().numpy()
    idx = np.arange(batch) if n_check is None else \
        np.unique(np.concatenate([[0, batch - 1], rng.choice(batch, n_check, replace=False)]))
    fo, jo = oracle_eval(case, th[idx])
    assert_parity(case, th[idx], f[idx], j[idx], fo, jo, 1e-4)
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 1e-10)], ids=["mixed", "fp64"])
def test_noiseless_identity_on_gpu(prec, tol):
    """Gamma^2 at the true parameters of a noiseless signal equals SNR^2 and the
    maximum sits on the injected coalescence sample."""
    require_gpu()
    case = Case("HLVK", 16384, 2048.0, snr=11.0, noise=False, cfg=11)
    ctx = make_ctx(case, prec, max_batch=1)
    upload(ctx, 0, case)
    f, j = ctx.eval(torch.from_numpy(case.theta0[None, :].copy()).to(dev()),
                    torch.zeros(1, dtype=torch.int32, device=dev()))
    assert f.item() == pytest.approx(121.0, rel=tol)
    assert j.item() == case.inj["tc_sample"]
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["mixed", "fp64"])
def test_detector_specific_noise_curves(prec):
    """Every detector with its own noise curve (knee, level, spectral lines:
    its own sigma_i and over-whitening): parity with the oracle on a batch with
    near, uniform, corner and outside points, and the noiseless identity
    Gamma^2(theta_0) = SNR^2 on the injected sample."""
    require_gpu()
    case = Case("HLVK", 16384, 2048.0, snr=12.0, cfg=16, psd="network")
    rng = np.random.default_rng(160 + prec)
    th = thetas_for(case, rng)
    ctx = make_ctx(case, prec, max_batch=len(th))
    upload(ctx, 0, case)
    f, j = ctx.eval(torch.from_numpy(th).to(dev()), torch.zeros(len(th), dtype=torch.int32, device=dev()))
    f, j = f.cpu().numpy(), j.cpu().numpy()
    fo, jo = oracle_eval(case, th)
    assert_parity(case, th, f, j, fo, jo, 1e-4 if prec == 0 else 1e-9)
    ctx.close()
    clean = Case("HLV", 16384, 2048.0, snr=11.0, noise=False, cfg=17, psd="network")
    ctx = make_ctx(clean, prec, max_batch=1)
    upload(ctx, 0, clean)
    f, j = ctx.eval(torch.from_numpy(clean.theta0[None, :].copy()).to(dev()),
                    torch.zeros(1, dtype=torch.int32, device=dev()))
    assert f.item() == pytest.approx(121.0, rel=1e-4 if prec == 0 else 1e-10)
    assert j.item() == clean.inj["tc_sample"]
    ctx.close()


def test_ragged_segments_in_one_call():
    """Segments of different lengths (different FFT plans) interleaved in one batch."""
    require_gpu()
    cases = [Case("HLV", n, 2048.0, snr=12.0, cfg=12, realization=i) for i, n in enumerate((8192, 24576, 16384))]
    rng = np.random.default_rng(3)
    ths, segs = [], []
    for i, c in enumerate(cases):
        t = thetas_for(c, rng, n_near=4, n_uniform=4, extras=False)
        ths.append(t)
        segs.append(np.full(len(t), i, dtype=np.int32))
    order = rng.permutation(sum(len(t) for t in ths))
    th = np.concatenate(ths)[order]
    sg = np.concatenate(segs)[order]
    ctx = make_ctx(cases[0], 0, max_batch=len(th), max_segments=3, max_samples=24576)
    for i, c in enumerate(cases):
        upload(ctx, i, c)
    f, j = ctx.eval(torch.from_numpy(th).to(dev()), torch.from_numpy(sg).to(dev()))
    f, j = f.cpu().numpy(), j.cpu().numpy()
    for i, c in enumerate(cases):
        m = sg == i
        fo, jo = oracle_eval(c, th[m])
        assert_parity(c, th[m], f[m], j[m], fo, jo, 1e-4)
    ctx.close()


@pytest.mark.parametrize("plan", [7, 16, 20, 31, 35, 36, 6, 12, 13, 14, 15, 24, 30, 34, 11, 18, 21, 33, 5, 17, 22,
                                  23, 32])
def test_eval_plans_sampled(plan):
    """Every plan of the 32-s to 128-s segments (65536 to 262144 samples:
    column lengths 128 to 512, 8- and 16-element threads, 256- to 1024-thread
    work-groups, rows in one or two wavefronts) matches the oracle on sampled
    points of a 16-point batch."""
    require_gpu()
    from paper_2002_02150_amd.fcas import plans
    n = dict(plans())[plan]["n"]
    assert n in (65536, 131072, 196608, 262144)
    case = Case("HLVK", n, 2048.0, snr=10.0, cfg=2, realization=plan)
    rng = np.random.default_rng(plan)
    th = thetas_for(case, rng, n_near=8, n_uniform=8, extras=False)
    ctx = make_ctx(case, 0, max_batch=len(th))
    ctx.select_plan(plan)
    upload(ctx, 0, case)
    f, j = ctx.eval(torch.from_numpy(th).to(dev()), torch.zeros(len(th), dtype=torch.int32, device=dev()))
    f, j = f.cpu().numpy(), j.cpu().numpy()
    idx = np.array([0, len(th) - 1])
    fo, jo = oracle_eval(case, th[idx])
    assert_parity(case, th[idx], f[idx], j[idx], fo, jo, 1e-4)
    ctx.close()


def test_results_do_not_depend_on_grid_or_batch():
    """A point's fitness and sample are bitwise the same whichever work-group
    evaluates it, how many work items each work-group takes (grids from one
    item per work-group to dozens), and in which batch: a batch of one
    repeated point gives one value, and every point of a random batch gets the
    value it gets when evaluated alone."""
    require_gpu()
    case = Case("HLVK", 32768, 2048.0, snr=12.0, cfg=20)
    rng = np.random.default_rng(31)
    th1 = thetas_for(case, rng, n_near=20, n_uniform=20, extras=False)
    rep = np.tile(th1[:1], (48, 1))
    ctx = make_ctx(case, 0, max_batch=len(th1) + len(rep), max_segments=1)
    from paper_2002_02150_amd.fcas import plans
    plan = next(p for p, d in plans() if d["n"] == 32768)
    results = []
    for g1, g2 in [(0, 0), (7, 5), (64, 64), (4096, 4096)]:
        ctx.select_plan(plan, g1, g2)
        upload(ctx, 0, case)
        for th in (th1, rep):
            t = torch.from_numpy(th).to(dev())
            f, j = ctx.eval(t, torch.zeros(len(th), dtype=torch.int32, device=dev()))
            results.append((f.cpu().numpy(), j.cpu().numpy()))
        f_rep = results[-1][0]
        assert np.all(f_rep == f_rep[0]) and np.all(results[-1][1] == results[-1][1][0])
    for (fa, ja), (fb, jb) in zip(results[0::2], results[2::2]):
        assert np.array_equal(fa, fb) and np.array_equal(ja, jb)
    singles = [ctx.eval(torch.from_numpy(th1[k:k + 1]).to(dev()),
                        torch.zeros(1, dtype=torch.int32, device=dev()))[0].item() for k in range(0, len(th1), 7)]
    assert np.array_equal(np.array(singles), results[-2][0][::7])
    ctx.close()


def test_chunked_workspace_is_bitwise_identical_and_repeatable():
    """Two-pass schedule: a workspace of three evaluations forces chunking;
    results equal the one-chunk run bit for bit, and repeated calls are bitwise
    identical."""
    require_gpu()
    case = Case("HLVK", 16384, 2048.0, snr=12.0, cfg=13)
    rng = np.random.default_rng(4)
    th = torch.from_numpy(thetas_for(case, rng)).to(dev())
    seg = torch.zeros(th.shape[0], dtype=torch.int32, device=dev())
    big = make_ctx(case, 0, max_batch=th.shape[0], schedule=1)
    small = make_ctx(case, 0, max_batch=th.shape[0], workspace_bytes=3 * 2 * 16384 * 8, schedule=1)
    upload(big, 0, case)
    upload(small, 0, case)
    f1, j1 = big.eval(th, seg)
    f2, j2 = small.eval(th, seg)
    f3, j3 = big.eval(th, seg)
    assert torch.equal(f1, f2) and torch.equal(j1, j2)
    assert torch.equal(f1, f3) and torch.equal(j1, j3)
    big.close()
    small.close()


@pytest.mark.parametrize("ws_slots", [0, 2, 1], ids=["default-workspace", "two-slots", "one-slot"])
def test_fused_schedule_equals_two_pass(ws_slots):
    """The fused persistent schedule (pipelined passes in one launch, slot
    reuse through device-scope release/acquire counters) gives the results of
    the two-pass schedule bit for bit on a ragged batch of several segments,
    also when the workspace holds only one or two evaluations, and never trips
    its wait bound; repeated calls are bit-identical."""
    require_gpu()
    cases = [Case("HLVK", n, 2048.0, snr=12.0, cfg=16, realization=i) for i, n in enumerate((16384, 24576, 8192))]
    rng = np.random.default_rng(17)
    ths, segs = [], []
    for i, c in enumerate(cases):
        t = thetas_for(c, rng, n_near=30, n_uniform=30)
        ths.append(t)
        segs.append(np.full(len(t), i, dtype=np.int32))
    order = rng.permutation(sum(len(t) for t in ths))
    th = torch.from_numpy(np.concatenate(ths)[order]).to(dev())
    sg = torch.from_numpy(np.concatenate(segs)[order]).to(dev())
    wsb = ws_slots * 2 * 24576 * 8
    fused = make_ctx(cases[0], 0, max_batch=th.shape[0], max_segments=3, max_samples=24576, workspace_bytes=wsb,
                     schedule=0)
    two = make_ctx(cases[0], 0, max_batch=th.shape[0], max_segments=3, max_samples=24576, schedule=1)
    for i, c in enumerate(cases):
        upload(fused, i, c)
        upload(two, i, c)
    f1, j1 = fused.eval(th, sg)
    f2, j2 = two.eval(th, sg)
    f3, j3 = fused.eval(th, sg)
    assert fused.device_error() == 0
    assert torch.equal(f1, f2) and torch.equal(j1, j2)
    assert torch.equal(f1, f3) and torch.equal(j1, j3)
    fused.close()
    two.close()


def test_unregistered_segment_and_batch_limits():
    require_gpu()
    from paper_2002_02150_amd import FcasError
    case = Case("HL", 4096, 2048.0, snr=10.0, cfg=14)
    ctx = make_ctx(case, 0, max_batch=4, max_segments=2)
    upload(ctx, 0, case)
    th = torch.from_numpy(np.tile(case.theta0, (4, 1))).to(dev())
    seg = torch.tensor([0, 1, 5, -1], dtype=torch.int32, device=dev())
    f, j = ctx.eval(th, seg)
    f, j = f.cpu().numpy(), j.cpu().numpy()
    assert np.isfinite(f[0]) and j[0] >= 0
    assert np.all(np.isnan(f[1:])) and np.all(j[1:] == -2)
    assert ctx.device_error() == 1
    assert ctx.device_error() == 0
    # empty batch is a no-op; more than max_batch is refused on the host
    e = torch.empty(0, 4, dtype=torch.float64, device=dev())
    ctx.eval(e, torch.empty(0, dtype=torch.int32, device=dev()))
    with pytest.raises(FcasError) as ei:
        ctx.eval(torch.zeros(5, 4, dtype=torch.float64, device=dev()), torch.zeros(5, dtype=torch.int32, device=dev()))
    assert ei.value.code == -6
    with pytest.raises(FcasError):
        ctx.set_segment(2, torch.zeros(2, 2049, dtype=torch.complex128, device=dev()),
                        torch.ones(2, 2049, dtype=torch.float64, device=dev()))
    ctx.close()


@pytest.mark.parametrize("psd", ["same", "network"])
def test_library_injection_matches_oracle_signal_model(psd):
    """fcas_inject (the benchmark's signal generator) reproduces the oracle's
    injection, amplitude normalisation included (network SNR over detectors
    with one noise curve or a curve each)."""
    require_gpu()
    import synth
    from oracle import signal as S
    case = Case("HLVK", 16384, 2048.0, snr=None, noise=False, cfg=15, psd=psd)
    ctx = make_ctx(case, 0, max_batch=1)
    th0 = np.array([2.1, -0.7, 40.0, 1.3])
    prm = dict(psi=0.4, phi_c=1.9, cos_iota=-0.3, tc_sample=5000)
    ref = S.injection(case.n_samples, case.fs, 30.0, 1000.0, case.net.pos_m, case.net.tensor, case.psd, th0,
                      prm["psi"], prm["phi_c"], prm["cos_iota"], prm["tc_sample"], snr=9.0)
    xf = torch.zeros(4, case.n_samples // 2 + 1, dtype=torch.complex128, device=dev())
    psd = torch.from_numpy(np.ascontiguousarray(case.psd)).to(dev())
    ctx.inject(xf, psd, *th0, prm["psi"], prm["phi_c"], prm["cos_iota"], prm["tc_sample"] / case.fs, 9.0)
    got = xf.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))
    ctx.close()


def test_coalescence_range_restriction():
    """fcas_set_segment_range limits the maximum over t_c to j_lo <= j < j_hi;
    the GPU follows the oracle with the same restriction, bad ranges are refused."""
    require_gpu()
    from paper_2002_02150_amd import FcasError
    case = Case("HLVK", 16384, 2048.0, snr=12.0, cfg=17)
    rng = np.random.default_rng(8)
    th = thetas_for(case, rng, n_near=8, n_uniform=8, extras=False)
    ctx = make_ctx(case, 0, max_batch=len(th), max_segments=2)
    upload(ctx, 0, case)
    t = torch.from_numpy(th).to(dev())
    seg = torch.zeros(len(th), dtype=torch.int32, device=dev())
    tc = case.inj["tc_sample"]
    for lo, hi in ((4096, 12288), (0, 1), (16383, 16384), (max(tc - 5, 0), min(tc + 6, 16384))):
        ctx.set_segment_range(0, lo, hi)
        f, j = ctx.eval(t, seg)
        f, j = f.cpu().numpy(), j.cpu().numpy()
        assert np.all((j >= lo) & (j < hi))
        fo, jo = oracle_eval_range(case, th, (lo, hi))
        assert_parity(case, th, f, j, fo, jo, 1e-4)
    for bad in ((-1, 10), (10, 10), (0, 16385)):
        with pytest.raises(FcasError):
            ctx.set_segment_range(0, *bad)
    with pytest.raises(FcasError):
        ctx.set_segment_range(1, 0, 10)   # not registered
    ctx.close()


def oracle_eval_range(case, thetas, j_range):
    import synth
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    return F.fitness_batch(case.seg, case.net.pos_m, case.net.tensor, thetas, np.array(lo), np.array(hi), j_range)
