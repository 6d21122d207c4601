"""fitness_eval_batch_static (the entry point whose scratch memory is the
library's static per-GPU array) against fitness_eval_batch, through the C ABI:
bitwise equal results on two calls in a row, the second with a smaller batch
on other segments, a graph-captured replay, and the capacity error."""
import numpy as np
import pytest
import torch

from tests._cases import Case
from tests._gpu import assert_parity, dev, make_ctx, oracle_eval, require_gpu, thetas_for, upload

pytestmark = pytest.mark.gpu


def _pair(ctx, th, sg):
    t = torch.from_numpy(np.ascontiguousarray(th)).to(dev())
    s = torch.from_numpy(np.ascontiguousarray(sg)).to(dev())
    f_ref, j_ref = ctx.eval(t, s)
    f = torch.full((len(th),), 7.0, dtype=torch.float64, device=dev())
    j = torch.full((len(th),), 7, dtype=torch.int32, device=dev())
    ctx.eval_static(t, s, f, j)
    return f_ref.cpu().numpy(), j_ref.cpu().numpy(), f.cpu().numpy(), j.cpu().numpy()


def test_static_scratch_entry_point_equals_eval():
    require_gpu()
    from paper_2002_02150_amd import FcasError
    rng = np.random.default_rng(77)
    cases = [Case("HLVK", n, 2048.0, snr=12.0, cfg=50, realization=i)
             for i, n in enumerate((131072, 16384, 262144))]
    ctx = make_ctx(cases[0], 0, max_batch=96, max_segments=3, max_samples=262144)
    for i, c in enumerate(cases):
        upload(ctx, i, c)
    # first call: 90 points over the three segments (the 262144-sample segment
    # leaves room for few workspace slots: the call runs in chunks)
    ths, sgs = [], []
    for i, c in enumerate(cases):
        t = thetas_for(c, rng, n_near=12, n_uniform=13)
        ths.append(t)
        sgs.append(np.full(len(t), i, dtype=np.int32))
    th = np.concatenate(ths)
    sg = np.concatenate(sgs)
    order = rng.permutation(len(th))
    th, sg = th[order], sg[order]
    fr, jr, fs, js = _pair(ctx, th, sg)
    assert np.array_equal(fr, fs, equal_nan=True) and np.array_equal(jr, js)
    for i, c in enumerate(cases):
        m = sg == i
        fo, jo = oracle_eval(c, th[m])
        assert_parity(c, th[m], fs[m], js[m], fo, jo, 1e-4)
    # second call, smaller: 11 points on one segment, the scratch still holding
    # the first call's contents
    th2 = thetas_for(cases[1], rng, n_near=3, n_uniform=3)
    sg2 = np.full(len(th2), 1, dtype=np.int32)
    fr2, jr2, fs2, js2 = _pair(ctx, th2, sg2)
    assert np.array_equal(fr2, fs2, equal_nan=True) and np.array_equal(jr2, js2)
    fo, jo = oracle_eval(cases[1], th2)
    assert_parity(cases[1], th2, fs2, js2, fo, jo, 1e-4)
    # captured in a HIP graph and replayed, with eager work in between
    t = torch.from_numpy(th2).to(dev())
    s = torch.from_numpy(sg2).to(dev())
    f = torch.empty(len(th2), dtype=torch.float64, device=dev())
    j = torch.empty(len(th2), dtype=torch.int32, device=dev())
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        ctx.eval_static(t, s, f, j)
    torch.cuda.current_stream().wait_stream(st)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.eval_static(t, s, f, j)
    for _ in range(3):
        f.fill_(0.0)
        j.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(f.cpu().numpy(), fr2, equal_nan=True) and np.array_equal(j.cpu().numpy(), jr2)
        _pair(ctx, th, sg)   # eager calls of both entry points between replays
    # beyond the scratch: the tables of the points alone exceed it
    small = Case("HL", 2048, 1024.0, snr=None, cfg=51)
    big = make_ctx(small, 0, max_batch=1 << 17, workspace_bytes=1 << 20)
    upload(big, 0, small)
    n = 1 << 17
    with pytest.raises(FcasError) as ei:
        big.eval_static(torch.zeros(n, 4, dtype=torch.float64, device=dev()), torch.zeros(n, dtype=torch.int32, device=dev()),
                        torch.empty(n, dtype=torch.float64, device=dev()), torch.empty(n, dtype=torch.int32, device=dev()))
    assert ei.value.code == -6
    assert ctx.device_error() == 0
    big.close()
    ctx.close()
