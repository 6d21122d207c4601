"""Helpers for the GPU tests: contexts built from the seeded test cases."""
import numpy as np
import pytest
import torch

import synth
from oracle import fitness as F


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_02150_amd import fcas
    fcas.library()   # raises if the HIP library is missing: no silent fallback


def dev():
    return torch.device("cuda", 0)


def make_ctx(case, precision=0, max_batch=64, max_segments=1, max_samples=None, workspace_bytes=0, schedule=1):
    from paper_2002_02150_amd import Context
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    return Context.from_network(case.net, fs=case.fs, f_low=case.f_low, f_high=case.f_high, box_lo=lo, box_hi=hi,
                                precision=precision, max_batch=max_batch, max_segments=max_segments,
                                max_samples=max_samples or case.n_samples, workspace_bytes=workspace_bytes,
                                schedule=schedule)


def upload(ctx, seg_id, case):
    ctx.set_segment(seg_id, torch.from_numpy(np.ascontiguousarray(case.xf)).to(dev()),
                    torch.from_numpy(np.ascontiguousarray(case.psd)).to(dev()))


def thetas_for(case, rng, n_near=8, n_uniform=12, extras=True):
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    pts = [synth.uniform_in_box(rng, n_uniform, lo, hi)]
    if case.theta0 is not None and n_near:
        pts.append(synth.near_point(rng, n_near, case.theta0, lo, hi, 0.01))
    th = np.concatenate(pts)
    if extras:
        out = np.array([[7.0, 0.1, 40.0, 1.2],                       # alpha outside
                        [1.0, 0.1, 10.0, 1.2],                        # tau0 outside
                        [np.nan, 0.1, 40.0, 1.2],                     # non-finite
                        list(lo),                                     # corner: inside
                        list(hi)])                                    # corner: inside
        th = np.concatenate([th, out])
    return th


def oracle_eval(case, thetas):
    lo, hi = synth.SEARCH_BOX_30HZ_LO, synth.SEARCH_BOX_30HZ_HI
    return F.fitness_batch(case.seg, case.net.pos_m, case.net.tensor, thetas, np.array(lo), np.array(hi))


def assert_parity(case, thetas, f_gpu, j_gpu, f_ora, j_ora, rtol):
    """Fitness within rtol relative; argmax equal within one sample, or (several
    results correct) the oracle's series at the GPU's sample within 1e-4 of its
    maximum; out-of-box points give (-inf, -1) on both sides."""
    for k in range(len(thetas)):
        if not np.isfinite(f_ora[k]):
            assert f_gpu[k] == -np.inf and j_gpu[k] == -1, (k, f_gpu[k], j_gpu[k])
            continue
        assert abs(f_gpu[k] - f_ora[k]) <= rtol * f_ora[k], (k, f_gpu[k], f_ora[k])
        dj = abs(int(j_gpu[k]) - int(j_ora[k]))
        dj = min(dj, case.n_samples - dj)
        if dj > 1:
            g_at = F.gamma2_at(case.seg, case.net.pos_m, case.net.tensor, thetas[k], int(j_gpu[k]))
            assert g_at >= (1 - 1e-4) * f_ora[k], (k, j_gpu[k], j_ora[k], g_at, f_ora[k])
