"""CPU emulation of the HIP fitness path (its tile, stage and reduction
functions driven thread by thread, built with the host address sanitizer)
against the FP64 oracle.  This checks the four-step index arithmetic of every
FFT plan, the prologue and the max reduction on the CPU, before any GPU run."""
import math
import os
import subprocess

import numpy as np
import pytest

from oracle import fitness as F
from tests._cases import Case

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "emu", "fcas_emu.cpp")
CSRC = os.path.join(ROOT, "paper_2002_02150_amd", "csrc")
BIN = os.path.join(ROOT, "tests", "emu", "_build", "fcas_emu")

# plan index -> N, mirrors the plan list of the library
PLANS = {0: 2048, 1: 4096, 2: 8192, 3: 16384, 4: 32768, 5: 65536, 6: 131072, 7: 262144,
         8: 24576, 9: 49152, 10: 98304, 11: 196608,
         12: 131072, 13: 131072, 14: 131072, 15: 131072, 16: 262144, 17: 65536, 18: 196608, 19: 8192,
         20: 262144, 21: 196608, 22: 65536, 23: 65536, 24: 131072, 25: 460800, 26: 3686400, 27: 7372800, 28: 7372800, 29: 3686400,
         30: 131072, 31: 262144, 32: 65536, 33: 196608, 34: 131072, 35: 262144, 36: 262144}


@pytest.fixture(scope="module")
def emu():
    deps = [SRC] + [os.path.join(CSRC, f) for f in ("fft_core.hpp", "fitness_tiles.hpp", "plans.hpp")]
    if not os.path.exists(BIN) or os.path.getmtime(BIN) < max(os.path.getmtime(d) for d in deps):
        os.makedirs(os.path.dirname(BIN), exist_ok=True)
        # -O0: the optimiser takes minutes over every plan instantiation, the runs take seconds either way
        # built under a private name and renamed, so that parallel test workers never run a half-written binary
        tmp = f"{BIN}.{os.getpid()}"
        subprocess.run(["g++", "-std=c++17", "-O0", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                        "-I" + CSRC, SRC, "-o", tmp], check=True)
        os.replace(tmp, BIN)
    return BIN


def _run(emu, tmp_path, case, theta, plan, prec):
    seg = case.seg
    D = case.net.n_det
    pre = str(tmp_path / "in")
    case.net.pos_m.astype(np.float64).tofile(pre + ".pos")
    case.net.tensor.reshape(D, 9).astype(np.float64).tofile(pre + ".ten")
    seg.sigma.astype(np.float64).tofile(pre + ".sigma")
    (case.f_low / seg.freqs).__pow__(1.0 / 3.0).astype(np.float64).tofile(pre + ".b")
    np.asarray(theta, dtype=np.float64).tofile(pre + ".theta")
    yt = np.ascontiguousarray(seg.y.T).astype(np.complex64 if prec == 0 else np.complex128)
    yt.tofile(pre + ".y")
    out = str(tmp_path / "out")
    subprocess.run([emu, str(prec), str(plan), str(D), str(seg.k_lo), str(seg.k_hi), repr(seg.df),
                    repr(case.f_low), pre, out], check=True)
    r = np.fromfile(out, dtype=np.float64)
    return r[:-2], r[-2], int(r[-1])


@pytest.mark.parametrize("plan,names,prec", [
    (0, "HL", 0), (1, "HLV", 0), (2, "HL", 0), (3, "HLVK", 0), (5, "HLVK", 0), (6, "HLVK", 0),
    (8, "HLV", 0), (7, "HLVK", 0), (2, "HLVK", 1), (8, "HL", 1), (4, "L", 0), (9, "HLVK", 0),
    (12, "HLVK", 0), (13, "HLVK", 0), (14, "HLVK", 0), (15, "HLVK", 0), (16, "HLVK", 0), (17, "HLV", 0),
    (18, "HLVK", 0), (19, "HL", 0), (12, "HLVK", 1), (18, "HL", 1), (20, "HLVK", 0), (20, "HL", 1),
    (21, "HLVK", 0), (22, "HLV", 0), (23, "HLVK", 0), (24, "HLVK", 0), (21, "HL", 1), (24, "HL", 1),
    (25, "HLVK", 0), (25, "HL", 1), (27, "HLVK", 0), (29, "HL", 1),
    (30, "HLVK", 0), (30, "HL", 1), (31, "HLVK", 0), (32, "HLVK", 0), (33, "HLVK", 0), (34, "HLVK", 0),
    (35, "HLVK", 0), (36, "HLVK", 0), (36, "HL", 1),
    # five and six detectors (a site repeated: a co-located pair with its own
    # noise) take the kernels' run-time detector loop
    (6, "HLVKH", 0), (25, "HLVKHL", 0), (2, "HLVKHL", 1),
])
def test_emulated_path_matches_oracle(emu, tmp_path, plan, names, prec):
    n = PLANS[plan]
    fs = 1024.0 if n in (2048, 8192) else 2048.0
    case = Case(names, n, fs, snr=12.0, cfg=50, realization=plan)
    theta = case.theta0 + np.array([0.01, -0.01, 0.02, 0.003])
    series, bg, bj = _run(emu, tmp_path, case, theta, plan, prec)
    ref = case.series(theta)
    tol = 2e-5 if prec == 0 else 1e-10
    scale = ref.max()
    assert np.max(np.abs(series - ref)) <= tol * scale
    j_ref = int(np.argmax(ref))
    assert bg == pytest.approx(ref[j_ref], rel=20 * tol)
    assert bj == j_ref or ref[bj] >= (1 - 1e-4) * ref[j_ref]
    assert series[bj] == bg


@pytest.mark.parametrize("T1,T2", [(32, 64), (1, 1), (12, 4), (64, 128), (48, 32)])
def test_fused_schedule_order(emu, T1, T2):
    """The fused persistent schedule visits every tile once and every wait
    targets an earlier item, for the lag / slot choices the library makes
    (slots = 2 lag + 2, or lag = slots - 1 when the workspace is short)."""
    cases = []
    for cnt in (1, 2, 3, 7, 40, 320):
        for lag in (0, 1, 5, 11, 40):
            for slots in (lag + 1, 2 * lag + 2):
                cases.append((cnt, min(lag, cnt), slots))
    for cnt, lag, slots in cases:
        r = subprocess.run([emu, "schedule", str(cnt), str(lag), str(slots), str(T1), str(T2)])
        assert r.returncode == 0, (cnt, lag, slots, r.returncode)
