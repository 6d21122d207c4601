"""The C ABI library loads on a machine without a GPU, exports every function
declared in include/fcas.h, and rejects bad arguments on the host before
touching a device."""
import ctypes
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcas.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2002_02150_amd import fcas
    if not os.path.exists(fcas.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return fcas.library()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("fitness_eval_batch", "fitness_grad_batch", "pso_step", "pso_init", "pso_best", "fcas_create",
                 "fcas_set_segment", "fcas_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2002_02150_amd import fcas
    names = _declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(fcas.EXPORTED) == names


def test_plan_table(lib):
    from paper_2002_02150_amd import fcas
    ps = fcas.plans()
    assert len(ps) >= 12
    for p, d in ps:
        assert d["n1"] * d["n2"] == d["n"]
        assert d["n1"] % d["e1"] == 0 and d["n2"] % d["e2"] == 0
    assert lib.fcas_plan_info(len(ps), None, None, None, None, None, None, None) == -1
    assert lib.fcas_select_plan(None, 0, 0, 0) == -1


def test_supported_lengths(lib):
    from paper_2002_02150_amd import fcas
    for n in (2048, 4096, 8192, 16384, 32768, 65536, 131072, 262144, 24576, 49152, 98304, 196608):
        assert fcas.supported_n(n)
    for n in (0, 1000, 100000, 524288, 3 * 4096):
        assert not fcas.supported_n(n)


def _good(prec=0):
    from paper_2002_02150_amd import fcas
    net = synth.network("HLVK")
    n = fcas._Network()
    n.n_det = 4
    for i in range(4):
        for a in range(3):
            n.pos_m[i][a] = net.pos_m[i][a]
            for b in range(3):
                n.tensor[i][a][b] = net.tensor[i][a][b]
    c = fcas._Config(fs_hz=2048.0, f_low_hz=30.0, f_high_hz=1000.0, precision=prec, max_batch=320,
                     max_segments=4, schedule=0, max_samples=131072, workspace_bytes=0)
    for d in range(4):
        c.box_lo[d] = synth.SEARCH_BOX_30HZ_LO[d]
        c.box_hi[d] = synth.SEARCH_BOX_30HZ_HI[d]
    return n, c


@pytest.mark.parametrize("mutate,code", [
    (lambda n, c: setattr(n, "n_det", 0), -1),
    (lambda n, c: setattr(n, "n_det", 9), -1),
    (lambda n, c: setattr(c, "precision", 7), -1),
    (lambda n, c: setattr(c, "max_batch", 0), -1),
    (lambda n, c: setattr(c, "max_samples", 100000), -3),
    (lambda n, c: setattr(c, "f_high_hz", 10.0), -1),
    (lambda n, c: setattr(c, "fs_hz", float("nan")), -1),
    (lambda n, c: c.box_lo.__setitem__(2, -1.0), -1),
    (lambda n, c: c.box_hi.__setitem__(0, -1.0), -1),
    (lambda n, c: n.pos_m[1].__setitem__(0, float("inf")), -1),
    (lambda n, c: setattr(c, "schedule", 5), -1),
])
def test_create_rejects_bad_arguments_without_device(lib, mutate, code):
    from paper_2002_02150_amd import fcas
    n, c = _good()
    mutate(n, c)
    h = ctypes.c_void_p()
    rc = lib.fcas_create(ctypes.byref(n), ctypes.byref(c), 0, ctypes.byref(h))
    assert rc == code, lib.fcas_last_error()
    assert not h.value
    assert lib.fcas_last_error()


def test_null_arguments(lib):
    n, c = _good()
    h = ctypes.c_void_p()
    assert lib.fcas_create(None, ctypes.byref(c), 0, ctypes.byref(h)) == -1
    assert lib.fcas_create(ctypes.byref(n), None, 0, ctypes.byref(h)) == -1
    assert lib.fcas_create(ctypes.byref(n), ctypes.byref(c), 0, None) == -1
    assert lib.fitness_eval_batch(None, 1, None, None, None, None, None) == -1
    assert lib.fcas_destroy(None) == -1
    assert lib.fcas_workspace_bytes(None) == 0


def test_valid_config_without_gpu_reports_hip_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    n, c = _good()
    h = ctypes.c_void_p()
    assert lib.fcas_create(ctypes.byref(n), ctypes.byref(c), 0, ctypes.byref(h)) == -4
    assert b"device" in lib.fcas_last_error()
