"""Pins of the PSO oracle: the published Philox known answers, the ring
neighbourhood, the velocity clamp and inertia schedule, let-them-fly, and
convergence on a smooth function."""
import json
import os

import numpy as np
import pytest

from oracle import pso

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(h, 16) for h in v["ctr"]]
        key = [int(h, 16) for h in v["key"]]
        assert list(pso.philox4x32_10(ctr, key)) == [int(h, 16) for h in v["out"]]


def test_uniforms_in_open_interval_and_distinct_streams():
    u = np.array([pso.uniforms4(7, it, i, r, s) for it in range(20) for i in range(5) for r in range(2) for s in range(4)])
    assert np.all(u > 0) and np.all(u < 1)
    assert abs(u.mean() - 0.5) < 0.03
    assert len(np.unique(u)) == u.size


def test_inertia_schedule_endpoints():
    p = pso.PsoParams(n_runs=1, n_iter=11)
    assert pso.inertia(p, 0) == 0.9
    assert pso.inertia(p, 10) == pytest.approx(0.4, abs=1e-15)
    assert pso.inertia(p, 5) == pytest.approx(0.65, abs=1e-15)


def test_init_inside_unit_box_and_clamped():
    p = pso.PsoParams(n_runs=3, n_particles=40, seed=123)
    st, th = pso.init(p, [0, 0, 0, 0], [1, 1, 1, 1])
    assert np.all((st.x > 0) & (st.x < 1))
    assert np.all(np.abs(st.v) <= p.vmax)
    assert np.array_equal(th.reshape(st.x.shape), st.x)
    assert np.all(np.isneginf(st.pbest_f))


def test_ring_neighbourhood_and_pbest():
    """Particle i is attracted to the best pbest among ring indices (i-1, i, i+1)
    (first of equal values in that order).  With w = c1 = 0 the new velocity is
    exactly c2 r2 (pbest[lbest] - x), which identifies lbest."""
    P = 8
    p = pso.PsoParams(n_runs=1, n_particles=P, n_iter=10, c1=0.0, c2=2.0, w0=0.0, w1=0.0, vmax=10.0, seed=9)
    st, _ = pso.init(p, [0] * 4, [1] * 4)
    fit = np.full(P, 1.0, dtype=np.float32)
    fit[3] = 5.0
    fit[6] = 2.0
    x0 = st.x[0].copy()
    pso.step(p, st, fit, np.arange(P), 0, [0] * 4, [1] * 4)
    expect_lbest = {0: 7, 1: 0, 2: 3, 3: 3, 4: 3, 5: 6, 6: 6, 7: 6}
    for i in range(P):
        r2 = pso.uniforms4(p.seed, 1, i, 0, 3)
        want = (p.c2 * r2) * (x0[expect_lbest[i]] - x0[i])
        assert np.array_equal(st.v[0, i], (0.0 + 0.0) + want), i
    assert st.pbest_f[0, 3] == 5.0
    assert st.best_f[0] == 5.0 and st.best_j[0] == 3


def test_velocity_clamp_and_let_them_fly():
    p = pso.PsoParams(n_runs=2, n_particles=6, n_iter=5, w0=5.0, w1=5.0, vmax=0.25, seed=4)
    st, _ = pso.init(p, [0] * 4, [1] * 4)
    fit = np.zeros(12, dtype=np.float32)
    for it in range(4):
        th = pso.step(p, st, fit, np.zeros(12), it, [0] * 4, [1] * 4)
        assert np.all(np.abs(st.v) <= 0.25)
    # with large inertia some particles leave the unit box; they are not pulled back
    assert np.any((th < 0) | (th > 1))
    # -inf fitness (outside the box) never becomes a personal best
    fit = np.full(12, -np.inf, dtype=np.float32)
    before = st.pbest_f.copy()
    pso.step(p, st, fit, np.full(12, -1), 4, [0] * 4, [1] * 4)
    assert np.array_equal(before, st.pbest_f)


def test_swarm_converges_on_smooth_peak():
    """Best-of-runs lbest PSO finds the maximum of a smooth unimodal function."""
    p = pso.PsoParams(n_runs=2, n_particles=20, n_iter=120, seed=2024)
    lo, hi = np.zeros(4), np.ones(4)
    centre = np.array([0.3, 0.7, 0.55, 0.2])
    st, th = pso.init(p, lo, hi)
    for it in range(p.n_iter):
        inside = np.all((th >= lo) & (th <= hi), axis=1)
        f = np.where(inside, 10.0 - np.sum((th - centre) ** 2, axis=1), -np.inf).astype(np.float32)
        th = pso.step(p, st, f, np.zeros(len(f)), it, lo, hi)
    bf, bx, _, _ = pso.best_of_runs(st, lo, hi)
    assert np.linalg.norm(bx - centre) < 1e-2
    assert bf > 10.0 - 1e-4

