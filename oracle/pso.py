"""Plain oracle of the lbest particle-swarm dynamics (Sec. III).

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the CPU-baseline leg of
the benchmark may use it; the HIP library never).

The paper describes the PSO variant only in words (random initialisation,
social and cognitive attraction, a ring of 40 particles with one neighbour on
each side, a fixed number of iterations, best of M independent runs) and
defers the dynamical equations to earlier work.  The reading taken here:

  * positions x and velocities v live in the unit hypercube coordinates
    x = (theta - lo) / (hi - lo) of the search rectangle;
  * initialisation: x ~ U[0,1]^4, v = u - x with u ~ U[0,1]^4, then clamped to
    [-vmax, vmax];
  * each iteration: pbest <- x where the fitness of x beats pbest_f (strictly);
    the local best of particle i is the best pbest among ring indices
    (i-1, i, i+1) (first of equal values in that order);
    v <- w v + c1 r1 (pbest - x) + c2 r2 (lbest - x), with w falling linearly
    from w0 to w1 over the iterations, r1, r2 ~ U[0,1] per coordinate, v clamped
    to [-vmax, vmax]; x <- x + v.  Particles that leave the rectangle keep
    flying and get fitness -inf (they are not evaluated there);
  * random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), key =
    (low, high) 32 bits of the seed, counter = (iteration, particle, run,
    stream) with stream 0 = initial x, 1 = initial u, 2 = r1, 3 = r2; the four
    32-bit outputs feed the four coordinates as (w + 0.5) / 2^32.

All arithmetic is IEEE float64 in a fixed order (no fused multiply-add), so
that an implementation following the same order reproduces the trajectories
bit for bit given the same fitness values.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on one counter (4 uint32) and key (2 uint32).

    Round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (64-bit products);
    c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); after every round but the
    last the key is bumped by the Weyl constants (W0, W1).
    """
    c0, c1, c2, c3 = (int(v) & _MASK for v in ctr)
    k0, k1 = (int(v) & _MASK for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + PHILOX_W0) & _MASK
            k1 = (k1 + PHILOX_W1) & _MASK
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 32, p0 & _MASK
        hi1, lo1 = p1 >> 32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniforms4(seed, iteration, particle, run, stream):
    """Four doubles in (0, 1) from one Philox call."""
    key = (seed & _MASK, (seed >> 32) & _MASK)
    w = philox4x32_10((iteration, particle, run, stream), key)
    return np.array([(float(v) + 0.5) / 4294967296.0 for v in w])


@dataclass
class PsoParams:
    n_runs: int
    n_particles: int = 40
    n_iter: int = 2000
    w0: float = 0.9
    w1: float = 0.4
    c1: float = 2.0
    c2: float = 2.0
    vmax: float = 0.5
    seed: int = 1


@dataclass
class PsoState:
    x: np.ndarray           # (R, P, 4) float64
    v: np.ndarray           # (R, P, 4) float64
    pbest_x: np.ndarray     # (R, P, 4) float64
    pbest_f: np.ndarray     # (R, P) float64
    pbest_j: np.ndarray     # (R, P) int32
    best_x: np.ndarray = field(default=None)   # (R, 4)
    best_f: np.ndarray = field(default=None)   # (R,) float64
    best_j: np.ndarray = field(default=None)   # (R,) int32


def to_theta(x, lo, hi):
    lo = np.asarray(lo, dtype=np.float64)
    span = np.asarray(hi, dtype=np.float64) - lo
    return lo + x * span


def init(p: PsoParams, lo, hi):
    R, P = p.n_runs, p.n_particles
    x = np.empty((R, P, 4))
    v = np.empty((R, P, 4))
    for r in range(R):
        for i in range(P):
            x[r, i] = uniforms4(p.seed, 0, i, r, 0)
            u = uniforms4(p.seed, 0, i, r, 1)
            v[r, i] = np.minimum(np.maximum(u - x[r, i], -p.vmax), p.vmax)
    st = PsoState(x=x, v=v, pbest_x=x.copy(),
                  pbest_f=np.full((R, P), -np.inf),
                  pbest_j=np.full((R, P), -1, dtype=np.int32),
                  best_x=np.zeros((R, 4)), best_f=np.full(R, -np.inf),
                  best_j=np.full(R, -1, dtype=np.int32))
    return st, to_theta(x, lo, hi).reshape(R * P, 4)


def inertia(p: PsoParams, iteration: int):
    if p.n_iter <= 1:
        return p.w0
    return p.w0 - (p.w0 - p.w1) * (float(iteration) / float(p.n_iter - 1))


def step(p: PsoParams, st: PsoState, fit, argmax, iteration: int, lo, hi):
    """One iteration given the fitness of the current positions; returns the
    parameters at which the next fitness batch is evaluated."""
    R, P = p.n_runs, p.n_particles
    fit = np.asarray(fit, dtype=np.float64).reshape(R, P)
    argmax = np.asarray(argmax, dtype=np.int32).reshape(R, P)
    for r in range(R):
        for i in range(P):
            if fit[r, i] > st.pbest_f[r, i]:
                st.pbest_f[r, i] = fit[r, i]
                st.pbest_x[r, i] = st.x[r, i]
                st.pbest_j[r, i] = argmax[r, i]
        b = 0
        for i in range(1, P):
            if st.pbest_f[r, i] > st.pbest_f[r, b]:
                b = i
        if st.pbest_f[r, b] > st.best_f[r]:
            st.best_f[r] = st.pbest_f[r, b]
            st.best_x[r] = st.pbest_x[r, b]
            st.best_j[r] = st.pbest_j[r, b]
    w = inertia(p, iteration)
    for r in range(R):
        lbest = np.empty(P, dtype=np.int64)
        for i in range(P):
            cand = ((i - 1) % P, i, (i + 1) % P)
            best = cand[0]
            for c in cand[1:]:
                if st.pbest_f[r, c] > st.pbest_f[r, best]:
                    best = c
            lbest[i] = best
        for i in range(P):
            r1 = uniforms4(p.seed, iteration + 1, i, r, 2)
            r2 = uniforms4(p.seed, iteration + 1, i, r, 3)
            for d in range(4):
                xv = st.x[r, i, d]
                t0 = w * st.v[r, i, d]
                t1 = (p.c1 * r1[d]) * (st.pbest_x[r, i, d] - xv)
                t2 = (p.c2 * r2[d]) * (st.pbest_x[r, lbest[i], d] - xv)
                vn = (t0 + t1) + t2
                vn = min(max(vn, -p.vmax), p.vmax)
                st.v[r, i, d] = vn
                st.x[r, i, d] = xv + vn
    return to_theta(st.x, lo, hi).reshape(R * P, 4)


def best_of_runs(st: PsoState, lo, hi):
    """Best-of-M-runs (Sec. III): the run with the largest final best fitness
    (lowest run index on ties)."""
    r = int(np.argmax(st.best_f))
    return float(st.best_f[r]), to_theta(st.best_x[r], lo, hi), int(st.best_j[r]), r
