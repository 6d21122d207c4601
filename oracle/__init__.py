"""FP64 CPU oracle of the coherent-fitness hot path (arXiv:2002.02150).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import, call or execute anything in this package.
The HIP library never does, and this package imports nothing from it.

  fitness   -- Gamma^2 and its maximising sample (Sec. II.C, II.D)
  gradient  -- dGamma^2/dtheta at the maximising sample
  signal    -- the signal model and the literal log-likelihood ratio
  pso       -- the lbest PSO dynamics with Philox4x32-10 random numbers (Sec. III)

Parity status of each function and what pins it is listed in the tests
(tests/test_oracle_*.py).
"""
from . import fitness, gradient, pso, signal  # noqa: F401
