"""MI355X-native coherent-fitness library for the PSO-driven fully-coherent
all-sky search for compact-binary inspirals (arXiv:2002.02150).

The compute path is libfcas.so (HIP kernels for gfx950 behind the C ABI in
include/fcas.h); `fcas` is its thin Python binding.
"""
from .fcas import (FP64, MIXED, Context, FcasError, FitnessFn, PsoConfig, Swarm, library,  # noqa: F401
                   polish, supported_n)
