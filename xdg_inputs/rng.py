"""Seeded random draws of the synthetic workloads (numpy PCG64 streams).

Draw order per problem: geometry parameters first, then right-hand sides.
"""
import numpy as np


def problem_rng(seed):
    return np.random.default_rng(seed)


def sphere_jitter(g, amp):
    """Centre offset, each component ~ U[-amp, amp]."""
    return g.uniform(-amp, amp, 3)


def ellipsoid_axes(g, lo, hi):
    """Three semi-axes ~ U[lo, hi]."""
    return g.uniform(lo, hi, 3)


def uniform_rhs(g, L, nrhs=1):
    """Right-hand side coefficients ~ U[-1, 1]; [L] or [L, nrhs]."""
    if nrhs == 1:
        return g.uniform(-1.0, 1.0, L)
    return g.uniform(-1.0, 1.0, (L, nrhs))
