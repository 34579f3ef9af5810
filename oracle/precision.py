"""Arithmetic type of the oracle.

Test infrastructure only (see the package header).  The oracle computes in
float64 unless a caller selects the host's extended type for a block of work:

    with precision.extended():
        sim = solver.Simulation(...)      # populations, weights, c_s^2, omega
        sim.run(n)                        # all in long double

`extended()` selects numpy.longdouble, the x87 80-bit format on x86-64 hosts
(64-bit significand, unit round-off 2^-64 ~ 5.4e-20, 2048 times finer than
float64).  An extended-precision run separates the oracle's own float64
rounding -- which, in a step that stores the populations f = w + O(u), leaves
the velocity with ~|w|/|u| fewer correct digits than the populations -- from a
GPU path's.  The geometry (fluid mask, q, wall velocities) stays float64 in
both modes: it is an input, the same numbers on every side.

Status: pinned (tests/test_oracle_precision.py: the type really carries 64
significand bits, the extended run agrees with the float64 run to float64's
accuracy, and conserves mass in a closed box to its own accuracy).
"""
import contextlib
from fractions import Fraction

import numpy as np

REAL = np.float64


@contextlib.contextmanager
def extended():
    """Compute in numpy.longdouble inside the block."""
    global REAL
    old = REAL
    REAL = np.longdouble
    try:
        yield
    finally:
        REAL = old


def real(x):
    """x as an array of the current arithmetic type."""
    return np.asarray(x, dtype=REAL)


def scalar(x):
    """A Python number or Fraction as a scalar of the current type (a Fraction
    is divided in that type, so 1/3 is rounded once, in that type)."""
    if isinstance(x, Fraction):
        return REAL(x.numerator) / REAL(x.denominator)
    return REAL(x)
