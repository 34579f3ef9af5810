"""Pins of the oracle's extended-precision mode (oracle.precision), which the
full-length FP64 parity tests use to separate the oracle's own float64 rounding
from the GPU path's.

* the host's long double carries a 64-bit significand (else the mode is
  pointless and these tests skip);
* inside extended() the weights and c_s^2 are rounded once in that type (their
  sum and 3 c_s^2 are 1 to its unit round-off), and a run's populations stay in
  it;
* the extended and float64 runs of the same flow agree to float64's accuracy
  (the mode changes rounding only, not the method);
* a closed box with half-way walls conserves mass exactly in exact arithmetic
  (tests/test_oracle_invariants.py); in float64 the sum drifts by rounding, in
  extended precision by ~2000 times less -- which fails if any part of the step
  (moments, equilibrium, collision, streaming, wall rebuild) silently fell back
  to float64.
"""
import numpy as np
import pytest

from oracle import geometry as G, lattice, precision, solver

pytestmark = pytest.mark.skipif(np.finfo(np.longdouble).nmant < 63,
                                reason="long double is not an extended type on this host")


def test_extended_type_and_constants():
    assert precision.REAL is np.float64
    with precision.extended():
        assert precision.REAL is np.longdouble
        for lat in (lattice.D2Q9, lattice.D3Q19, lattice.D3Q27):
            assert lat.w.dtype == np.longdouble
            assert abs(lat.w.sum() - 1) <= 4 * np.finfo(np.longdouble).eps
            assert abs(3 * lat.cs2 - 1) <= 2 * np.finfo(np.longdouble).eps
        # the weight of 1/36 is not the float64 one widened
        w = lattice.D2Q9.w[5]
        assert w != np.longdouble(1.0 / 36.0) and abs(w * 36 - 1) <= 2 * np.finfo(np.longdouble).eps
    assert precision.REAL is np.float64 and lattice.D2Q9.w.dtype == np.float64


def _box(variant, q):
    dom = G.Domain(lattice.D2Q9, 9, 7, 1, periodic=(False, False, True))
    faces = [G.FaceWall(f, q) for f in range(4)]
    fluid = np.ones(dom.shape, bool)
    sim = solver.Simulation(dom, 0.9)
    sim.set_geometry(fluid, G.cut_links(dom, fluid, [], faces), variant)
    sim.init_equilibrium()
    rng = np.random.default_rng(5)
    sim.f = sim.f * (1.0 + 0.1 * rng.random(sim.f.shape))
    return sim


def _run(variant, q, steps, ext):
    if ext:
        with precision.extended():
            sim = _box(variant, q)
            m0 = sim.f.sum()
            sim.run(steps)
            assert sim.f.dtype == np.longdouble
            return sim.f.copy(), m0
    sim = _box(variant, q)
    m0 = sim.f.sum()
    sim.run(steps)
    return sim.f.copy(), m0


@pytest.mark.parametrize("variant", ["FQ", "HWBB"])
def test_extended_run_agrees_and_conserves_mass_tighter(variant):
    f64, m64 = _run(variant, 0.5, 200, False)
    fx, mx = _run(variant, 0.5, 200, True)
    # same flow to float64 accuracy
    assert np.abs(f64 - fx.astype(np.float64)).max() <= 1e-13
    drift64 = abs(float(f64.sum() - m64)) / float(m64)
    driftx = abs(float((fx.sum() - mx) / mx))
    assert driftx <= 1e-17
    assert drift64 > 0 and driftx * 100 < drift64, (drift64, driftx)


def test_extended_run_of_interpolated_walls():
    """q = 0.3 (interpolated ELIBB-FQ, moving-wall-free): the same populations to
    float64 accuracy; the q != 1/2 mass change itself is the method's, equal in
    both precisions."""
    f64, m64 = _run("FQ", 0.3, 100, False)
    fx, mx = _run("FQ", 0.3, 100, True)
    assert np.abs(f64 - fx.astype(np.float64)).max() <= 1e-13
    d64 = float(f64.sum() - m64)
    dx = float(fx.sum() - mx)
    # float64 sums of ~570 populations carry ~1e-13 each; 100 steps of its drift
    assert abs(d64) > 1e-8 and abs(d64 - dx) <= 1e-11
