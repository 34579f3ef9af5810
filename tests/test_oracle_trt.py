"""Pins of the oracle's TRT collision (Sec. II.A, TRT models; eq. magic-parameter).

* with Lambda = (tau - 1/2)^2 the two rates coincide and TRT is BGK;
* the collision conserves mass and adds exactly F to the momentum under Guo
  forcing (split into symmetric and antisymmetric parts);
* Lambda = 3/16 makes half-way bounce-back viscosity independent: force-driven
  plane Poiseuille is reproduced exactly for any tau (BGK only at its "magic"
  tau) -- a planted swap of the two rates or an unsplit force term fails this;
* circular Couette with ELIBB-FQ keeps second-order convergence under TRT.
"""
import numpy as np
import pytest

from oracle import analytic, lattice, metrics, solver
from tests import cases


def _random_state(lat, n, seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.05 * rng.standard_normal(n)
    u = 0.04 * rng.standard_normal((3, n))
    if lat.d == 2:
        u[2] = 0.0
    f = solver.equilibrium(lat, rho, u) * (1.0 + 0.02 * rng.standard_normal((lat.q, n)))
    return f


@pytest.mark.parametrize("lat", [lattice.D2Q9, lattice.D3Q19], ids=["D2Q9", "D3Q19"])
def test_trt_equals_bgk_with_equal_rates(lat):
    f = _random_state(lat, 200, 1)
    F = (1e-4, -2e-4, 3e-4 if lat.d == 3 else 0.0)
    tau = 0.83
    a = solver.collide(lat, f, tau, F)[0]
    b = solver.collide(lat, f, tau, F, magic=(tau - 0.5) ** 2)[0]
    assert np.abs(a - b).max() < 1e-15 * np.abs(a).max() * 10


@pytest.mark.parametrize("lat", [lattice.D2Q9, lattice.D3Q19], ids=["D2Q9", "D3Q19"])
def test_trt_conserves_mass_and_adds_the_force(lat):
    f = _random_state(lat, 300, 2)
    F = np.array([2e-4, -1e-4, 5e-5 if lat.d == 3 else 0.0])
    fs = solver.collide(lat, f, 0.7, F, magic=3.0 / 16.0)[0]
    c = lat.c.astype(np.float64)
    np.testing.assert_allclose(fs.sum(0), f.sum(0), rtol=0, atol=1e-14)
    np.testing.assert_allclose(c.T @ fs, c.T @ f + F[:, None], rtol=0, atol=1e-14)


def test_magic_parameter_relation():
    for tau in (0.55, 0.8, 2.0):
        om_m = solver.trt_omega_minus(tau, 3.0 / 16.0)
        assert abs((tau - 0.5) * (1.0 / om_m - 0.5) - 3.0 / 16.0) < 1e-15


@pytest.mark.parametrize("tau", [0.6, 1.5])
def test_trt_poiseuille_exact_for_any_tau(tau):
    ny, F = 8, 1e-5
    nu = (tau - 0.5) / 3
    steps = int(12 * ny * ny / nu)

    def err(magic):
        sim = cases.channel(3, ny, tau=tau, force=(F, 0, 0), magic=magic)
        sim.run(steps)
        _, u = sim.macros()
        uth = analytic.poiseuille(sim.dom.coords()[1] + 0.5, ny, F, 1.0, nu)
        return np.abs(u[0] - uth).max() / uth.max()

    assert err(3.0 / 16.0) < 1e-10
    assert err(None) > 1e-2          # BGK: the wall moves with the viscosity


def test_trt_couette_second_order():
    errs = []
    for scale in (1.0, 2.0):
        sim, p, om1 = cases.annulus(scale, tau=0.8, magic=3.0 / 16.0)
        sim.run(int(3500 * scale * scale))
        _, u = sim.macros()
        X = sim.dom.coords().astype(float)
        fl = sim.fluid
        r = np.hypot(X[0, fl] - p["centre"][0], X[1, fl] - p["centre"][1])
        uth = analytic.circular_couette(r, p["r1"], p["r2"], om1)
        errs.append(metrics.rrse(np.sqrt((u[:, fl] ** 2).sum(0)), uth))
    assert errs[0] < 0.05
    assert np.log(errs[0] / errs[1]) / np.log(2.0) > 1.8
