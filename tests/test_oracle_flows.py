"""Whole-scheme pins of the oracle against closed-form flows.

* circular Couette (Sec. III.B closed form): rRSE of the velocity norm and
  second-order convergence under diffusive refinement (tau fixed; the paper
  reports second order for all ELIBB variants, Sec. III.B "rRSE convergence");
* impulsively started plane Couette (eq. solution-couette, 100-term series);
* force-driven plane Poiseuille: exact with half-way walls at the BGK "magic"
  relaxation tau = 1/2 + sqrt(3/16) (Lambda = 3/16, Sec. II.A TRT paragraph),
  second order with interpolated walls in a channel tilted at slope 1/2.
"""
import numpy as np
import pytest

from oracle import analytic, geometry as G, lattice, metrics, solver
from tests import cases


def _couette_rrse(scale, variant="FQ", tau=0.8, steps_per_area=3500):
    sim, p, om1 = cases.annulus(scale, tau=tau, variant=variant)
    sim.run(int(steps_per_area * scale * scale))
    rho, u = sim.macros()
    X = sim.dom.coords().astype(float)
    fl = sim.fluid
    r = np.hypot(X[0, fl] - p["centre"][0], X[1, fl] - p["centre"][1])
    uth = analytic.circular_couette(r, p["r1"], p["r2"], om1)
    return metrics.rrse(np.sqrt((u[:, fl] ** 2).sum(0)), uth), rho[fl]


def test_circular_couette_counts():
    sim, p, _ = cases.annulus(1.0)
    assert sim.fluid.sum() == 1048
    assert sim.links["node"].size == 544
    assert np.unique(sim.links["node"]).size == 224


@pytest.mark.parametrize("variant,bound", [("FQ", 5e-3), ("F", 6e-3), ("U", 8e-3), ("HWBB", 3e-2)])
def test_circular_couette_accuracy(variant, bound):
    e, rho = _couette_rrse(1.0, variant, steps_per_area=5000)
    assert e < bound
    assert metrics.mean_density_fluctuation(rho) < 2e-3


def test_circular_couette_second_order():
    e1, _ = _couette_rrse(0.75)
    e2, _ = _couette_rrse(1.5)
    slope = np.log(e1 / e2) / np.log(2.0)
    assert slope > 1.8, (e1, e2, slope)


def test_quadratic_unified_variant_unstable_near_q_one():
    """Under the readings used here, ELIBB-UQ is unstable on the 48x48 annulus at
    tau = 0.8 (links with q close to 1: the coincident nodes P0, P2); it is stable
    at tau = 1.5.  FQ, the default, is stable at both."""
    e_hi, _ = _couette_rrse(1.0, "UQ", tau=1.5, steps_per_area=2000)
    assert e_hi < 0.06
    with np.errstate(all="ignore"):
        e_lo, _ = _couette_rrse(1.0, "UQ", tau=0.8, steps_per_area=2000)
    assert not (e_lo < 0.06)


def test_impulsive_couette_series():
    errs = []
    for n in (10, 20):
        q, U, tau = 0.3, 0.01, 0.8
        h = n - 1 + 2 * q
        nu = (tau - 0.5) / 3
        sim = cases.channel(2, n, q=q, u_top=(U, 0, 0), tau=tau)
        T = int(round(0.2 * h * h / nu))
        sim.run(T)
        _, u = sim.macros()
        y = sim.dom.coords()[1] + q
        errs.append(metrics.rrse(u[0], analytic.impulsive_couette(y, h, U, nu, T)))
    assert errs[0] < 3e-4 and errs[1] < 5e-5
    assert np.log(errs[0] / errs[1]) / np.log((20 - 0.4) / (10 - 0.4)) > 1.8


def test_poiseuille_magic_tau_half_way_exact():
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    ny, F = 8, 1e-5
    sim = cases.channel(3, ny, tau=tau, force=(F, 0, 0))
    sim.run(4000)
    _, u = sim.macros()
    y = sim.dom.coords()[1]
    uth = analytic.poiseuille(y + 0.5, ny, F, 1.0, (tau - 0.5) / 3)
    assert np.abs(u[0] - uth).max() < 1e-11 * uth.max()
    assert np.abs(u[1]).max() < 1e-15


def _tilted(m):
    lat = lattice.D2Q9
    dom = G.Domain(lat, 2 * m, m, 1)
    W = 0.7 * m
    band = G.TiltedBand(0.5, 0.123 * m / 10, m, W)
    fluid = G.classify(dom, [band])
    links = G.cut_links(dom, fluid, [band])
    tau = 0.8
    nu = (tau - 0.5) / 3
    e = np.array([2.0, 1.0, 0.0]) / np.sqrt(5)
    Fm = 4e-6 * (10.0 / m) ** 2
    sim = solver.Simulation(dom, tau, force=Fm * e)
    sim.set_geometry(fluid, links, "FQ")
    sim.init_equilibrium()
    H = W * 2 / np.sqrt(5)
    sim.run(int(8 * H * H / nu))
    _, u = sim.macros()
    X = dom.coords().astype(float)
    fl = fluid.reshape(-1)
    n = band.g(X[:, fl]) * 2 / np.sqrt(5)
    return metrics.rrse(e[:2] @ u[:2, fl], analytic.poiseuille(n, H, Fm, 1.0, nu))


def test_tilted_poiseuille_second_order():
    e10, e20 = _tilted(10), _tilted(20)
    assert e10 < 0.04 and e20 < 0.01
    assert np.log(e10 / e20) / np.log(2.0) > 1.8


def test_analytic_forms_are_solutions():
    # circular Couette: boundary values and the steady Stokes operator u'' + u'/r - u/r^2 = 0
    r1, r2, om = 8.0, 20.0, 0.01 / 8
    assert abs(analytic.circular_couette(r1, r1, r2, om) - om * r1) < 1e-15
    assert abs(analytic.circular_couette(r2, r1, r2, om)) < 1e-15
    r = np.linspace(9, 19, 11)
    h = 1e-3
    u = lambda x: analytic.circular_couette(x, r1, r2, om)
    lap = (u(r + h) - 2 * u(r) + u(r - h)) / h ** 2 + (u(r + h) - u(r - h)) / (2 * h * r) - u(r) / r ** 2
    assert np.abs(lap).max() < 1e-8
    # impulsive Couette: steady limit, boundary values, heat equation
    y = np.linspace(0, 2.0, 9)
    np.testing.assert_allclose(analytic.impulsive_couette(y, 2.0, 1.0, 0.1, 1e6), y / 2.0, atol=1e-12)
    assert abs(analytic.impulsive_couette(0.0, 2.0, 1.0, 0.1, 3.0)) < 1e-15
    yy, t, dt, dy = np.linspace(0.3, 1.7, 8), 2.0, 1e-4, 1e-3
    U = lambda yv, tv: analytic.impulsive_couette(yv, 2.0, 1.0, 0.1, tv)
    ut = (U(yy, t + dt) - U(yy, t - dt)) / (2 * dt)
    uyy = (U(yy + dy, t) - 2 * U(yy, t) + U(yy - dy, t)) / dy ** 2
    np.testing.assert_allclose(ut, 0.1 * uyy, atol=1e-5)
    # Poiseuille: u'' = -F / (rho nu), zero at both walls
    n = np.array([0.0, 3.0])
    np.testing.assert_allclose(analytic.poiseuille(n, 3.0, 1.0, 1.0, 0.2), 0.0, atol=1e-15)


def test_metrics_elementary():
    a = np.array([1.0, 2.0, 3.0])
    assert metrics.rrse(a, a) == 0.0
    assert abs(metrics.rrse(a * 1.01, a) - 0.01) < 1e-14
    assert abs(metrics.rel_l2(a * 0.98, a) - 0.02) < 1e-14
    assert abs(metrics.mean_density_fluctuation([1.1, 0.9, 1.3]) - 0.1) < 1e-14


def test_wall_distance_matters_little_for_elibb_and_much_for_hwbb():
    """The paper finds that q has a small effect on the error of the ELIBB
    variants and a large one for half-way bounce-back (Sec. III.B, q-dependence):
    force-driven Poiseuille (BGK, tau 0.8) between walls at distance q from the
    first and last node layers, against the parabola between the true walls."""
    ny, F, tau = 8, 1e-5, 0.8
    nu = (tau - 0.5) / 3
    err = {}
    for v in ("FQ", "HWBB"):
        for q in (0.1, 0.5, 0.9):
            sim = cases.channel(3, ny, q=q, tau=tau, force=(F, 0, 0), variant=v)
            sim.run(int(12 * ny * ny / nu))
            _, u = sim.macros()
            y = sim.dom.coords()[1].astype(float) + q           # distance from the lower wall
            H = ny - 1 + 2 * q
            uth = F / (2 * nu) * y * (H - y)
            err[v, q] = np.abs(u[0] - uth).max() / uth.max()
    assert err["FQ", 0.5] == err["HWBB", 0.5]                   # q = 1/2: the same scheme
    assert max(err["FQ", q] for q in (0.1, 0.5, 0.9)) < 0.04
    for q in (0.1, 0.9):
        assert err["HWBB", q] > 5 * err["FQ", q]


def _inlet_channel(nx=60, ny=12, u_max=0.02, tau=0.8):
    per = (False, False, True)
    faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(ny, u_max)), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5)]
    dom = G.Domain(lattice.D2Q9, nx, ny, 1, periodic=per, outlet_face=1)
    sim = solver.Simulation(dom, tau)
    fluid = np.ones(dom.shape, bool)
    sim.set_geometry(fluid, G.cut_links(dom, fluid, [], faces), "FQ")
    sim.init_equilibrium()
    return sim


def test_zero_gradient_outlet_mass_grows_under_velocity_inlet():
    """A straight channel fed with the Poiseuille profile (velocity inlet, walls at
    q = 1/2) and the zero-gradient outlet: the mass keeps growing (the outflow
    falls short of the inflow and the inlet's momentum term scales with the
    density) while the flow stays symmetric.  A finding about the outlet reading,
    asserted so that the GPU path is held to the same behaviour."""
    nx, ny = 60, 12
    zg = _inlet_channel(nx, ny)
    zg.run(6000)
    m_a = zg.macros()[0].sum()
    zg.run(600)
    rho, u = zg.macros()
    assert rho.sum() > 1.02 * m_a                                   # keeps growing
    ux = u[0].reshape(ny, nx)
    np.testing.assert_allclose(ux, ux[::-1], rtol=1e-10, atol=1e-15)   # symmetric about the centre line
    assert np.all(ux[:, nx // 2] > 0)
