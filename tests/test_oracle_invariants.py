"""Exact invariants of the oracle's full step (Sec. II.A-E).

* rest state f = f^eq(rho0, 0) with resting walls is a fixed point for every
  variant and any q;
* co-moving uniform flow f = f^eq(rho, U) with every wall moving at U is a
  fixed point for every variant and any q, at rho != 1, with either wall
  non-equilibrium estimator (pins the wall
  equilibria at rho_F, the Ladd term of eq. ME-solid-to-fluid with rho_F, and
  the partition of unity of the coefficients);
* a periodic all-fluid box conserves mass and momentum; Guo forcing adds
  exactly F per node and step to the momentum;
* a closed box whose walls sit half-way between nodes conserves mass exactly
  (the q = 1/2 reduction of every fragmented/quadratic variant is bounce-back).
"""
import numpy as np
import pytest

from oracle import boundary, geometry as G, lattice, solver


def _sphere_box(lat, variant, V=(0.0, 0.0, 0.0), rho=1.0, U=(0.0, 0.0, 0.0), tau=0.7, n=(14, 12, 10),
                wall_neq="bounceback"):
    nz = 1 if lat.d == 2 else n[2]
    dom = G.Domain(lat, n[0], n[1], nz)
    centre = (6.3, 5.6, 4.7 if lat.d == 3 else 0.0)
    sph = G.Sphere(centre, 3.4, True, V=V)
    fluid = G.classify(dom, [sph])
    links = G.cut_links(dom, fluid, [sph])
    assert links["q"].min() < 0.3 and links["q"].max() > 0.7
    sim = solver.Simulation(dom, tau, rho0=rho, u0=U)
    sim.set_geometry(fluid, links, variant, wall_neq=wall_neq)
    sim.init_equilibrium()
    return sim


@pytest.mark.parametrize("wall_neq", boundary.WALL_NEQ)
@pytest.mark.parametrize("lat", [lattice.D2Q9, lattice.D3Q19, lattice.D3Q27], ids=lambda l: l.name)
@pytest.mark.parametrize("variant", boundary.VARIANTS)
def test_rest_state_is_fixed_point(lat, variant, wall_neq):
    sim = _sphere_box(lat, variant, wall_neq=wall_neq)
    f0 = sim.f.copy()
    sim.run(25)
    fl = sim.fluid
    np.testing.assert_allclose(sim.f[:, fl], f0[:, fl], rtol=0, atol=1e-15)


@pytest.mark.parametrize("wall_neq", boundary.WALL_NEQ)
@pytest.mark.parametrize("lat", [lattice.D2Q9, lattice.D3Q19, lattice.D3Q27], ids=lambda l: l.name)
@pytest.mark.parametrize("variant", boundary.VARIANTS)
def test_comoving_uniform_flow_is_fixed_point(lat, variant, wall_neq):
    U = (0.03, -0.02, 0.015 if lat.d == 3 else 0.0)
    sim = _sphere_box(lat, variant, V=U, rho=1.1, U=U, wall_neq=wall_neq)
    f0 = sim.f.copy()
    sim.run(25)
    fl = sim.fluid
    np.testing.assert_allclose(sim.f[:, fl], f0[:, fl], rtol=1e-14, atol=1e-16)


def test_comoving_flow_breaks_without_ladd_density(monkeypatch):
    """The same invariant fails if the Ladd term used rho = 1 instead of rho_F
    (a mistake planted in the oracle): the invariant is sensitive to that term."""
    U = (0.03, -0.02, 0.0)
    sim = _sphere_box(lattice.D2Q9, "FQ", V=U, rho=1.1, U=U)
    orig = boundary.link_points
    monkeypatch.setattr(boundary, "link_points", lambda *a: _wrong_ladd(orig, *a))
    f0 = sim.f.copy()
    sim.run(3)
    assert np.abs(sim.f[:, sim.fluid] - f0[:, sim.fluid]).max() > 1e-6


def _wrong_ladd(orig, lat, i, rho_F, feq_F, f_F, fstar_F, uw_t, uw_t1, wall_neq="bounceback"):
    P = orig(lat, i, rho_F, feq_F, f_F, fstar_F, uw_t, uw_t1, wall_neq)
    cu = (lat.c[i].T * uw_t).sum(0)
    P[2] += 2.0 * lat.w[i] * (1.0 - rho_F) * cu / lat.cs2
    return P


@pytest.mark.parametrize("lat", [lattice.D2Q9, lattice.D3Q19, lattice.D3Q27], ids=lambda l: l.name)
def test_periodic_conservation_and_guo_momentum(lat):
    rng = np.random.default_rng(3)
    nz = 1 if lat.d == 2 else 5
    dom = G.Domain(lat, 8, 6, nz)
    F = np.array([2e-4, -1e-4, 5e-5 if lat.d == 3 else 0.0])
    sim = solver.Simulation(dom, 0.73, force=F)
    sim.set_geometry(np.ones(dom.shape, bool), G.cut_links(dom, np.ones(dom.shape, bool)))
    sim.init_equilibrium()
    sim.f = sim.f * (1.0 + 0.05 * rng.standard_normal(sim.f.shape))
    c = lat.c.astype(float)
    m0 = sim.f.sum()
    p0 = (c.T @ sim.f).sum(axis=1)
    nsteps = 13
    sim.run(nsteps)
    assert abs(sim.f.sum() - m0) < 1e-12 * m0
    p1 = (c.T @ sim.f).sum(axis=1)
    np.testing.assert_allclose(p1 - p0, nsteps * dom.N * F, rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("variant", ["FQ", "F", "UQ", "HWBB"])
def test_closed_box_half_way_walls_conserve_mass(variant):
    lat = lattice.D2Q9
    dom = G.Domain(lat, 7, 6, 1, periodic=(False, False, True))
    faces = [G.FaceWall(f, 0.5) for f in range(4)]
    fluid = np.ones(dom.shape, bool)
    links = G.cut_links(dom, fluid, [], faces)
    assert np.all(links["q"] == 0.5)
    sim = solver.Simulation(dom, 0.9)
    sim.set_geometry(fluid, links, variant)
    sim.init_equilibrium()
    rng = np.random.default_rng(5)
    sim.f = sim.f * (1.0 + 0.1 * rng.random(sim.f.shape))
    m0 = sim.f.sum()
    sim.run(40)
    assert abs(sim.f.sum() - m0) < 1e-13 * m0


def test_general_q_box_does_not_conserve_mass_exactly():
    """Interpolated walls at q != 1/2 do not conserve mass exactly (Sec. III.B, mass
    conservation violation): the closed-box test above is therefore a real check."""
    lat = lattice.D2Q9
    dom = G.Domain(lat, 7, 6, 1, periodic=(False, False, True))
    faces = [G.FaceWall(f, 0.3) for f in range(4)]
    fluid = np.ones(dom.shape, bool)
    sim = solver.Simulation(dom, 0.9)
    sim.set_geometry(fluid, G.cut_links(dom, fluid, [], faces), "FQ")
    sim.init_equilibrium()
    rng = np.random.default_rng(5)
    sim.f = sim.f * (1.0 + 0.1 * rng.random(sim.f.shape))
    m0 = sim.f.sum()
    sim.run(40)
    assert abs(sim.f.sum() - m0) > 1e-8 * m0
