"""The node-wise form of the oracle step (used for sampled parity checks at full
size) agrees with the whole-lattice step."""
import numpy as np

from oracle import geometry as G, lattice, solver


def _check(dom, fluid, links, tau, force, variant):
    sim = solver.Simulation(dom, tau, force=force)
    sim.set_geometry(fluid, links, variant)
    sim.init_equilibrium()
    rng = np.random.default_rng(2)
    fl = sim.fluid
    sim.f[:, fl] *= 1.0 + 0.02 * rng.standard_normal((dom.lat.q, fl.sum()))
    f0 = sim.f.copy()
    sim.step()
    nodes = np.flatnonzero(fl)
    sub = G.cut_links(dom, fluid, *_shapes[id(dom)], nodes=nodes[::3])
    out = solver.step_at(dom, f0, fluid, sub, nodes[::3], tau, force, variant)
    np.testing.assert_allclose(out, sim.f[:, nodes[::3]], rtol=1e-15, atol=1e-17)


_shapes = {}


def test_step_at_channel_with_outlet():
    lat = lattice.D2Q9
    nx, ny = 30, 14
    dom = G.Domain(lat, nx, ny, 1, periodic=(False, False, True), outlet_face=1)
    cyl = G.Sphere((9.3, 7.1, 0), 3.2, True)
    faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(ny, 0.04)), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5)]
    _shapes[id(dom)] = ([cyl], faces)
    fluid = G.classify(dom, [cyl])
    _check(dom, fluid, G.cut_links(dom, fluid, [cyl], faces), 0.6, (0, 0, 0), "FQ")


def test_step_at_sphere_with_force():
    lat = lattice.D3Q19
    dom = G.Domain(lat, 14, 13, 12)
    sph = G.Sphere((6.2, 6.7, 5.9), 3.6, True, V=(0.01, 0, 0), Omega=(0, 0.002, 0.001))
    _shapes[id(dom)] = ([sph], [])
    fluid = G.classify(dom, [sph])
    _check(dom, fluid, G.cut_links(dom, fluid, [sph]), 0.9, (1e-5, 0, 2e-6), "FQ")
