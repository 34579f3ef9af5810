"""The zero-gradient outlet through the C-ABI: the GPU path reproduces the
oracle's behaviour under a velocity inlet (the mass grows) to FP64 parity over
a long run, also with an obstacle next to the outlet face layer."""
import numpy as np
import pytest

from oracle import geometry as G, lattice as OL, solver

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def test_zero_gradient_outlet_mass_growth_matches_oracle(gpu_lib):
    B = gpu_lib
    nx, ny, u_max, tau = 60, 12, 0.02, 0.8
    _say("case inlet channel 60x12 zero-gradient outlet f64, 6600 steps")
    dom = G.Domain(OL.D2Q9, nx, ny, 1, periodic=(False, False, True), outlet_face=1)
    faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(ny, u_max)), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5)]
    fluid = np.ones(dom.shape, bool)
    sim = solver.Simulation(dom, tau)
    sim.set_geometry(fluid, G.cut_links(dom, fluid, [], faces), "FQ")
    sim.init_equilibrium()
    g = B.Geometry("D2Q9", nx, ny, 1, periodic=(False, False, True), outlet_face="+x")
    g.add_face_wall("-x", 0.5, uw=(u_max, 0, 0), profile=1)
    g.add_face_wall("-y", 0.5)
    g.add_face_wall("+y", 0.5)
    mask, links = g.build()
    g.close()
    d = B.Domain("D2Q9", nx, ny, 1, mask, tau, storage="f64", periodic=(False, False, True), outlet_face="+x")
    d.set_boundary_links(links)
    sim.run(6000)
    d.step(6000)
    m_a = d.macros(fields=False)[2][0]
    assert abs(m_a / sim.macros()[0].sum() - 1.0) < 1e-12
    sim.run(600)
    d.step(600)
    rho_g, u_g, sums, unstable = d.macros()
    assert not unstable
    rho_o, u_o = sim.macros()
    err = np.linalg.norm(u_g - u_o[:2].T) / np.linalg.norm(u_o[:2])
    _say("rel L2 velocity", err, "mass growth", sums[0] / m_a - 1.0)
    assert err <= 1e-12
    assert sums[0] > 1.02 * m_a
    d.close()


def test_obstacle_next_to_outlet_face_layer(gpu_lib):
    """An obstacle whose solid nodes touch the outlet face layer: the face nodes
    next to it have both cut links and clamped outlet pulls that read the same
    face-layer slots (FP64 parity with the oracle)."""
    B = gpu_lib
    nx, ny, tau = 40, 16, 0.7
    _say("case channel 40x16 with an obstacle next to the outlet face layer, f64, 800 steps")
    g = B.Geometry("D2Q9", nx, ny, 1, periodic=(False, False, True), outlet_face="+x")
    g.add_sphere((nx - 3.0, 8.0, 0.0), 1.2)           # solid nodes next to the outlet face layer x = nx - 1
    g.add_face_wall("-x", 0.5, uw=(0.02, 0, 0), profile=1)
    g.add_face_wall("-y", 0.5)
    g.add_face_wall("+y", 0.5)
    mask, links = g.build()
    g.close()
    d = B.Domain("D2Q9", nx, ny, 1, mask, tau, storage="f64", periodic=(False, False, True), outlet_face="+x")
    d.set_boundary_links(links)
    dom = G.Domain(OL.D2Q9, nx, ny, 1, periodic=(False, False, True), outlet_face=1)
    sph = G.Sphere((nx - 3.0, 8.0, 0.0), 1.2, True)
    faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(ny, 0.02)), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5)]
    fluid = G.classify(dom, [sph])
    assert np.array_equal(fluid.reshape(-1).astype(np.uint8), mask)
    sim = solver.Simulation(dom, tau)
    sim.set_geometry(fluid, G.cut_links(dom, fluid, [sph], faces), "FQ")
    sim.init_equilibrium()
    d.step(800)
    sim.run(800)
    _, u_g, _, unstable = d.macros()
    assert not unstable
    _, u_o = sim.macros()
    fl = sim.fluid
    err = np.linalg.norm(u_g[fl] - u_o[:2, fl].T) / np.linalg.norm(u_o[:2, fl])
    _say("rel L2 velocity", err)
    d.close()
    assert err <= 1e-12
