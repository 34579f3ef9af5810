"""Small oracle set-ups shared by the CPU tests (built only from oracle/ and synth/)."""
import numpy as np

import synth
from oracle import geometry as G, lattice, solver


def annulus(scale=1.0, u_inner=0.01, tau=0.8, variant="FQ", omega_outer=0.0, magic=None, wall_neq="bounceback"):
    p = synth.couette_annulus(scale, u_inner=u_inner, tau=tau)
    dom = G.Domain(lattice.D2Q9, p["nx"], p["ny"], 1)
    om1 = p["u_inner"] / p["r1"]
    inner = G.Sphere(p["centre"], p["r1"], True, Omega=(0, 0, om1))
    outer = G.Sphere(p["centre"], p["r2"], False, Omega=(0, 0, omega_outer))
    fluid = G.classify(dom, [inner, outer])
    links = G.cut_links(dom, fluid, [inner, outer])
    sim = solver.Simulation(dom, p["tau"], magic=magic)
    sim.set_geometry(fluid, links, variant, wall_neq=wall_neq)
    sim.init_equilibrium()
    return sim, p, om1


def channel(nx, ny, walls=("-y", "+y"), q=0.5, u_top=(0.0, 0.0, 0.0), tau=0.8, force=(0, 0, 0),
            variant="FQ", periodic_x=True, lat=lattice.D2Q9, nz=1, magic=None, wall_neq="bounceback"):
    per = (periodic_x, False, True)
    dom = G.Domain(lat, nx, ny, nz, periodic=per)
    faces = []
    for w in walls:
        f = G.FACES.index(w)
        faces.append(G.FaceWall(f, q, u_top if w == "+y" else None))
    fluid = np.ones(dom.shape, dtype=bool)
    links = G.cut_links(dom, fluid, [], faces)
    sim = solver.Simulation(dom, tau, force=force, magic=magic)
    sim.set_geometry(fluid, links, variant, wall_neq=wall_neq)
    sim.init_equilibrium()
    return sim
