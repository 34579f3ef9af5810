"""Shared set-ups for the GPU parity tests: one case description, built twice --
by the oracle (oracle/) and by the product path (library builder + kernels)."""
import numpy as np

from oracle import geometry as G, lattice as OL, solver


class Case:
    def __init__(self, lat, n, periodic=(True, True, True), outlet=None, spheres=(), faces=(), tau=0.8,
                 force=(0.0, 0.0, 0.0), rho0=1.0, u0=(0.0, 0.0, 0.0), magic=None):
        self.lat = lat
        self.n = tuple(n)
        self.periodic = tuple(periodic)
        self.outlet = outlet
        self.spheres = list(spheres)     # (centre, r, inside, V, Omega)
        self.faces = list(faces)         # (face, q, uw, profile)
        self.tau, self.force, self.rho0, self.u0 = tau, tuple(force), rho0, tuple(u0)
        self.magic = magic               # TRT magic parameter, None = BGK

    # -- oracle ---------------------------------------------------------------
    def oracle_geometry(self):
        lat = OL.get(self.lat)
        nx, ny, nz = self.n
        dom = G.Domain(lat, nx, ny, nz, periodic=self.periodic, outlet_face=self.outlet)
        z = (0.0, 0.0, 0.0)
        sh = [G.Sphere(c, r, ins, V=z if V is None else V, Omega=z if Om is None else Om)
              for c, r, ins, V, Om in self.spheres]
        fcs = []
        for f, q, uw, prof in self.faces:
            vel = None
            if uw is not None:
                vel = G.parabolic_inlet(ny, uw[0]) if prof == 1 else uw
            fcs.append(G.FaceWall(f, q, vel))
        fluid = G.classify(dom, sh)
        return dom, fluid, sh, fcs

    def oracle(self, variant="FQ", q_cut=0.01, wall_neq="bounceback"):
        dom, fluid, sh, fcs = self.oracle_geometry()
        sim = solver.Simulation(dom, self.tau, force=self.force, rho0=self.rho0, u0=self.u0, magic=self.magic)
        sim.set_geometry(fluid, G.cut_links(dom, fluid, sh, fcs), variant, q_cut, wall_neq=wall_neq)
        sim.init_equilibrium()
        return sim

    # -- product path ----------------------------------------------------------
    def gpu(self, B, storage="f64", variant="FQ", q_cut=0.01, layout="compact", wall_neq="bounceback"):
        nx, ny, nz = self.n
        g = B.Geometry(self.lat, nx, ny, nz, periodic=self.periodic, outlet_face=self.outlet)
        for c, r, ins, V, Om in self.spheres:
            g.add_sphere(c, r, ins, V=V, Omega=Om)
        for f, q, uw, prof in self.faces:
            g.add_face_wall(f, q, uw=uw, profile=prof)
        mask, links = g.build()
        g.close()
        trt = {} if self.magic is None else {"collision": "TRT", "magic": self.magic}
        d = B.Domain(self.lat, nx, ny, nz, mask, self.tau, storage=storage, periodic=self.periodic,
                     force=self.force, rho0=self.rho0, u0=self.u0, outlet_face=self.outlet, layout=layout, **trt)
        d.set_boundary_links(links, variant=variant, q_cutoff=q_cut)
        if wall_neq != "bounceback":
            d.set_wall_neq(wall_neq)
        return d, mask, links


def fluid_velocity_error(d, sim):
    rho_g, u_g, sums, unstable = d.macros()
    rho_o, u_o = sim.macros()
    fl = sim.fluid
    D = d.D
    ug = u_g[fl]                      # (n, D)
    uo = u_o[:D, fl].T
    err = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    return err, rho_g[fl], rho_o[fl], sums, unstable


def annulus_case(scale=1.0, tau=0.8, u_inner=0.01, magic=None):
    n = int(round(48 * scale))
    c = (n / 2.0, n / 2.0, 0.0)
    om1 = u_inner / (8.0 * scale)
    return Case("D2Q9", (n, n, 1), spheres=[(c, 8.0 * scale, True, None, (0, 0, om1)), (c, 20.0 * scale, False, None, None)],
                tau=tau, magic=magic)


def channel_case(nx=200, ny=80, radius=6.0, centre=(40.3, 40.6), u_max=0.05, tau=0.6, magic=None):
    return Case("D2Q9", (nx, ny, 1), periodic=(False, False, True), outlet=1,
                spheres=[((centre[0], centre[1], 0.0), radius, True, None, None)],
                faces=[(0, 0.5, (u_max, 0.0, 0.0), 1), (2, 0.5, None, 0), (3, 0.5, None, 0)], tau=tau, magic=magic)
