"""Pins of the oracle's momentum-exchange force (Sec. II "Force computation",
the Galilean-invariant form of Wen et al.; see oracle.boundary.momentum_exchange).

* momentum balance, every step, with resting walls: the force on the walls is the
  body force on the fluid minus the change of the fluid's momentum,
  F_walls = N F_body - dP (this fixes the sign and the reading of the outgoing
  population as f*_ibar);
* with a moving wall the Galilean term enters: F_walls = N F_body - dP + u_w dM,
  dM the fluid mass change, checked on a disk with a uniform wall velocity in a
  transient where mass crosses its surface;
* steady plane Couette: the walls feel the shear stress rho nu U / h per unit
  length, equal and opposite.
"""
import numpy as np
import pytest

from oracle import geometry as G, lattice, solver
from tests import cases


def _P_M(sim):
    fl = sim.fluid
    f = np.nan_to_num(sim.f[:, fl])
    c = sim.lat.c.astype(np.float64)
    return (c.T @ f).sum(axis=1), f.sum()


@pytest.mark.parametrize("q", [0.3, 0.5, 0.8])
def test_force_is_momentum_balance_with_resting_walls(q):
    F = np.array([1e-5, -3e-6, 0.0])
    sim = cases.channel(5, 10, q=q, tau=0.7, force=tuple(F))
    n = sim.fluid.sum()
    for _ in range(6):
        p0, _ = _P_M(sim)
        sim.step()
        p1, _ = _P_M(sim)
        bal = n * F - (p1 - p0)
        Fw = sim.last_force.sum(axis=0)
        assert np.abs(Fw - bal).max() < 1e-9 * np.abs(bal).max()


def test_force_galilean_term_with_moving_wall():
    """A disk with wall velocity V (static geometry) in a periodic box: mass
    crosses its surface while the flow develops, and the force must balance the
    momentum change with the Galilean term (the plain momentum exchange misses it
    by up to 1e-3 of the force here)."""
    lat = lattice.D2Q9
    V = np.array([0.02, -0.01, 0.0])
    dom = G.Domain(lat, 24, 20, 1)
    sph = G.Sphere((11.3, 9.7, 0.0), 5.2, True, V=tuple(V))
    fluid = G.classify(dom, [sph])
    sim = solver.Simulation(dom, 0.75, rho0=1.03)
    sim.set_geometry(fluid, G.cut_links(dom, fluid, [sph]), "FQ")
    sim.init_equilibrium()
    masses = []
    for _ in range(6):
        p0, m0 = _P_M(sim)
        sim.step()
        p1, m1 = _P_M(sim)
        dM = m1 - m0
        masses.append(abs(dM))
        expect = -(p1 - p0) + V * dM
        Fw = sim.last_force.sum(axis=0)
        assert np.abs(Fw - expect).max() < 1e-11 * np.abs(expect).max()
    assert max(masses) > 1e-3        # mass did cross the moving wall: the u_w term was exercised


@pytest.mark.parametrize("q", [0.5, 0.3])
def test_steady_couette_wall_shear(q):
    U, tau, ny, nx = 0.01, 0.8, 10, 3
    sim = cases.channel(nx, ny, q=q, u_top=(U, 0, 0), tau=tau)
    sim.set_link_groups(sim.links["shape"], 2)          # faces: 0 = bottom, 1 = top
    nu = (tau - 0.5) / 3
    h = ny - 1 + 2 * q
    sim.run(int(30 * h * h / nu))
    Fb, Ft = sim.last_force
    shear = nu * U / h * nx
    assert abs(Fb[0] - shear) < 1e-10 * shear
    assert abs(Ft[0] + shear) < 1e-10 * shear
