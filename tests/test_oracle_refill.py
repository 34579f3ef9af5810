"""Pins of the oracle's fresh-node refill and of the prescribed sphere kinematics.

Refill (reading of the fresh-node treatment of Sec. III.C, run before the step
as in the LIR appendix): a node that is solid at t-1 and fluid at t takes
f^eq(rho_bar, u_body(x)), rho_bar the mean density of its lattice neighbours
x + c_j (j = 1..Q-1) that are fluid at both t-1 and t, or rho0 when there is
none.  The neighbour sets below are listed by hand on tiny D2Q9 grids (node
n = x + nx y), so that a wrong neighbour set, a refill that always takes rho0,
one that also counts fresh neighbours or one that counts neighbours that turned
solid fails.

Kinematics: x_c(t) = x_0 + A sin(2 pi t / T) e; its velocity V(t) must be the
time derivative of x_c, checked against central differences over one period.
"""
import numpy as np
import pytest

from oracle import geometry as G, lattice, moving, solver


def _eq_d2q9(rho, u):
    """Second-order equilibrium written out for D2Q9 (eq. Eq2ndOrder, c_s^2 = 1/3)."""
    c = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1)]
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    uu = u[0] * u[0] + u[1] * u[1]
    out = []
    for (cx, cy), wi in zip(c, w):
        cu = cx * u[0] + cy * u[1]
        out.append(wi * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu))
    return np.array(out)


def _mask_links(dom, fluid):
    """Half-way links (q = 1/2, walls at rest) for every population a mask leaves missing."""
    lat = dom.lat
    nodes = np.flatnonzero(fluid)
    X = dom.coords(nodes)
    node, dirs = [], []
    for i in range(1, lat.q):
        src, inside = G._source(dom, X.copy(), lat.c[i])
        sidx = np.where(inside, G._index(dom, np.where(inside, src, 0)), 0)
        miss = ~(inside & fluid[sidx])
        node.append(nodes[miss])
        dirs.append(np.full(miss.sum(), i))
    node, dirs = np.concatenate(node), np.concatenate(dirs)
    n = node.size
    return {"node": node, "dir": dirs, "q": np.full(n, 0.5), "uw_t": np.zeros((3, n)), "uw_t1": np.zeros((3, n))}


def _setup(nx, ny, old_solid, rho0, seed, periodic=(True, True, True)):
    dom = G.Domain(lattice.D2Q9, nx, ny, 1, periodic=periodic)
    fluid = np.ones(dom.N, bool)
    for (x, y) in old_solid:
        fluid[x + nx * y] = False
    sim = solver.Simulation(dom, 0.8, rho0=rho0)
    sim.set_geometry(fluid, _mask_links(dom, fluid))
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.2 * rng.random(dom.N)          # clearly non-uniform densities
    u = 0.02 * (rng.random((3, dom.N)) - 0.5)
    u[2] = 0.0
    sim.init_equilibrium(rho, u)
    return sim, dom, rho


def _new_mask(dom, new_solid):
    m = np.ones(dom.N, bool)
    for (x, y) in new_solid:
        m[x + dom.n[0] * y] = False
    return m


def test_refill_mean_over_neighbours_fluid_at_both_times():
    nx, ny = 6, 5
    # solid at t-1: (1,2) (2,2); solid at t: (3,2) (4,2)
    # fresh at t: (1,2) = 13 and (2,2) = 14, next to each other; (3,2) = 15 was
    # fluid at t-1 and is solid at t
    sim, dom, rho = _setup(nx, ny, [(1, 2), (2, 2)], 1.0, seed=11)
    new = _new_mask(dom, [(3, 2), (4, 2)])
    ub = np.zeros((3, dom.N))
    ub[0], ub[1] = 0.013, -0.007
    fresh = sim.refill(new, ub)
    assert sorted(fresh.tolist()) == [13, 14]
    # hand-listed neighbours x + c_j fluid at both times:
    #   node 14 (2,2): (3,2) = 15 turned solid, (1,2) = 13 is fresh -> both excluded
    #   node 13 (1,2): (2,2) = 14 is fresh -> excluded; (0,2) = 12 stays fluid
    valid = {14: [20, 8, 21, 9, 19, 7], 13: [12, 19, 7, 20, 8, 18, 6]}
    for n, nb in valid.items():
        np.testing.assert_allclose(sim.f[:, n], _eq_d2q9(rho[nb].mean(), ub[:, n]), rtol=0, atol=1e-15)
    # the planted mistakes this pin must catch move rho_bar by far more than the
    # tolerance: always rho0, counting the neighbour that turned solid (its t-1
    # density is at hand), counting a fresh neighbour (taken at rho0)
    for n, nb in valid.items():
        assert abs(rho[nb].mean() - 1.0) > 1e-3
    assert abs(rho[valid[14]].mean() - rho[valid[14] + [15]].mean()) > 1e-4
    assert abs(rho[valid[13]].mean() - np.mean(list(rho[valid[13]]) + [1.0])) > 1e-4
    # nodes that stay fluid keep their populations; nodes that turned solid hold none
    keep = new & ~np.isin(np.arange(dom.N), fresh)
    assert np.isnan(sim.f[:, ~new]).all()
    rho_keep = sim.f[:, keep].sum(axis=0)
    np.testing.assert_allclose(rho_keep, rho[keep], rtol=1e-15)


def test_refill_without_valid_neighbour_takes_rho0():
    nx, ny = 5, 5
    block = [(x, y) for x in (1, 2, 3) for y in (1, 2, 3)]
    ring = [p for p in block if p != (2, 2)]
    rho0 = 1.07
    sim, dom, rho = _setup(nx, ny, block, rho0, seed=12)
    new = _new_mask(dom, ring)                    # the centre (2,2) = 12 opens, its 8 neighbours are solid
    ub = np.zeros((3, dom.N))
    ub[0], ub[1] = -0.011, 0.004
    fresh = sim.refill(new, ub)
    assert fresh.tolist() == [12]
    np.testing.assert_allclose(sim.f[:, 12], _eq_d2q9(rho0, ub[:, 12]), rtol=0, atol=1e-15)


def test_refill_neighbours_beyond_a_non_periodic_face_excluded():
    nx, ny = 5, 4
    # (2,0) on the -y face is solid at t-1 and fluid at t
    sim, dom, rho = _setup(nx, ny, [(2, 0)], 1.0, seed=13, periodic=(True, False, True))
    sim.refill(np.ones(dom.N, bool), np.zeros((3, dom.N)))
    # neighbours inside the domain (y >= 0): (3,0) (1,0) (2,1) (3,1) (1,1)
    nb = [3, 1, 2 + nx, 3 + nx, 1 + nx]
    np.testing.assert_allclose(sim.f[:, 2], _eq_d2q9(rho[nb].mean(), (0.0, 0.0)), rtol=0, atol=1e-15)


@pytest.mark.parametrize("period", [2000.0, 37.5])
def test_kinematics_velocity_is_derivative_of_centre(period):
    e = np.array([0.36, -0.48, 0.8])
    x0 = np.array([50.0, 61.0, 40.0])
    kin = moving.Kinematics(x0, amplitude=8.0, period=period, direction=e, omega=(0, 0, 0.001))
    h = 1e-4
    for t in np.linspace(0.0, period, 17):
        fd = (kin.centre(t + h) - kin.centre(t - h)) / (2 * h)
        np.testing.assert_allclose(kin.velocity(t), fd, rtol=0, atol=1e-9)
    # closed values: at t = 0 the sphere is at x0 moving at A 2 pi / T along e;
    # a quarter period later it is at x0 + A e and at rest
    np.testing.assert_allclose(kin.centre(0.0), x0, atol=0)
    np.testing.assert_allclose(kin.velocity(0.0), 8.0 * 2 * np.pi / period * e, rtol=1e-15)
    np.testing.assert_allclose(kin.centre(period / 4), x0 + 8.0 * e, rtol=1e-14)
    np.testing.assert_allclose(kin.velocity(period / 4), 0.0, atol=1e-15)
