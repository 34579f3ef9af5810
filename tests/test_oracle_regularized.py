"""Pins of the regularised wall non-equilibrium (eq. fi_neq, App. C) in the oracle.

* Lattice moments of the rebuilt non-equilibrium, for random stresses and
  velocities: zero mass and momentum and a second moment equal to the stress it
  was built from (every lattice, by 4th-order isotropy); third-order Hermite
  moments equal to the recursion's a3 (eq. malaspinas) on the components the
  lattice represents: D2Q9 and D3Q27 are tensor products of D1Q3, so every
  component with no axis taken three times is exact there.  D3Q19 lacks the
  corners and aliases its third-order moments (sum_i w_i H_xxy H_yzz != 0), so
  only the two lower moments are exact on it.
* With walls at rest and a non-equilibrium of pure second-order Hermite form,
  the regularised and the bounce-back estimates coincide link by link (H2 is
  even in c), through a full step of the solver.
* Whole scheme: plane Couette with interpolated walls (q = 0.3, moving top wall)
  is reproduced exactly; circular Couette stays second order with an error close
  to the bounce-back estimate's (the paper finds the two estimators similar at
  low Re); half-way bounce-back uses no wall population and is unchanged.
"""
import itertools

import numpy as np
import pytest

from oracle import analytic, boundary, lattice, metrics, solver
from tests import cases

LATS = [lattice.D2Q9, lattice.D3Q19, lattice.D3Q27]


def _random_case(lat, rng):
    D = lat.d
    A = rng.standard_normal((D, D)) * 1e-3
    Pi = A + A.T
    u = np.zeros(3)
    u[:D] = 0.05 * rng.standard_normal(D)
    i = np.arange(lat.q)
    n = boundary.regularized_neq(lat, i, np.repeat(Pi[None], lat.q, 0), np.repeat(u[:, None], lat.q, 1))
    return Pi, u[:D], n


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_mass_momentum_and_stress(lat):
    rng = np.random.default_rng(3)
    c = lat.c[:, :lat.d].astype(float)
    for _ in range(5):
        Pi, _, n = _random_case(lat, rng)
        assert abs(n.sum()) < 1e-17
        np.testing.assert_allclose(c.T @ n, 0.0, atol=1e-17)
        np.testing.assert_allclose(np.einsum("ia,ib,i->ab", c, c, n), Pi, atol=1e-17)


@pytest.mark.parametrize("lat", [lattice.D2Q9, lattice.D3Q27], ids=lambda l: l.name)
def test_third_order_hermite_moments(lat):
    rng = np.random.default_rng(4)
    D = lat.d
    H3 = boundary.hermite3(lat, np.arange(lat.q))
    for _ in range(5):
        Pi, u, n = _random_case(lat, rng)
        m3 = np.einsum("iabg,i->abg", H3, n)
        for a, b, g in itertools.product(range(D), repeat=3):
            if a == b == g:
                continue           # H_aaa vanishes on the lattice (c^3 = c, cs2 = 1/3)
            want = u[a] * Pi[b, g] + u[b] * Pi[a, g] + u[g] * Pi[a, b]
            assert abs(m3[a, b, g] - want) < 1e-17, (a, b, g)


def test_d3q19_aliases_third_order():
    """The reason D3Q19 is left out above, shown on the lattice itself."""
    lat = lattice.D3Q19
    H3 = boundary.hermite3(lat, np.arange(lat.q))
    cross = (lat.w * H3[:, 0, 0, 1] * H3[:, 1, 2, 2]).sum()
    assert abs(cross + 1.0 / 27.0) < 1e-15      # -cs2^3 where the continuum gives 0


@pytest.mark.parametrize("variant", ["FQ", "F", "U"])
def test_matches_bounce_back_for_second_order_neq_at_rest(variant):
    sim, _, _ = cases.annulus(0.5, u_inner=0.0, variant=variant)
    lat, dom = sim.lat, sim.dom
    rng = np.random.default_rng(5)
    fl = sim.fluid
    N = dom.N
    rho = 1.0 + 0.01 * rng.standard_normal(N)
    u = np.zeros((3, N))
    u[:2] = 0.02 * rng.standard_normal((2, N))
    # pure second-order Hermite non-equilibrium: w_i (c_i.Pi.c_i - cs2 tr Pi) / (2 cs2^2)
    P = 1e-3 * rng.standard_normal((3, N))          # Pi_xx, Pi_yy, Pi_xy
    c = lat.c.astype(float)
    cPc = c[:, :1] ** 2 * P[0] + c[:, 1:2] ** 2 * P[1] + 2 * c[:, :1] * c[:, 1:2] * P[2]
    neq = lat.w[:, None] * (cPc - lat.cs2 * (P[0] + P[1])) / (2 * lat.cs2 ** 2)
    f0 = solver.equilibrium(lat, rho, u) + neq
    f0[:, ~fl] = np.nan
    out = {}
    for wn in boundary.WALL_NEQ:
        sim.set_geometry(fl, sim.links, variant, wall_neq=wn)
        sim.f = f0.copy()
        sim.step()
        out[wn] = sim.f
    n, d = sim.links["node"], sim.links["dir"]
    assert n.size > 0
    np.testing.assert_allclose(out["regularized"][d, n], out["bounceback"][d, n], rtol=0, atol=1e-15)


@pytest.mark.parametrize("q,tau", [(0.3, 0.6), (0.3, 1.5), (0.7, 0.8)])
def test_plane_couette_exact(q, tau):
    ny, U = 8, 0.02
    sim = cases.channel(3, ny, q=q, u_top=(U, 0, 0), tau=tau, wall_neq="regularized")
    # the start-up error decays as exp(-nu pi^2 t / H^2): 10 ny^2 / nu steps take it far below 1e-12
    sim.run(int(10 * ny * ny / ((tau - 0.5) / 3)))
    _, u = sim.macros()
    y = sim.dom.coords()[1].astype(float)
    uth = U * (y + q) / (ny - 1 + 2 * q)
    assert np.abs(u[0] - uth).max() / U < 1e-12


def _couette_rrse(scale, wall_neq, variant="FQ", steps_per_area=3500):
    sim, p, om1 = cases.annulus(scale, variant=variant, wall_neq=wall_neq)
    sim.run(int(steps_per_area * scale * scale))
    _, u = sim.macros()
    X = sim.dom.coords().astype(float)
    fl = sim.fluid
    r = np.hypot(X[0, fl] - p["centre"][0], X[1, fl] - p["centre"][1])
    return metrics.rrse(np.sqrt((u[:, fl] ** 2).sum(0)), analytic.circular_couette(r, p["r1"], p["r2"], om1))


def test_circular_couette_second_order_and_close_to_bounce_back():
    e1 = _couette_rrse(0.75, "regularized")
    e2 = _couette_rrse(1.5, "regularized")
    assert np.log(e1 / e2) / np.log(2.0) > 1.8, (e1, e2)
    eb = _couette_rrse(0.75, "bounceback")
    assert 0.5 < e1 / eb < 1.5


def test_half_way_bounce_back_is_unchanged():
    a = _couette_rrse(0.5, "regularized", "HWBB", 2000)
    b = _couette_rrse(0.5, "bounceback", "HWBB", 2000)
    assert a == b
