"""Pins of the oracle's link builder: q is the first wall crossing along the
link, normalised by |c_i| (Sec. II.B, eq. bfl and the boundary-node figure)."""
import numpy as np
import pytest

from oracle import geometry as G, lattice, solver


def _bisect_q(dom, sph, xf, c):
    """Reference: bisection on the signed squared distance along the segment."""
    def g(lam):
        p = xf - lam * c
        d = dom.min_image((p - sph.centre)[:, None])[:, 0]
        v = (d * d).sum() - sph.radius ** 2
        return v if sph.solid_inside else -v
    lo, hi = 0.0, 1.0
    assert g(lo) > 0 and g(hi) <= 0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            lo = mid
        else:
            hi = mid
    return hi


@pytest.mark.parametrize("lat", [lattice.D2Q9, lattice.D3Q19], ids=lambda l: l.name)
@pytest.mark.parametrize("inside", [True, False])
def test_sphere_q_matches_bisection(lat, inside):
    nz = 1 if lat.d == 2 else 16
    dom = G.Domain(lat, 18, 17, nz)
    ctr = (8.37, 8.61, 7.93 if lat.d == 3 else 0.0)
    sph = G.Sphere(ctr, 5.3 if inside else 7.2, inside)
    fluid = G.classify(dom, [sph])
    L = G.cut_links(dom, fluid, [sph])
    assert L["node"].size > 50
    X = dom.coords()
    for k in range(0, L["node"].size, max(1, L["node"].size // 40)):
        xf = X[:, L["node"][k]].astype(float)
        c = lat.c[L["dir"][k]].astype(float)
        assert abs(L["q"][k] - _bisect_q(dom, sph, xf, c)) < 1e-12


def test_lattice_points_on_circle_give_q_one():
    dom = G.Domain(lattice.D2Q9, 48, 48, 1)
    inner = G.Sphere((24, 24, 0), 8.0, True)
    fluid = G.classify(dom, [inner]).reshape(-1)
    assert not fluid[32 + 48 * 24]          # (32, 24): r^2 = 64 exactly -> solid
    assert fluid[33 + 48 * 24]
    L = G.cut_links(dom, fluid.reshape(dom.shape), [inner])
    k = np.flatnonzero((L["node"] == 33 + 48 * 24) & (L["dir"] == 1))
    assert k.size == 1 and L["q"][k[0]] == 1.0


@pytest.mark.parametrize("qf", [0.5, 0.25, 0.8])
def test_face_wall_q(qf):
    dom = G.Domain(lattice.D2Q9, 4, 5, 1, periodic=(True, False, True))
    fluid = np.ones(dom.shape, bool)
    L = G.cut_links(dom, fluid, [], [G.FaceWall(2, qf), G.FaceWall(3, qf)])
    np.testing.assert_allclose(L["q"], qf, rtol=1e-15)
    # 3 missing directions on each wall layer of 4 nodes
    assert L["node"].size == 2 * 3 * 4


def test_sphere_wall_velocity_is_rigid_body():
    dom = G.Domain(lattice.D3Q19, 16, 16, 16)
    sph = G.Sphere((7.7, 8.2, 8.1), 4.1, True, V=(0.01, 0.0, -0.02), Omega=(0.001, -0.002, 0.003))
    fluid = G.classify(dom, [sph])
    L = G.cut_links(dom, fluid, [sph])
    X = dom.coords()[:, L["node"]].astype(float)
    xw = X - L["q"] * lattice.D3Q19.c[L["dir"]].T
    r = xw - sph.centre[:, None]
    np.testing.assert_allclose(np.sqrt((r * r).sum(0)), 4.1, rtol=1e-12)
    expect = sph.V[:, None] + np.cross(sph.Omega, r.T).T
    np.testing.assert_allclose(L["uw_t"], expect, atol=1e-15)


def test_channel_with_outlet_is_fully_covered():
    """Inlet, walls and outlet of a small cylinder channel cover every population;
    the outlet corners fall to the walls (cut links with q = 1/2)."""
    lat = lattice.D2Q9
    nx, ny = 30, 12
    dom = G.Domain(lat, nx, ny, 1, periodic=(False, False, True), outlet_face=1)
    cyl = G.Sphere((8.3, 6.1, 0), 2.5, True)
    faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(ny, 0.05)), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5)]
    fluid = G.classify(dom, [cyl])
    L = G.cut_links(dom, fluid, [cyl], faces)
    sim = solver.Simulation(dom, 0.6)
    sim.set_geometry(fluid, L)           # raises if any population is uncovered
    corner = (nx - 1) + nx * 0
    k = np.flatnonzero((L["node"] == corner) & (L["dir"] == 7))   # c = (-1, 1): from (nx, -1)
    assert k.size == 1 and L["q"][k[0]] == 0.5
    assert np.flatnonzero(L["node"] % nx == nx - 1).size == 2 * 3   # corners only: 3 each
    # inlet links carry the parabolic profile at the wall point
    inl = np.flatnonzero((L["node"] % nx == 0) & (L["dir"] == 1))
    y = L["node"][inl] // nx
    np.testing.assert_allclose(L["uw_t"][0, inl], 4 * 0.05 * (y + 0.5) * (ny - 0.5 - y) / ny ** 2, rtol=1e-14)


def _bisect_q_cylinder(dom, cyl, xf, c):
    """Reference for a cylinder along z: bisection on the squared xy-distance."""
    def g(lam):
        p = xf - lam * c
        d = dom.min_image((p - cyl.centre)[:, None])[:, 0]
        v = d[0] * d[0] + d[1] * d[1] - cyl.radius ** 2
        return v if cyl.solid_inside else -v
    lo, hi = 0.0, 1.0
    assert g(lo) > 0 and g(hi) <= 0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            lo = mid
        else:
            hi = mid
    return hi


@pytest.mark.parametrize("lat", [lattice.D3Q19, lattice.D3Q27], ids=lambda l: l.name)
@pytest.mark.parametrize("inside", [True, False])
def test_cylinder_q_matches_bisection(lat, inside):
    dom = G.Domain(lat, 18, 17, 5)
    cyl = G.Cylinder((8.37, 8.61, 2.3), 5.3 if inside else 7.2, inside)
    fluid = G.classify(dom, [cyl])
    L = G.cut_links(dom, fluid, [cyl])
    assert L["node"].size > 50
    X = dom.coords()
    for k in range(0, L["node"].size, max(1, L["node"].size // 60)):
        xf = X[:, L["node"][k]].astype(float)
        c = lat.c[L["dir"][k]].astype(float)
        assert c[0] != 0 or c[1] != 0                  # an axial direction never crosses
        assert abs(L["q"][k] - _bisect_q_cylinder(dom, cyl, xf, c)) < 1e-12


def test_cylinder_layers_equal_the_disk():
    """Every z-layer of a cylinder on D3Q19 is the D2Q9 disk: same fluid nodes,
    and every link's q is the disk's q of the link's in-plane projection; the
    wall moves at |Omega| R."""
    n, nz, R, om = 30, 4, 9.3, 2e-3
    ctr = (14.6, 15.2, 0.0)
    d2 = G.Domain(lattice.D2Q9, n, n, 1)
    disk = G.Sphere(ctr, R, True, Omega=(0, 0, om))
    f2 = G.classify(d2, [disk]).reshape(-1)
    L2 = G.cut_links(d2, f2.reshape(d2.shape), [disk])
    q2 = {(int(nd), tuple(lattice.D2Q9.c[d][:2])): q for nd, d, q in zip(L2["node"], L2["dir"], L2["q"])}
    d3 = G.Domain(lattice.D3Q19, n, n, nz)
    cyl = G.Cylinder(ctr, R, True, Omega=(0, 0, om))
    f3 = G.classify(d3, [cyl]).reshape(nz, n * n)
    for z in range(nz):
        assert np.array_equal(f3[z], f2)
    L3 = G.cut_links(d3, f3.reshape(d3.shape), [cyl])
    assert L3["node"].size > 0
    for nd, d, q in zip(L3["node"], L3["dir"], L3["q"]):
        cxy = tuple(lattice.D3Q19.c[d][:2])
        assert q2[(int(nd) % (n * n), cxy)] == q
    np.testing.assert_allclose(np.linalg.norm(L3["uw_t"], axis=0), om * R, rtol=1e-12)
