"""Self-consistency of the oracle's moving-sphere step and zero-gradient outlet
(both "parity unpinned": the paper specifies neither the equilibrium refill nor
open boundaries)."""
import numpy as np

import synth
from oracle import geometry as G, lattice, moving, solver


def test_comoving_uniform_flow_with_moving_sphere_and_refill():
    lat = lattice.D3Q19
    dom = G.Domain(lat, 20, 18, 16)
    U = np.array([0.05, -0.03, 0.02])
    # constant velocity U: amplitude*2pi/T = |U| with a long period, sampled near t=0
    # constant velocity U: amplitude * 2 pi / T = |U| with a period long enough for
    # cos(2 pi t / T) to be 1 to double precision over the run
    kin = moving.Kinematics((9.3, 8.7, 7.9), amplitude=np.linalg.norm(U) * 1e12 / (2 * np.pi),
                            period=1e12, direction=U / np.linalg.norm(U), omega=(0, 0, 0))
    m = moving.MovingSphereSim(dom, 4.2, kin, tau=0.8, rho0=1.1, u0=U)
    fresh_total = 0
    for _ in range(30):
        before = m.sim.fluid.copy()
        m.step()
        fresh_total += (m.sim.fluid & ~before).sum()
        fl = m.sim.fluid
        rho, u = m.sim.macros()
        np.testing.assert_allclose(rho[fl], 1.1, rtol=1e-11)
        np.testing.assert_allclose(u[:, fl], np.repeat(U[:, None], fl.sum(), 1), atol=1e-12)
    assert fresh_total > 0


def test_sampled_path_of_the_sinusoid_reproduces_it():
    """A path given by the sinusoid's own samples drives the same steps: fields
    identical to the bit after 12 steps (fresh nodes included)."""
    lat = lattice.D3Q19
    dom = G.Domain(lat, 22, 20, 18)
    kin = moving.Kinematics((10.4, 9.7, 8.6), amplitude=3.0, period=40.0, direction=(0.6, 0.8, 0.0),
                            omega=(0.002, -0.001, 0.003))
    C = np.array([kin.centre(t) for t in range(14)])
    V = np.array([kin.velocity(t) for t in range(14)])
    path = moving.SampledKinematics(C, V, kin.Omega)
    a = moving.MovingSphereSim(dom, 4.1, kin, tau=0.8)
    b = moving.MovingSphereSim(dom, 4.1, path, tau=0.8)
    a.run(12)
    b.run(12)
    assert np.array_equal(a.sim.fluid, b.sim.fluid)
    assert np.array_equal(a.sim.f, b.sim.f, equal_nan=True)   # solid nodes hold NaN


def test_comoving_uniform_flow_on_a_sampled_straight_path():
    """A sphere carried along a straight sampled path at the velocity of a
    uniform flow, with rotation off, leaves the flow unchanged to round-off,
    fresh nodes included (the path is not the sinusoid's)."""
    lat = lattice.D3Q19
    dom = G.Domain(lat, 20, 18, 16)
    U = np.array([-0.04, 0.025, 0.035])
    n = 27
    C = np.array([(8.8, 9.1, 7.3)]) + np.arange(n)[:, None] * U[None, :]
    path = moving.SampledKinematics(C, np.repeat(U[None, :], n, 0), (0.0, 0.0, 0.0))
    m = moving.MovingSphereSim(dom, 3.9, path, tau=0.7, rho0=1.05, u0=U)
    fresh_total = 0
    for _ in range(n - 2):
        before = m.sim.fluid.copy()
        m.step()
        fresh_total += (m.sim.fluid & ~before).sum()
        fl = m.sim.fluid
        rho, u = m.sim.macros()
        np.testing.assert_allclose(rho[fl], 1.05, rtol=1e-11)
        np.testing.assert_allclose(u[:, fl], np.repeat(U[:, None], fl.sum(), 1), atol=1e-12)
    assert fresh_total > 0


def test_constant_spin_samples_reproduce_the_constant_spin():
    """Angular velocity given per step with every sample equal to a constant
    drives the same steps as the constant: fields identical after 10 steps."""
    lat = lattice.D3Q19
    dom = G.Domain(lat, 22, 20, 18)
    kin = moving.Kinematics((10.4, 9.7, 8.6), amplitude=3.0, period=40.0, direction=(0.6, 0.8, 0.0),
                            omega=(0.002, -0.001, 0.003))
    C = np.array([kin.centre(t) for t in range(12)])
    V = np.array([kin.velocity(t) for t in range(12)])
    a = moving.MovingSphereSim(dom, 4.1, moving.SampledKinematics(C, V, kin.Omega), tau=0.8)
    b = moving.MovingSphereSim(dom, 4.1, moving.SampledKinematics(C, V, np.repeat(kin.Omega[None, :], 12, 0)),
                               tau=0.8)
    a.run(10)
    b.run(10)
    assert np.array_equal(a.sim.f, b.sim.f, equal_nan=True)


def test_sampled_spin_enters_the_wall_velocity_at_its_own_time():
    """An impulsive spin-up about z (Omega(0) = 0, Omega(t >= 1) = W e_z) of a
    resting sphere: the links of the geometry of time 0 carry u_w(0) = 0 and
    u_w(1) = W e_z x r at their wall points, i.e. tangential, of size W times
    the wall point's distance from the axis, and in the sense of the rotation."""
    lat = lattice.D3Q19
    dom = G.Domain(lat, 20, 20, 16)
    n, W = 6, 0.004
    C = np.repeat(np.array([[9.6, 10.3, 7.8]]), n, 0)
    V = np.zeros((n, 3))
    Om = np.zeros((n, 3))
    Om[1:, 2] = W
    m = moving.MovingSphereSim(dom, 4.3, moving.SampledKinematics(C, V, Om), tau=0.8)
    fluid, links, _ = m.geometry(0)
    assert links["node"].size > 0
    assert np.abs(links["uw_t"]).max() == 0.0
    X = dom.coords(links["node"]).astype(np.float64)
    cvec = lat.c[links["dir"]].T.astype(np.float64)
    xw = X - links["q"][None, :] * cvec
    r = xw - C[0][:, None]
    u1 = links["uw_t1"]
    rperp = np.hypot(r[0], r[1])
    np.testing.assert_allclose(np.hypot(u1[0], u1[1]), W * rperp, rtol=1e-12, atol=1e-15)
    assert np.abs(u1[2]).max() == 0.0
    assert np.all(r[0] * u1[0] + r[1] * u1[1] <= 1e-15)        # tangential
    assert np.all(r[0] * u1[1] - r[1] * u1[0] >= -1e-15)       # counter-clockwise about +z
    # one step later both velocities are the spin's
    _, links1, _ = m.geometry(1)
    assert np.abs(links1["uw_t"]).max() > 0.0


def test_reversed_spin_mirrors_the_flow():
    """A sphere spinning up about z with Omega(t) and one spinning with
    -Omega(t), both at rest in a box symmetric under y -> -y about the sphere's
    centre: after 12 steps the second flow is the mirror image of the first
    (u_x even, u_y odd in y)."""
    lat = lattice.D3Q19
    ny = 20
    dom = G.Domain(lat, 18, ny, 14)
    n = 14
    C = np.repeat(np.array([[8.7, (ny - 1) / 2.0, 6.9]]), n, 0)
    V = np.zeros((n, 3))
    Om = np.zeros((n, 3))
    Om[:, 2] = 0.003 * np.minimum(np.arange(n), 5) / 5.0
    a = moving.MovingSphereSim(dom, 3.8, moving.SampledKinematics(C, V, Om), tau=0.8)
    b = moving.MovingSphereSim(dom, 3.8, moving.SampledKinematics(C, V, -Om), tau=0.8)
    a.run(12)
    b.run(12)
    _, ua = a.sim.macros()
    _, ub = b.sim.macros()
    ua = ua.reshape(3, 14, ny, 18)
    ub = ub.reshape(3, 14, ny, 18)
    fl = a.sim.fluid.reshape(14, ny, 18)
    assert np.array_equal(fl, fl[:, ::-1, :])
    assert np.abs(ua[:, fl]).max() > 1e-4
    np.testing.assert_allclose(ub[0][fl], ua[0][:, ::-1, :][fl], atol=1e-15)
    np.testing.assert_allclose(ub[1][fl], -ua[1][:, ::-1, :][fl], atol=1e-15)


def _two_paths(n, U, c_a=(5.2, 6.1, 5.3), c_b=(14.6, 13.4, 10.2)):
    t = np.arange(n)[:, None]
    return (np.asarray(c_a)[None, :] + t * U[None, :], np.asarray(c_b)[None, :] + t * U[None, :])


def test_comoving_uniform_flow_with_two_spheres():
    """Two spheres carried at the velocity of a uniform flow, rotation off, on
    sampled paths: the flow stays uniform to round-off, fresh nodes of both
    spheres included."""
    lat = lattice.D3Q19
    dom = G.Domain(lat, 22, 20, 16)
    U = np.array([0.035, -0.03, 0.025])
    n = 24
    Ca, Cb = _two_paths(n, U)
    Vs = np.repeat(U[None, :], n, 0)
    zero = (0.0, 0.0, 0.0)
    m = moving.MovingSpheresSim(dom, [3.4, 2.9], [moving.SampledKinematics(Ca, Vs, zero),
                                                   moving.SampledKinematics(Cb, Vs, zero)], tau=0.7, rho0=1.05, u0=U)
    fresh = 0
    for _ in range(n - 2):
        prev = m.sim.fluid.copy()
        m.step()
        fresh += int((m.sim.fluid & ~prev).sum())
    assert fresh > 20
    rho, u = m.sim.macros()
    fl = m.sim.fluid
    assert np.abs(u[:, fl] - U[:, None]).max() < 1e-13
    assert np.abs(rho[fl] - 1.05).max() < 1e-13


def test_two_sphere_order_does_not_matter():
    """Spheres that stay apart give the same flow whichever is listed first
    (each link crosses one sphere, each fresh node has one nearest sphere)."""
    lat = lattice.D3Q19
    dom = G.Domain(lat, 22, 20, 16)
    n = 12
    U = np.array([0.02, 0.015, -0.01])
    Ca, Cb = _two_paths(n, U)
    ka = moving.SampledKinematics(Ca, np.repeat(U[None, :], n, 0), (0.0, 0.0, 0.004))
    kb = moving.SampledKinematics(Cb, np.repeat(-U[None, :], n, 0), (0.003, 0.0, 0.0))
    a = moving.MovingSpheresSim(dom, [3.4, 2.9], [ka, kb], tau=0.8)
    b = moving.MovingSpheresSim(dom, [2.9, 3.4], [kb, ka], tau=0.8)
    a.run(10)
    b.run(10)
    assert np.array_equal(a.sim.fluid, b.sim.fluid)
    assert np.array_equal(a.sim.f, b.sim.f, equal_nan=True)
    # each sphere's own force and torque (its links, about its centre) follow it
    assert np.abs(a.sim.last_force).max() > 1e-6
    assert np.array_equal(a.sim.last_force, b.sim.last_force[::-1])
    assert np.array_equal(a.sim.last_torque, b.sim.last_torque[::-1])


def test_mirrored_spheres_have_mirrored_forces():
    """Two spheres mirror images of each other in the plane x = 12 of a periodic
    box, moving and spinning as mirror images: the flow is mirror symmetric, so
    the second sphere's force is the first's with F_x negated, and its torque
    (an axial vector, about its own centre) the first's with T_y and T_z
    negated.  A link counted for the wrong sphere or a torque about the wrong
    centre breaks the symmetry."""
    lat = lattice.D3Q19
    dom = G.Domain(lat, 24, 22, 20)
    n = 10
    t = np.arange(n, dtype=np.float64)[:, None]
    V = np.array([0.02, 0.004, -0.003])
    Ca = np.array([[8.3, 11.1, 9.7]]) + t * V[None, :]
    Cb = Ca * np.array([-1.0, 1.0, 1.0]) + np.array([24.0, 0.0, 0.0])
    Vb = V * np.array([-1.0, 1.0, 1.0])
    Om = np.array([0.002, 0.0015, 0.001])
    ka = moving.SampledKinematics(Ca, np.repeat(V[None, :], n, 0), Om)
    kb = moving.SampledKinematics(Cb, np.repeat(Vb[None, :], n, 0), Om * np.array([1.0, -1.0, -1.0]))
    m = moving.MovingSpheresSim(dom, [2.4, 2.4], [ka, kb], tau=0.8)
    for _ in range(n - 2):
        m.step()
        F, T = m.sim.last_force, m.sim.last_torque
        scale = max(np.abs(F).max(), np.abs(T).max())
        assert scale > 1e-5
        assert np.abs(F[1] - F[0] * np.array([-1.0, 1.0, 1.0])).max() <= 1e-10 * scale
        assert np.abs(T[1] - T[0] * np.array([1.0, -1.0, -1.0])).max() <= 1e-10 * scale


def test_refill_velocity_is_the_nearest_spheres():
    """The refill's body velocity at a point is the rigid-body velocity of the
    sphere whose surface is nearest: hand-placed points next to each sphere."""
    lat = lattice.D3Q19
    dom = G.Domain(lat, 22, 20, 16)
    A = G.Sphere((5.0, 6.0, 5.0), 3.0, True, V=(0.01, 0.0, 0.0), Omega=(0.0, 0.0, 0.002))
    Bs = G.Sphere((15.0, 13.0, 10.0), 2.0, True, V=(0.0, -0.02, 0.0), Omega=(0.001, 0.0, 0.0))
    m = moving.MovingSpheresSim(dom, [3.0], [moving.Kinematics((5.0, 6.0, 5.0), 0.0, 10.0, (1, 0, 0), (0, 0, 0))],
                                tau=0.8)
    X = np.array([[8.5, 6.0, 5.0],      # 0.5 off A's surface, far from B
                  [15.0, 15.5, 10.0],   # 0.5 off B's surface
                  [10.0, 9.0, 8.0]]).T  # between them: |x - cA| - 3 = 3.56, |x - cB| - 2 = 4.92 -> A
    u = m.body_velocity([A, Bs], X)
    # V + Omega x (x - c) of the nearest sphere, written out per point
    np.testing.assert_allclose(u[:, 0], [0.01 - 0.002 * 0.0, 0.0 + 0.002 * 3.5, 0.0], atol=1e-17)
    np.testing.assert_allclose(u[:, 1], [0.0, -0.02 - 0.001 * 0.0, 0.0 + 0.001 * 2.5], atol=1e-17)
    np.testing.assert_allclose(u[:, 2], [0.01 - 0.002 * 3.0, 0.0 + 0.002 * 5.0, 0.0], atol=1e-17)


def test_moving_box_runs_and_conserves_mass_roughly():
    box = synth.moving_boxes(1, side_min=40, side_max=40, r_min=6, r_max=6, period=200)[0]
    lat = lattice.D3Q19
    dom = G.Domain(lat, box["nx"], box["ny"], box["nz"])
    kin = moving.Kinematics(box["x0"], box["amplitude"] / 4, box["period"], box["direction"], box["omega"])
    m = moving.MovingSphereSim(dom, box["radius"], kin, tau=box["tau"])
    m.run(10)
    rho, u = m.sim.macros()
    fl = m.sim.fluid
    assert np.isfinite(rho[fl]).all()
    assert abs(rho[fl].mean() - 1.0) < 1e-3


def test_outlet_is_zero_gradient_on_missing_populations():
    """At the outlet layer every population not covered by a wall link equals the
    same population one node upstream after the step (zero normal gradient)."""
    lat = lattice.D2Q9
    nx, ny, umax = 40, 12, 0.03
    dom = G.Domain(lat, nx, ny, 1, periodic=(False, False, True), outlet_face=1)
    faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(ny, umax)), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5)]
    fluid = np.ones(dom.shape, bool)
    L = G.cut_links(dom, fluid, [], faces)
    sim = solver.Simulation(dom, 0.7)
    sim.set_geometry(fluid, L)
    sim.init_equilibrium()
    sim.run(300)
    f = sim.f.reshape(lat.q, ny, nx)
    cut = set(zip(L["node"].tolist(), L["dir"].tolist()))
    checked = 0
    for i in range(lat.q):
        if lat.c[i][0] != -1:
            continue
        for y in range(ny):
            if ((nx - 1) + nx * y, i) in cut:
                continue
            assert f[i, y, nx - 1] == f[i, y, nx - 2]
            checked += 1
    assert checked == 3 * ny - 2
    # the flow is symmetric about the channel centre line
    rho, u = sim.macros()
    ux = u[0].reshape(ny, nx)
    np.testing.assert_allclose(ux, ux[::-1], rtol=1e-10, atol=1e-15)
