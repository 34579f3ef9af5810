"""GPU parity of the moving-sphere path (device link rebuild every step, equilibrium
refill of fresh nodes, slot-mode boundary writes) against the oracle's
MovingSphereSim on the same kinematics."""
import numpy as np
import pytest

from oracle import geometry as G, lattice as OL, moving

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _case(n=40):
    return dict(x0=(19.7, 20.3, 20.1), radius=6.2, amplitude=4.0, period=60.0,
                direction=np.array([0.6, -0.48, 0.64]), omega=(0.0015, -0.002, 0.001), tau=0.8, n=n)


def _oracle(c):
    n = c["n"]
    dom = G.Domain(OL.D3Q19, n, n, n)
    kin = moving.Kinematics(c["x0"], c["amplitude"], c["period"], c["direction"], c["omega"])
    return moving.MovingSphereSim(dom, c["radius"], kin, c["tau"])


def _gpu(B, c, storage):
    n = c["n"]
    d = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), c["tau"], storage=storage, layout="dense")
    d.set_moving_sphere(c["x0"], c["radius"], c["amplitude"], c["period"], c["direction"], c["omega"])
    return d


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_moving_sphere_matches_oracle(gpu_lib, storage, tol):
    c = _case()
    _say("case moving sphere 40^3", storage)
    d = _gpu(gpu_lib, c, storage)
    m = _oracle(c)
    fresh_seen = 0
    for block in range(6):
        d.step(5)
        before = m.sim.fluid.copy()
        for _ in range(5):
            prev = m.sim.fluid.copy()
            m.step()
            fresh_seen += int((m.sim.fluid & ~prev).sum())
        info = d.info()
        # geometry of the current time: identical fluid set and link count
        assert info["n_fluid"] == int(m.sim.fluid.sum())
        assert info["n_links"] == m.sim.links["node"].size
        rho_g, u_g, _, unstable = d.macros()
        assert not unstable
        rho_o, u_o = m.sim.macros()
        fl = m.sim.fluid
        err = np.linalg.norm(u_g[fl] - u_o[:, fl].T) / np.linalg.norm(u_o[:, fl])
        _say("t", m.t, "rel L2 velocity", err)
        assert err <= tol
        np.testing.assert_allclose(rho_g[fl], rho_o[fl], rtol=10 * tol, atol=0)
    assert fresh_seen > 0
    d.close()


def test_moving_sphere_requires_dense_periodic(gpu_lib):
    B = gpu_lib
    c = _case(24)
    n = 24
    d = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage="f32")   # compact
    with pytest.raises(B.LBMError) as e:
        d.set_moving_sphere((12, 12, 12), 3.0, 1.0, 50.0, (1, 0, 0), (0, 0, 0))
    assert e.value.code == B.LBM_ESTATE
    d.close()
    d = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage="f32", layout="dense")
    with pytest.raises(B.LBMError) as e:
        d.set_moving_sphere((12, 12, 12), 9.0, 4.0, 50.0, (1, 0, 0), (0, 0, 0))   # sweep too large
    assert e.value.code == B.LBM_EINVAL
    d.close()


@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_moving_sphere_force_and_torque_match_oracle(gpu_lib, storage, tol):
    """Force and torque on the moving sphere (momentum exchange over the links of
    the geometry each step used, taken before the rebuild) against the oracle's
    per-step force and torque about the sphere centre."""
    B = gpu_lib
    c = _case()
    _say("case moving sphere force 40^3", storage)
    d = _gpu(B, c, storage)
    d.set_force_tracking(True)
    with pytest.raises(B.LBMError) as e:
        d.moving_force()                                  # no step with tracking yet
    assert e.value.code == B.LBM_ESTATE
    m = _oracle(c)
    for n in (1, 7, 12):
        d.step(n)
        m.run(n)
        F, T = d.moving_force()
        Fo, To = m.sim.last_force[0], m.sim.last_torque[0]
        ferr = np.abs(F - Fo).max() / np.abs(Fo).max()
        terr = np.abs(T - To).max() / np.abs(To).max()
        _say("t", m.t, "force", F, "torque", T, "rel err", ferr, terr)
        assert ferr <= tol and terr <= tol
    d.close()
    static = B.Domain("D3Q19", 16, 16, 16, np.ones(16 ** 3, np.uint8), 0.8, storage="f32")
    with pytest.raises(B.LBMError) as e:
        static.set_force_tracking(True)                   # static links: lbm_force_torque
    assert e.value.code == B.LBM_ESTATE
    static.close()


def _circle_path(n_samples, c0=(20.2, 19.6, 20.4), R=3.5, period=50.0):
    """A sphere carried round a circle in a tilted plane: samples of the centre
    and of its velocity (the exact derivative) per step."""
    t = np.arange(n_samples, dtype=np.float64)
    w = 2.0 * np.pi / period
    e1 = np.array([1.0, 0.0, 0.0])
    e2 = np.array([0.0, 0.8, 0.6])
    C = np.asarray(c0)[None, :] + R * (np.cos(w * t)[:, None] * e1 + np.sin(w * t)[:, None] * e2)
    V = R * w * (-np.sin(w * t)[:, None] * e1 + np.cos(w * t)[:, None] * e2)
    return C, V


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_sampled_path_matches_oracle(gpu_lib, storage, tol):
    """lbm_set_moving_sphere_path: a circular path (not the sinusoid) against the
    oracle driven by the same samples; identical fluid and link sets."""
    B = gpu_lib
    n, steps = 40, 30
    C, V = _circle_path(steps + 2)
    om = (0.001, 0.002, -0.0015)
    _say("case sampled circular path 40^3", storage)
    d = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage=storage, layout="dense")
    d.set_moving_sphere_path(5.7, om, C, V)
    m = moving.MovingSphereSim(G.Domain(OL.D3Q19, n, n, n), 5.7, moving.SampledKinematics(C, V, om), 0.8)
    fresh_seen = 0
    for block in range(6):
        d.step(5)
        for _ in range(5):
            prev = m.sim.fluid.copy()
            m.step()
            fresh_seen += int((m.sim.fluid & ~prev).sum())
        info = d.info()
        assert info["n_fluid"] == int(m.sim.fluid.sum())
        assert info["n_links"] == m.sim.links["node"].size
        _, u_g, _, unstable = d.macros()
        assert not unstable
        _, u_o = m.sim.macros()
        fl = m.sim.fluid
        err = np.linalg.norm(u_g[fl] - u_o[:, fl].T) / np.linalg.norm(u_o[:, fl])
        _say("t", m.t, "rel L2 velocity", err)
        assert err <= tol
    assert fresh_seen > 0
    # the path is used up: a further step is refused, the state stays
    with pytest.raises(B.LBMError) as e:
        d.step(1)
    assert e.value.code == B.LBM_ESTATE
    assert d.info()["steps_done"] == steps
    d.close()


@pytest.mark.parametrize("storage", ["f32", "bf16s-sr"])
def test_sampled_sinusoid_equals_parametric_motion(gpu_lib, storage):
    """The sinusoid's own samples through lbm_set_moving_sphere_path give, to the
    bit, what lbm_set_moving_sphere gives, alone and in a batch; a batch call
    longer than a member's path is refused."""
    B = gpu_lib
    c = _case()
    n, steps = c["n"], 40
    kin = moving.Kinematics(c["x0"], c["amplitude"], c["period"], c["direction"], c["omega"])
    C = np.array([kin.centre(t) for t in range(steps + 2)])
    V = np.array([kin.velocity(t) for t in range(steps + 2)])

    def path_domain():
        d = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), c["tau"], storage=storage, layout="dense")
        d.set_moving_sphere_path(c["radius"], c["omega"], C, V)
        return d
    a = _gpu(B, c, storage)
    p = path_domain()
    q = path_domain()
    a.step(steps)
    p.step(steps)
    b = B.Batch()
    b.step([q], 25)
    with pytest.raises(B.LBMError) as e:
        b.step([q], steps - 25 + 1)
    assert e.value.code == B.LBM_ESTATE
    b.step([q], steps - 25)
    b.close()
    fa, fp, fq = a.get_state(), p.get_state(), q.get_state()
    assert np.array_equal(fa, fp) and np.array_equal(fa, fq)
    for d in (a, p, q):
        d.close()


def _spin_up(n_samples, W=0.004, ramp=8):
    """Angular velocity per step: a tilted axis whose spin ramps up over `ramp`
    steps from rest."""
    t = np.arange(n_samples, dtype=np.float64)
    Om = np.zeros((n_samples, 3))
    Om[:, 0] = 0.25 * W * np.minimum(t, ramp) / ramp
    Om[:, 2] = W * np.minimum(t, ramp) / ramp
    return Om


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_sampled_spin_matches_oracle(gpu_lib, storage, tol):
    """lbm_set_moving_sphere_motion: the circular path with an angular velocity
    that spins up from rest, against the oracle driven by the same samples."""
    B = gpu_lib
    n, steps = 40, 30
    C, V = _circle_path(steps + 2)
    Om = _spin_up(steps + 2)
    _say("case sampled spin-up on a circular path 40^3", storage)
    d = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage=storage, layout="dense")
    d.set_moving_sphere_motion(5.7, C, V, Om)
    m = moving.MovingSphereSim(G.Domain(OL.D3Q19, n, n, n), 5.7, moving.SampledKinematics(C, V, Om), 0.8)
    for block in range(6):
        d.step(5)
        m.run(5)
        info = d.info()
        assert info["n_fluid"] == int(m.sim.fluid.sum())
        assert info["n_links"] == m.sim.links["node"].size
        _, u_g, _, unstable = d.macros()
        assert not unstable
        _, u_o = m.sim.macros()
        fl = m.sim.fluid
        err = np.linalg.norm(u_g[fl] - u_o[:, fl].T) / np.linalg.norm(u_o[:, fl])
        _say("t", m.t, "rel L2 velocity", err)
        assert err <= tol
    with pytest.raises(B.LBMError) as e:
        d.step(1)
    assert e.value.code == B.LBM_ESTATE
    d.close()


@pytest.mark.parametrize("storage", ["f32", "bf16s-sr"])
def test_constant_spin_samples_equal_the_path_form(gpu_lib, storage):
    """A sampled spin whose samples all equal the constant gives, to the bit,
    what lbm_set_moving_sphere_path gives; a sampled spin-up gives the same
    alone and in a batch."""
    B = gpu_lib
    n, steps = 40, 24
    C, V = _circle_path(steps + 2)
    om = np.array([0.001, 0.002, -0.0015])

    def dom():
        return B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage=storage, layout="dense")
    p = dom()
    p.set_moving_sphere_path(5.7, om, C, V)
    q = dom()
    q.set_moving_sphere_motion(5.7, C, V, np.repeat(om[None, :], steps + 2, 0))
    a = dom()
    a.set_moving_sphere_motion(5.7, C, V, _spin_up(steps + 2))
    b = dom()
    b.set_moving_sphere_motion(5.7, C, V, _spin_up(steps + 2))
    p.step(steps)
    q.step(steps)
    a.step(steps)
    bt = B.Batch()
    bt.step([b], 10)
    bt.step([b], steps - 10)
    bt.close()
    assert np.array_equal(p.get_state(), q.get_state())
    fa, fb = a.get_state(), b.get_state()
    assert np.array_equal(fa, fb)
    assert not np.array_equal(fa, p.get_state())
    for d in (p, q, a, b):
        d.close()


def test_sampled_spin_validation(gpu_lib):
    B = gpu_lib
    n = 24
    C, V = _circle_path(10, c0=(12.0, 12.0, 12.0), R=2.0)
    Om = _spin_up(10)
    Om[4, 1] = np.inf
    d = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage="f32", layout="dense")
    with pytest.raises(B.LBMError) as e:
        d.set_moving_sphere_motion(3.0, C, V, Om)
    assert e.value.code == B.LBM_EINVAL
    with pytest.raises(ValueError):
        d.set_moving_sphere_motion(3.0, C, V, Om[:5])
    d.set_moving_sphere_motion(3.0, C, V, _spin_up(10))
    with pytest.raises(B.LBMError) as e:      # once per domain
        d.set_moving_sphere_motion(3.0, C, V, _spin_up(10))
    assert e.value.code == B.LBM_ESTATE
    d.close()


def _two_sphere_paths(n_samples):
    """Sphere A round the tilted circle, sphere B along a straight line, both
    spinning; [n, 2, 3] arrays of centres, velocities and angular velocities."""
    C_a, V_a = _circle_path(n_samples, c0=(12.2, 13.6, 14.4), R=3.0)
    t = np.arange(n_samples, dtype=np.float64)[:, None]
    U = np.array([-0.05, 0.03, 0.04])
    C_b = np.array([[28.3, 26.9, 25.1]]) + t * U[None, :]
    V_b = np.repeat(U[None, :], n_samples, 0)
    Om_a = _spin_up(n_samples)
    Om_b = np.repeat(np.array([[0.0, -0.003, 0.001]]), n_samples, 0)
    return (np.stack([C_a, C_b], 1), np.stack([V_a, V_b], 1), np.stack([Om_a, Om_b], 1))


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_two_spheres_match_oracle(gpu_lib, storage, tol):
    """lbm_set_moving_spheres: two spheres on different paths with different
    spins in one 40^3 box against the oracle; identical fluid and link sets."""
    B = gpu_lib
    n, steps = 40, 30
    C, V, Om = _two_sphere_paths(steps + 2)
    radii = [5.2, 4.1]
    _say("case two moving spheres 40^3", storage)
    d = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage=storage, layout="dense")
    d.set_moving_spheres(radii, C, V, Om)
    m = moving.MovingSpheresSim(G.Domain(OL.D3Q19, n, n, n), radii,
                                [moving.SampledKinematics(C[:, s], V[:, s], Om[:, s]) for s in range(2)], 0.8)
    fresh = 0
    for block in range(6):
        d.step(5)
        for _ in range(5):
            prev = m.sim.fluid.copy()
            m.step()
            fresh += int((m.sim.fluid & ~prev).sum())
        info = d.info()
        assert info["n_fluid"] == int(m.sim.fluid.sum())
        assert info["n_links"] == m.sim.links["node"].size
        _, u_g, _, unstable = d.macros()
        assert not unstable
        _, u_o = m.sim.macros()
        fl = m.sim.fluid
        err = np.linalg.norm(u_g[fl] - u_o[:, fl].T) / np.linalg.norm(u_o[:, fl])
        _say("t", m.t, "rel L2 velocity", err)
        assert err <= tol
    assert fresh > 0
    d.close()


@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_two_sphere_forces_match_oracle(gpu_lib, storage, tol):
    """Force tracking with two spheres: each link counts for the sphere holding
    its solid node, torques about that sphere's centre; per-sphere force and
    torque against the oracle's link groups, and a one-sphere list against the
    one-sphere call."""
    B = gpu_lib
    n, steps = 40, 16
    C, V, Om = _two_sphere_paths(steps + 2)
    radii = [5.2, 4.1]
    _say("case two moving spheres force 40^3", storage)
    d = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage=storage, layout="dense")
    d.set_moving_spheres(radii, C, V, Om)
    d.set_force_tracking(True)
    m = moving.MovingSpheresSim(G.Domain(OL.D3Q19, n, n, n), radii,
                                [moving.SampledKinematics(C[:, s], V[:, s], Om[:, s]) for s in range(2)], 0.8)
    for k in (1, 6, 9):
        d.step(k)
        m.run(k)
        F, T = d.moving_forces(2)
        Fo, To = m.sim.last_force, m.sim.last_torque
        for sp in range(2):
            ferr = np.abs(F[sp] - Fo[sp]).max() / np.abs(Fo[sp]).max()
            terr = np.abs(T[sp] - To[sp]).max() / np.abs(To[sp]).max()
            _say("t", m.t, "sphere", sp, "force", F[sp], "torque", T[sp], "rel err", ferr, terr)
            assert ferr <= tol and terr <= tol
    d.close()
    one = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage=storage, layout="dense")
    ref = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage=storage, layout="dense")
    one.set_moving_spheres(radii[:1], C[:, :1], V[:, :1], Om[:, :1])
    ref.set_moving_sphere_motion(radii[0], C[:, 0], V[:, 0], Om[:, 0])
    for x in (one, ref):
        x.set_force_tracking(True)
        x.step(5)
    F1, T1 = one.moving_forces(1)
    F0, T0 = ref.moving_force()
    assert np.array_equal(F1[0], F0) and np.array_equal(T1[0], T0)
    one.close()
    ref.close()


@pytest.mark.parametrize("storage", ["f32", "bf16s-sr"])
def test_sphere_lists_equal_single_forms_and_batches(gpu_lib, storage):
    """A one-sphere list equals lbm_set_moving_sphere_motion to the bit; a
    two-sphere domain gives the same alone and in a batch beside a one-sphere
    domain."""
    B = gpu_lib
    n, steps = 40, 20
    C, V, Om = _two_sphere_paths(steps + 2)

    def dom():
        return B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage=storage, layout="dense")
    a = dom()
    a.set_moving_sphere_motion(5.2, C[:, 0], V[:, 0], Om[:, 0])
    b = dom()
    b.set_moving_spheres([5.2], C[:, :1], V[:, :1], Om[:, :1])
    two = dom()
    two.set_moving_spheres([5.2, 4.1], C, V, Om)
    two_b = dom()
    two_b.set_moving_spheres([5.2, 4.1], C, V, Om)
    one_b = dom()
    one_b.set_moving_sphere_motion(5.2, C[:, 0], V[:, 0], Om[:, 0])
    a.step(steps)
    b.step(steps)
    two.step(steps)
    bt = B.Batch()
    bt.step([two_b, one_b], 7)
    bt.step([two_b, one_b], steps - 7)
    bt.close()
    fa = a.get_state()
    assert np.array_equal(fa, b.get_state())
    assert np.array_equal(fa, one_b.get_state())
    assert np.array_equal(two.get_state(), two_b.get_state())
    assert not np.array_equal(fa, two.get_state())
    for d in (a, b, two, two_b, one_b):
        d.close()


def test_sphere_list_validation(gpu_lib):
    B = gpu_lib
    n = 40
    C, V, Om = _two_sphere_paths(8)

    def dom():
        return B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage="f32", layout="dense")
    d = dom()
    close = C.copy()
    close[:, 1] = close[:, 0] + np.array([5.2 + 4.1 + 1.5, 0.0, 0.0])   # surfaces 1.5 apart
    with pytest.raises(B.LBMError) as e:
        d.set_moving_spheres([5.2, 4.1], close, V, Om)
    assert e.value.code == B.LBM_EINVAL
    five = np.concatenate([C, C, C[:, :1]], 1)
    with pytest.raises(B.LBMError) as e:
        d.set_moving_spheres([2.0] * 5, five, np.zeros_like(five), np.zeros_like(five))
    assert e.value.code == B.LBM_EINVAL
    with pytest.raises(ValueError):
        d.set_moving_spheres([5.2, 4.1], C, V, Om[:, :1])
    d.set_moving_spheres([5.2, 4.1], C, V, Om)
    d.set_force_tracking(True)
    d.step(1)
    with pytest.raises(B.LBMError) as e:       # two spheres: the per-sphere form
        d.moving_force()
    assert e.value.code == B.LBM_EINVAL
    with pytest.raises(B.LBMError) as e:
        d.moving_forces(3)
    assert e.value.code == B.LBM_EINVAL
    F, T = d.moving_forces(2)
    assert np.isfinite(F).all() and np.isfinite(T).all()
    # the spheres are set once (the force scratch is sized by their link capacity)
    with pytest.raises(B.LBMError) as e:
        d.set_moving_spheres([6.5, 5.5], C, V, Om)
    assert e.value.code == B.LBM_ESTATE
    d.step(1)
    F2, T2 = d.moving_forces(2)
    assert np.isfinite(F2).all() and np.isfinite(T2).all()
    d.close()


def test_sampled_path_validation(gpu_lib):
    B = gpu_lib
    n = 24
    C, V = _circle_path(10, c0=(12.0, 12.0, 12.0), R=2.0)

    def fresh(layout="dense"):
        return B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage="f32", layout=layout)
    for args, code in [((3.0, (0, 0, 0), C[:1], V[:1]), B.LBM_EINVAL),          # one sample
                       ((0.0, (0, 0, 0), C, V), B.LBM_EINVAL),                  # radius
                       ((3.0, (0, 0, 0), C + np.array([0, 0, 1e300 * 1e10]), V), B.LBM_EINVAL),   # non-finite
                       ((10.5, (0, 0, 0), C, V), B.LBM_EINVAL)]:                # sweep too large for the box
        d = fresh()
        with pytest.raises(B.LBMError) as e:
            d.set_moving_sphere_path(*args)
        assert e.value.code == code
        d.close()
    d = fresh("compact")
    with pytest.raises(B.LBMError) as e:
        d.set_moving_sphere_path(3.0, (0, 0, 0), C, V)
    assert e.value.code == B.LBM_ESTATE
    d.close()
