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
