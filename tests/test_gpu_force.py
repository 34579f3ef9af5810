"""GPU momentum-exchange force and torque (lbm_set_link_groups,
lbm_momentum_exchange, lbm_force_torque) against the oracle's per-step force
and torque, per object, and the momentum balance of the whole packing at full
size (force on the walls = body force on the fluid minus the change of the
fluid's momentum, from the library's own FP64 sums)."""
import numpy as np
import pytest

from tests.gpu_cases import Case, channel_case

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _force_error(Fg, Fo):
    return np.abs(Fg - Fo).max() / np.abs(Fo).max()


@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 1e-5)])
@pytest.mark.parametrize("layout", ["compact", "dense"])
def test_channel_cylinder_forces_per_object(gpu_lib, storage, tol, layout):
    """Cylinder, inlet, bottom and top walls as four groups (channel with outlet)."""
    case = channel_case()
    _say("case force channel", storage, layout)
    d, mask, links = case.gpu(gpu_lib, storage, layout=layout)
    sim = case.oracle()
    groups = links["shape"]                   # 0 cylinder, 1 inlet, 2 bottom, 3 top
    centres = np.array([[40.3, 40.6, 0.0], [0.0, 40.0, 0.0], [100.0, 0.0, 0.0], [100.0, 80.0, 0.0]])
    d.set_link_groups(groups, 4)
    sim.set_link_groups(sim.links["shape"], 4, centres=centres)
    for n in (1, 60):
        d.step(n)
        sim.run(n)
        Fg, Fo = d.force(), sim.last_force
        err = _force_error(Fg, Fo)
        Fg2, Tg = d.force_torque(centres)
        terr = _force_error(Tg, sim.last_torque)
        _say("step", sim.t, "cylinder force", Fg[0], "torque", Tg[0], "max rel err", err, terr)
        assert err <= tol and terr <= tol
        assert np.array_equal(Fg, Fg2)
    d.close()


@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_moving_walls_force(gpu_lib, storage, tol):
    """Sliding walls (the Galilean term) and a rotating sphere, ragged 3D box."""
    case = Case("D3Q19", (67, 29, 23), periodic=(True, False, True),
                spheres=[((30.4, 14.2, 11.7), 6.3, True, (0.01, -0.005, 0.002), (0.001, 0.0015, -0.002))],
                faces=[(2, 0.3, None, 0), (3, 0.3, (0.02, 0.0, 0.01), 0)], tau=0.75, rho0=1.02)
    _say("case force ragged 3D", storage)
    d, _, links = case.gpu(gpu_lib, storage)
    sim = case.oracle()
    centres = np.array([[30.4, 14.2, 11.7], [33.0, -0.5, 11.0], [33.0, 28.5, 11.0]])
    d.set_link_groups(links["shape"], 3)
    sim.set_link_groups(sim.links["shape"], 3, centres=centres)
    d.step(25)
    sim.run(25)
    err = _force_error(d.force(), sim.last_force)
    F, T = d.force_torque(centres)
    terr = _force_error(T, sim.last_torque)
    _say("max rel err force", err, "torque", terr)
    assert err <= tol and terr <= tol
    d.close()


def test_packing_momentum_balance_full_size(gpu_lib):
    """256^3 packing (the benchmark workload), FP32: each step the walls take
    exactly the body force minus the fluid's momentum gain."""
    from paper_2009_04604_amd import workloads as W
    _say("case force balance packing 256^3")
    d, mask, links = W.packing_domain(256, "f32")
    F = np.array([1e-6, 0.0, 0.0])
    nfl = int(mask.sum())
    d.step(20)
    for _ in range(3):
        p0 = np.array(d.macros(fields=False)[2][1:4])
        d.step(1)
        p1 = np.array(d.macros(fields=False)[2][1:4])
        Fw = d.force()[0]
        bal = nfl * F - (p1 - p0)
        rel = np.abs(Fw - bal).max() / np.abs(bal).max()
        _say("wall force", Fw, "N F - dP", bal, "rel", rel)
        assert rel < 1e-5               # FP32 populations: the sums carry their rounding (6.5e-7 measured)
    d.close()


def test_force_validation(gpu_lib):
    B = gpu_lib
    case = channel_case()
    d, _, links = case.gpu(B, "f32")
    with pytest.raises(B.LBMError) as e:
        d.force()                        # no step yet
    assert e.value.code == B.LBM_ESTATE
    with pytest.raises(B.LBMError) as e:
        d.set_link_groups(np.full(len(links["node"]), 5), 4)
    assert e.value.code == B.LBM_EINVAL
    d.step(2)
    f = d.get_state()
    d.set_state(f)
    with pytest.raises(B.LBMError) as e:
        d.force_torque()                 # no step since the state was set
    assert e.value.code == B.LBM_ESTATE
    d.step(1)
    with pytest.raises(B.LBMError) as e:
        d.force_torque(np.array([[np.nan, 0.0, 0.0]]))
    assert e.value.code == B.LBM_EINVAL
    d.force_torque(np.zeros((1, 3)))
    d.close()
