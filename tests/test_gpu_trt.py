"""GPU parity of the TRT collision (Sec. II.A, TRT models; Lambda = 3/16 as in
the paper's experiments) against the FP64 oracle, through the C-ABI: the
circular Couette annulus, the cylinder channel with its outlet, a forced random
packing, a moving sphere and a batch mixing BGK and TRT domains."""
import numpy as np
import pytest

import synth
from oracle import geometry as G, lattice as OL, moving
from tests.gpu_cases import Case, annulus_case, channel_case, fluid_velocity_error

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
LAMBDA = 3.0 / 16.0


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_trt_couette(gpu_lib, storage):
    case = annulus_case(magic=LAMBDA)
    _say("case TRT annulus 48x48", storage)
    d, _, _ = case.gpu(gpu_lib, storage)
    sim = case.oracle()
    d.step(3000)
    sim.run(3000)
    err = fluid_velocity_error(d, sim)[0]
    _say("rel L2 velocity", err)
    assert err <= TOL[storage]
    d.close()


@pytest.mark.parametrize("layout", ["compact", "dense"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_trt_packing_with_force(gpu_lib, storage, layout):
    """Forced flow from rest: the velocity after 150 steps is small, and the FP64
    oracle's own rounding noise relative to it scales with 1/|u| (two equivalent
    orderings of the TRT update differ by 3.6e-13 at F = 1e-5 and 3.6e-14 at
    F = 1e-4 on this case), so the force is 1e-4 to keep that floor well below
    the FP64 bar."""
    n = 40
    c, r = synth.sphere_packing(n=n, r_min=3.0, r_max=6.0, solid_fraction=0.4, seed=5)
    case = Case("D3Q19", (n, n, n), spheres=[(cc, rr, True, None, None) for cc, rr in zip(c, r)],
                tau=0.9, force=(1e-4, 2e-5, 0.0), magic=LAMBDA)
    _say("case TRT packing 40^3", storage, layout)
    d, _, _ = case.gpu(gpu_lib, storage, layout=layout)
    sim = case.oracle()
    d.step(150)
    sim.run(150)
    err = fluid_velocity_error(d, sim)[0]
    _say("rel L2 velocity", err)
    assert err <= TOL[storage]
    d.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_trt_channel_outlet(gpu_lib, storage):
    case = channel_case(magic=LAMBDA)
    _say("case TRT channel 200x80", storage)
    d, _, _ = case.gpu(gpu_lib, storage)
    sim = case.oracle()
    d.step(400)
    sim.run(400)
    err = fluid_velocity_error(d, sim)[0]
    _say("rel L2 velocity", err)
    assert err <= TOL[storage]
    d.close()


def test_trt_moving_sphere(gpu_lib):
    B = gpu_lib
    n = 32
    x0, rad, A, T = (15.7, 16.3, 16.1), 5.2, 3.0, 50.0
    e, om = np.array([0.6, -0.48, 0.64]), (0.0015, -0.002, 0.001)
    _say("case TRT moving sphere 32^3 f64")
    d = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage="f64", layout="dense",
                 collision="TRT", magic=LAMBDA)
    d.set_moving_sphere(x0, rad, A, T, e, om)
    m = moving.MovingSphereSim(G.Domain(OL.D3Q19, n, n, n), rad, moving.Kinematics(x0, A, T, e, om), 0.8,
                               magic=LAMBDA)
    d.step(12)
    m.run(12)
    _, u_g, _, unstable = d.macros()
    assert not unstable
    _, u_o = m.sim.macros()
    fl = m.sim.fluid
    err = np.linalg.norm(u_g[fl] - u_o[:, fl].T) / np.linalg.norm(u_o[:, fl])
    _say("rel L2 velocity", err)
    assert err <= 1e-12
    d.close()


def test_batch_mixing_bgk_and_trt(gpu_lib):
    B = gpu_lib
    _say("case batch BGK + TRT")
    mk = [lambda: annulus_case(magic=LAMBDA).gpu(B, "f32")[0], lambda: annulus_case().gpu(B, "f32")[0],
          lambda: channel_case(magic=LAMBDA).gpu(B, "f32")[0], lambda: channel_case().gpu(B, "f32")[0]]
    alone = [m() for m in mk]
    batched = [m() for m in mk]
    b = B.Batch()
    for n in (5, 8):
        for d in alone:
            d.step(n)
        b.step(batched, n)
    for a, c in zip(alone, batched):
        assert np.array_equal(a.get_state(), c.get_state())
    b.close()
    for d in alone + batched:
        d.close()


def test_collision_validation(gpu_lib):
    B = gpu_lib
    m = np.ones(16 * 16, np.uint8)
    with pytest.raises(B.LBMError) as e:
        B.Domain("D2Q9", 16, 16, 1, m, 0.8, collision=7)
    assert e.value.code == B.LBM_EINVAL
    with pytest.raises(B.LBMError) as e:
        B.Domain("D2Q9", 16, 16, 1, m, 0.8, collision="TRT", magic=0.0)
    assert e.value.code == B.LBM_EINVAL
