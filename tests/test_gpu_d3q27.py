"""GPU parity of the D3Q27 lattice (the paper's 3D lattice, Sec. III) against
the FP64 oracle through the C-ABI: a forced random packing (BGK and TRT with
Lambda = 3/16), a ragged box with sliding walls and a moving-wall sphere (with
the momentum-exchange force per object), a moving sphere rebuilt on the device,
and a batch mixing D3Q27 with D3Q19."""
import numpy as np
import pytest

import synth
from oracle import geometry as G, lattice as OL, moving
from tests.gpu_cases import Case, fluid_velocity_error

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _say(*a):
    print(*a, flush=True)


def _packing(magic=None, force=(1e-4, 2e-5, 0.0)):
    n = 36
    c, r = synth.sphere_packing(n=n, r_min=3.0, r_max=5.5, solid_fraction=0.4, seed=9)
    return Case("D3Q27", (n, n, n), spheres=[(cc, rr, True, None, None) for cc, rr in zip(c, r)],
                tau=0.9, force=force, magic=magic)


@pytest.mark.parametrize("layout", ["compact", "dense"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("magic", [None, 3.0 / 16.0], ids=["BGK", "TRT"])
def test_d3q27_packing(gpu_lib, storage, layout, magic):
    case = _packing(magic)
    _say("case D3Q27 packing 36^3", storage, layout, "TRT" if magic else "BGK")
    d, _, _ = case.gpu(gpu_lib, storage, layout=layout)
    sim = case.oracle()
    d.step(120)
    sim.run(120)
    err = fluid_velocity_error(d, sim)[0]
    _say("rel L2 velocity", err)
    assert err <= TOL[storage]
    d.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_d3q27_ragged_walls_and_force(gpu_lib, storage):
    case = Case("D3Q27", (67, 29, 23), periodic=(True, False, True),
                spheres=[((30.4, 14.2, 11.7), 6.3, True, (0.01, -0.005, 0.002), (0.001, 0.0015, -0.002))],
                faces=[(2, 0.3, None, 0), (3, 0.3, (0.02, 0.0, 0.01), 0)], tau=0.75, rho0=1.02)
    _say("case D3Q27 ragged 67x29x23", storage)
    d, _, links = case.gpu(gpu_lib, storage)
    sim = case.oracle()
    d.set_link_groups(links["shape"], 3)
    sim.set_link_groups(sim.links["shape"], 3)
    d.step(40)
    sim.run(40)
    err = fluid_velocity_error(d, sim)[0]
    ferr = np.abs(d.force() - sim.last_force).max() / np.abs(sim.last_force).max()
    _say("rel L2 velocity", err, "force rel err", ferr)
    assert err <= TOL[storage]
    assert ferr <= (1e-11 if storage == "f64" else 1e-5)
    d.close()


def test_d3q27_moving_sphere(gpu_lib):
    B = gpu_lib
    n = 32
    x0, rad, A, T = (15.7, 16.3, 16.1), 5.2, 3.0, 50.0
    e, om = np.array([0.6, -0.48, 0.64]), (0.0015, -0.002, 0.001)
    _say("case D3Q27 moving sphere 32^3 f64")
    d = B.Domain("D3Q27", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage="f64", layout="dense")
    d.set_moving_sphere(x0, rad, A, T, e, om)
    m = moving.MovingSphereSim(G.Domain(OL.D3Q27, n, n, n), rad, moving.Kinematics(x0, A, T, e, om), 0.8)
    for _ in range(3):
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
    _say("rel L2 velocity", err)
    assert err <= 1e-12
    d.close()


def test_d3q27_in_a_batch(gpu_lib):
    B = gpu_lib
    _say("case batch D3Q27 + D3Q19")
    mk = [lambda: _packing().gpu(B, "f32")[0],
          lambda: Case("D3Q19", (36, 36, 36), spheres=[((18.2, 17.6, 18.9), 7.1, True, None, None)],
                       tau=0.8, force=(1e-5, 0.0, 0.0)).gpu(B, "f32")[0],
          lambda: _packing(3.0 / 16.0).gpu(B, "bf16s", layout="dense")[0]]
    alone, batched = [m() for m in mk], [m() for m in mk]
    b = B.Batch()
    for n in (3, 6):
        for d in alone:
            d.step(n)
        b.step(batched, n)
    for a, c in zip(alone, batched):
        assert np.array_equal(a.get_state(), c.get_state())
    b.close()
    for d in alone + batched:
        d.close()
