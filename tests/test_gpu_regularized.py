"""GPU parity of the regularised wall non-equilibrium (eq. fi_neq; the
estimator selected by lbm_set_wall_neq) against the FP64 oracle, through the
C-ABI: the annulus with its rotating inner wall (per-link wall velocities), BGK
and TRT; a forced 3D packing on both layouts and on D3Q27; the channel with its
parabolic inlet and outlet; a moving sphere (wall velocities written by the
device-side link rebuild, alone and batched); a switch of estimator in the
middle of a run; a batch mixing both estimators; the full-size packing in the benchmark configuration;
the 16-bit errors; argument checks."""
import numpy as np
import pytest

import synth
from oracle import geometry as G, lattice as OL, moving, solver
from tests.gpu_cases import Case, annulus_case, channel_case, fluid_velocity_error

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
REG = "regularized"


def _say(*a):
    print(*a, flush=True)


def _compare(B, case, storage, steps, layout="compact", tol=None):
    d, _, _ = case.gpu(B, storage, layout=layout, wall_neq=REG)
    sim = case.oracle(wall_neq=REG)
    d.step(steps)
    sim.run(steps)
    err = fluid_velocity_error(d, sim)[0]
    _say("rel L2 velocity", err)
    d.close()
    assert err <= (TOL[storage] if tol is None else tol)
    return err


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("magic", [None, 3.0 / 16.0], ids=["BGK", "TRT"])
def test_annulus(gpu_lib, storage, magic):
    _say("case regularised annulus 48x48", storage, "TRT" if magic else "BGK")
    _compare(gpu_lib, annulus_case(magic=magic), storage, 2000)


@pytest.mark.parametrize("layout", ["compact", "dense"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_packing_with_force(gpu_lib, storage, layout):
    n = 40
    c, r = synth.sphere_packing(n=n, r_min=3.0, r_max=6.0, solid_fraction=0.4, seed=5)
    case = Case("D3Q19", (n, n, n), spheres=[(cc, rr, True, None, None) for cc, rr in zip(c, r)],
                tau=0.9, force=(1e-4, 2e-5, 0.0))
    _say("case regularised packing 40^3", storage, layout)
    _compare(gpu_lib, case, storage, 150, layout)


def test_packing_d3q27_trt(gpu_lib):
    n = 24
    c, r = synth.sphere_packing(n=n, r_min=2.5, r_max=4.5, solid_fraction=0.35, seed=9)
    case = Case("D3Q27", (n, n, n), spheres=[(cc, rr, True, None, None) for cc, rr in zip(c, r)],
                tau=0.8, force=(1e-4, 0.0, 3e-5), magic=3.0 / 16.0)
    _say("case regularised packing D3Q27 24^3 TRT f64")
    _compare(gpu_lib, case, "f64", 80)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_channel_outlet(gpu_lib, storage):
    _say("case regularised channel 200x80", storage)
    _compare(gpu_lib, channel_case(), storage, 400)


def test_moving_sphere(gpu_lib):
    B = gpu_lib
    n = 32
    x0, rad, A, T = (15.7, 16.3, 16.1), 5.2, 3.0, 50.0
    e, om = np.array([0.6, -0.48, 0.64]), (0.0015, -0.002, 0.001)
    _say("case regularised moving sphere 32^3 f64")
    d = B.Domain("D3Q19", n, n, n, np.ones(n ** 3, np.uint8), 0.8, storage="f64", layout="dense")
    d.set_wall_neq(REG)
    d.set_moving_sphere(x0, rad, A, T, e, om)
    m = moving.MovingSphereSim(G.Domain(OL.D3Q19, n, n, n), rad, moving.Kinematics(x0, A, T, e, om), 0.8,
                               wall_neq=REG)
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


def test_switch_in_the_middle_of_a_run(gpu_lib):
    _say("case annulus f64: 300 steps bounce-back, 300 regularised, 300 bounce-back")
    case = annulus_case()
    d, _, _ = case.gpu(gpu_lib, "f64")
    sim = case.oracle()
    for mode in ("bounceback", REG, "bounceback"):
        d.set_wall_neq(mode)
        sim.set_geometry(sim.fluid, sim.links, sim.variant, sim.q_cut, wall_neq=mode)
        d.step(300)
        sim.run(300)
    err = fluid_velocity_error(d, sim)[0]
    _say("rel L2 velocity", err)
    d.close()
    assert err <= 1e-12


def test_batch_mixing_estimators(gpu_lib):
    B = gpu_lib
    _say("case batch bounce-back + regularised")
    mk = [lambda: annulus_case().gpu(B, "f32", wall_neq=REG)[0], lambda: annulus_case().gpu(B, "f32")[0],
          lambda: channel_case().gpu(B, "f32", wall_neq=REG)[0], lambda: channel_case().gpu(B, "f32")[0]]
    alone = [m() for m in mk]
    batched = [m() for m in mk]
    b = B.Batch()
    for n in (5, 8):
        for d in alone:
            d.step(n)
        b.step(batched, n)
    # a member switching estimator is picked up by the batch
    alone[1].set_wall_neq(REG)
    batched[1].set_wall_neq(REG)
    for d in alone:
        d.step(6)
    b.step(batched, 6)
    for a, c in zip(alone, batched):
        assert np.array_equal(a.get_state(), c.get_state())
    b.close()
    for d in alone + batched:
        d.close()


def test_moving_batch_mixing_estimators(gpu_lib):
    """Moving spheres with the regularised estimator in a batch (the batched link
    rebuild writes the wall velocities) end bit-identical to the same boxes
    stepped alone, next to a box with the bounced estimator."""
    from paper_2009_04604_amd import workloads as W
    B = gpu_lib
    _say("case moving batch, regularised + bounce-back")
    boxes = synth.moving_boxes(n_boxes=3, side_min=40, side_max=56, r_min=5.0, r_max=7.0, amplitude=4.0,
                               period=120.0, seed=5)
    modes = [REG, REG, "bounceback"]
    alone = [W.moving_box_domain(bx, storage="f32", wall_neq=m) for bx, m in zip(boxes, modes)]
    batched = [W.moving_box_domain(bx, storage="f32", wall_neq=m) for bx, m in zip(boxes, modes)]
    b = B.Batch()
    for n in (3, 300):               # 300 crosses a kinematics upload chunk
        for d in alone:
            d.step(n)
        b.step(batched, n)
        for a, c in zip(alone, batched):
            assert np.array_equal(a.get_state(), c.get_state())
    b.close()
    for d in alone + batched:
        d.close()


def test_full_size_packing_256_f32_one_step(gpu_lib):
    from paper_2009_04604_amd import workloads as W
    n = 256
    c, r = synth.sphere_packing(n=n)
    _say("case regularised packing 256^3 f32")
    d, mask, links = W.packing_domain(n, "f32", spheres=(c, r), wall_neq=REG)
    d.step(20)
    f0 = d.get_state()
    d.step(1)
    f1 = d.get_state()
    d.close()
    dom = G.Domain(OL.D3Q19, n, n, n)
    sh = [G.Sphere(cc, rr, True) for cc, rr in zip(c, r)]
    fluid = G.classify(dom, sh)
    rng = np.random.default_rng(7)
    fl = np.flatnonzero(mask)
    bn = np.unique(links["node"])
    z = bn // (n * n)
    nodes = np.unique(np.concatenate([rng.choice(fl, 20000, replace=False), bn[(z == 0) | (z == 97)]]))
    sub = G.cut_links(dom, fluid, sh, nodes=nodes)
    out = solver.step_at(dom, f0, fluid, sub, nodes, 0.9, force=(1e-6, 0.0, 0.0), wall_neq=REG)
    got = f1[:, nodes]
    err = np.abs(got - out).max()
    rel = np.linalg.norm(got - out) / np.linalg.norm(out)
    _say("max |df|", err, "rel L2", rel, "nodes", nodes.size)
    assert np.isfinite(out).all() and err <= 1e-6 and rel <= 1e-6


@pytest.mark.parametrize("storage,bound", [("f16s", 1e-3), ("bf16s", 1e-2), ("f16s-sr", 1e-3), ("bf16s-sr", 1e-2)])
def test_16bit_error_stated(gpu_lib, storage, bound):
    _say("case regularised annulus 48x48", storage)
    err = _compare(gpu_lib, annulus_case(), storage, 2000, tol=bound)
    _say("16-bit error against the FP64 oracle", storage, err)


def test_validation(gpu_lib):
    B = gpu_lib
    d = B.Domain("D3Q19", 16, 16, 16, np.ones(16 ** 3, np.uint8), 0.8, layout="dense")
    with pytest.raises(B.LBMError) as e:
        d.set_wall_neq(2)
    assert e.value.code == B.LBM_EINVAL
    d.set_moving_sphere((8.0, 8.0, 8.0), 3.0, 0.0, 10.0, (1.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    with pytest.raises(B.LBMError) as e:
        d.set_wall_neq(REG)
    assert e.value.code == B.LBM_ESTATE
    d.close()
