"""The fixed-density (pressure) outlet through the C-ABI: parity of the cylinder
channel with the oracle (FP64, FP32); bounded mass over a long run where the
zero-gradient outlet lets it grow; a batch mixing both outlets bit-identical to
stepping alone; one full-size step (2048 x 1024, FP32) against the oracle's
node-wise step including the outlet column; argument checks."""
import numpy as np
import pytest

import synth
from oracle import geometry as G, lattice as OL, solver

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _say(*a):
    print(*a, flush=True)


def _oracle(p, nodes_fluid=None):
    nx, ny = p["nx"], p["ny"]
    dom = G.Domain(OL.D2Q9, nx, ny, 1, periodic=(False, False, True))
    cyl = G.Sphere(p["centre"], p["radius"], True)
    faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(ny, p["u_max"])), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5),
             G.PressureFace(1)]
    return dom, cyl, faces


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_pressure_outlet_channel_parity(gpu_lib, storage):
    from paper_2009_04604_amd import workloads as W
    p = synth.cylinder_channel(nx=200, ny=80, radius=6.0, centre=(40.3, 40.6), tau=0.6)
    _say("case pressure-outlet channel 200x80", storage)
    d, mask, links = W.channel_domain(p, storage, outlet="pressure")
    assert (links["q"] == 0.0).sum() > 0
    dom, cyl, faces = _oracle(p)
    fluid = G.classify(dom, [cyl])
    sim = solver.Simulation(dom, p["tau"], rho_out=1.0)
    sim.set_geometry(fluid, G.cut_links(dom, fluid, [cyl], faces), "FQ")
    sim.init_equilibrium()
    d.step(400)
    sim.run(400)
    _, u_g, _, unstable = d.macros()
    assert not unstable
    _, u_o = sim.macros()
    fl = sim.fluid
    err = np.linalg.norm(u_g[fl] - u_o[:2, fl].T) / np.linalg.norm(u_o[:2, fl])
    _say("rel L2 velocity", err)
    d.close()
    assert err <= TOL[storage]


def test_pressure_outlet_keeps_mass_bounded(gpu_lib):
    from paper_2009_04604_amd import workloads as W
    # viscous development over the height takes ~ny^2/nu = 5760 steps here
    p = synth.cylinder_channel(nx=120, ny=24, radius=3.0, centre=(30.0, 12.0), u_max=0.02, tau=0.8)
    masses = {}
    for outlet in ("pressure", "zero-gradient"):
        d, _, _ = W.channel_domain(p, "f64", outlet=outlet)
        d.step(40000)
        m1 = d.macros(fields=False)[2][0]
        d.step(10000)
        m2 = d.macros(fields=False)[2][0]
        d.close()
        masses[outlet] = (m1, m2)
        _say(outlet, "mass after 40000 and 50000 steps", m1, m2)
    m1, m2 = masses["pressure"]
    assert abs(m2 / m1 - 1.0) < 1e-8
    m1, m2 = masses["zero-gradient"]
    assert m2 / m1 - 1.0 > 10 * abs(masses["pressure"][1] / masses["pressure"][0] - 1.0)


def test_batch_mixing_outlets(gpu_lib):
    from paper_2009_04604_amd import workloads as W
    B = gpu_lib
    p = synth.cylinder_channel(nx=160, ny=64, radius=5.0, centre=(40.0, 32.0), tau=0.6)
    mk = [lambda: W.channel_domain(p, "f32", outlet="pressure")[0],
          lambda: W.channel_domain(p, "f32")[0],
          lambda: W.channel_domain(p, "f16s", outlet="pressure", rho_out=1.01)[0]]
    alone = [m() for m in mk]
    batched = [m() for m in mk]
    b = B.Batch()
    for n in (5, 8):
        for d in alone:
            d.step(n)
        b.step(batched, n)
    alone[0].set_outlet_density(0.99)       # a changed density is picked up by the batch
    batched[0].set_outlet_density(0.99)
    for d in alone:
        d.step(6)
    b.step(batched, 6)
    for a, c in zip(alone, batched):
        assert np.array_equal(a.get_state(), c.get_state())
    b.close()
    for d in alone + batched:
        d.close()


def test_pressure_outlet_full_size_one_step(gpu_lib):
    from paper_2009_04604_amd import workloads as W
    p = synth.cylinder_channel()
    _say("case pressure-outlet channel 2048x1024 f32")
    d, mask, links = W.channel_domain(p, "f32", outlet="pressure")
    d.step(60)
    f0 = d.get_state()
    d.step(1)
    f1 = d.get_state()
    d.close()
    nx, ny = p["nx"], p["ny"]
    dom, cyl, faces = _oracle(p)
    fluid = G.classify(dom, [cyl])
    rng = np.random.default_rng(5)
    fl = np.flatnonzero(mask)
    bn = np.unique(links["node"])
    x = bn % nx
    nodes = np.unique(np.concatenate([rng.choice(fl, 20000, replace=False), bn[(x < 3) | (x > nx - 3)]]))
    sub = G.cut_links(dom, fluid, [cyl], faces, nodes=nodes)
    out = solver.step_at(dom, f0, fluid, sub, nodes, p["tau"], rho_out=1.0)
    got = f1[:, nodes]
    err = np.abs(got - out).max()
    rel = np.linalg.norm(got - out) / np.linalg.norm(out)
    _say("max |df|", err, "rel L2", rel, "nodes", nodes.size)
    assert np.isfinite(out).all() and err <= 1e-6 and rel <= 1e-6


def test_outlet_density_validation(gpu_lib):
    from paper_2009_04604_amd import workloads as W
    B = gpu_lib
    p = synth.cylinder_channel(nx=64, ny=32, radius=3.0, centre=(16.0, 16.0), tau=0.6)
    mask, links = W.channel_geometry(p, outlet="pressure")
    d = B.Domain("D2Q9", p["nx"], p["ny"], 1, mask, p["tau"], periodic=(False, False, True))
    with pytest.raises(B.LBMError) as e:
        d.set_boundary_links(links)                # open links before the density
    assert e.value.code == B.LBM_EINVAL
    for bad in (0.0, -1.0, float("nan")):
        with pytest.raises(B.LBMError) as e:
            d.set_outlet_density(bad)
        assert e.value.code == B.LBM_EINVAL
    d.set_outlet_density(1.0)
    d.set_boundary_links(links)
    d.step(3)
    d.close()
