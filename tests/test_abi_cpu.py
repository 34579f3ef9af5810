"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, rejects invalid descriptors before touching a device, and its host
geometry builder reproduces the oracle's fluid mask and cut links (integer
(node, dir) sets bit-exact, q and wall velocities to round-off)."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import geometry as G, lattice
from tests.libutil import declared_symbols, ensure_built


@pytest.fixture(scope="module")
def B():
    return ensure_built()


def test_exports_every_declared_symbol(B):
    syms = declared_symbols()
    assert len(syms) >= 18
    L = B.lib()
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(B.EXPORTED)


@pytest.mark.parametrize("field,value", [("tau", 0.5), ("tau", float("nan")), ("lattice", 7), ("nz", 3),
                                         ("storage", 9), ("outlet_face", 0), ("rho0", -1.0),
                                         ("rounding", 2), ("rounding", 1)])   # stochastic needs 16-bit storage
def test_init_rejects_invalid_descriptor(B, field, value):
    d = B.make_desc("D2Q9", 8, 8, 1, 0.8, periodic=(True, True, True))
    if field == "nz":
        d.nz = value
    elif field == "outlet_face":
        d.outlet_face = value          # -x face on a periodic axis
    else:
        setattr(d, field, value)
    h = ctypes.c_void_p()
    m = np.ones(64 * max(1, d.nz), np.uint8)
    code = B.lib().lbm_init_domain(ctypes.byref(d), m.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
    assert code == B.LBM_EINVAL
    assert B.lib().lbm_last_error().decode()


@pytest.mark.parametrize("name,storage,rounding", [("f16s", 2, 0), ("bf16s", 3, 0), ("f16s-sr", 2, 1),
                                                  ("bf16s-sr", 3, 1), ("f32", 1, 0)])
def test_storage_names_map_to_storage_and_rounding(B, name, storage, rounding):
    d = B.make_desc("D2Q9", 8, 8, 1, 0.8, storage=name)
    assert (d.storage, d.rounding) == (storage, rounding)


def test_init_rejects_a_lattice_beyond_32_bit_indexing(B):
    """2048 x 1024 x 1024 stored nodes (dense layout) exceed the kernels' 32-bit
    population index; refused before any device call (the mask is never read)."""
    d = B.make_desc("D3Q19", 2048, 1024, 1024, 0.8, periodic=(True, True, True), layout="dense")
    m = np.zeros(2048 * 1024 * 1024, np.uint8)       # untouched pages: no memory is used
    h = ctypes.c_void_p()
    code = B.lib().lbm_init_domain(ctypes.byref(d), m.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
    assert code == B.LBM_EINVAL
    assert "too large" in B.lib().lbm_last_error().decode()
    assert not h.value


def _compare(mask, links, fluid, ol):
    assert np.array_equal(mask.astype(bool), fluid.reshape(-1))
    assert np.array_equal(links["node"], ol["node"])
    assert np.array_equal(links["dir"], ol["dir"])
    assert np.abs(links["q"] - ol["q"]).max(initial=0) <= 1e-12
    assert np.abs(links["uw_t"].T - ol["uw_t"]).max(initial=0) <= 1e-14
    assert np.array_equal(links["shape"], ol["shape"])


def test_builder_matches_oracle_annulus(B):
    from paper_2009_04604_amd import workloads as W
    p = synth.couette_annulus()
    mask, links = W.annulus_geometry(p)
    dom = G.Domain(lattice.D2Q9, p["nx"], p["ny"], 1)
    om1 = p["u_inner"] / p["r1"]
    sh = [G.Sphere(p["centre"], p["r1"], True, Omega=(0, 0, om1)), G.Sphere(p["centre"], p["r2"], False)]
    fluid = G.classify(dom, sh)
    _compare(mask, links, fluid, G.cut_links(dom, fluid, sh))


def test_builder_matches_oracle_channel(B):
    from paper_2009_04604_amd import workloads as W
    p = synth.cylinder_channel(nx=300, ny=120, radius=9.0, centre=(60.0, 60.0))
    mask, links = W.channel_geometry(p)
    dom = G.Domain(lattice.D2Q9, p["nx"], p["ny"], 1, periodic=(False, False, True), outlet_face=1)
    cyl = G.Sphere(p["centre"], p["radius"], True)
    faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(p["ny"], p["u_max"])), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5)]
    fluid = G.classify(dom, [cyl])
    _compare(mask, links, fluid, G.cut_links(dom, fluid, [cyl], faces))


def test_builder_matches_oracle_packing(B):
    from paper_2009_04604_amd import workloads as W
    n = 64
    c, r = synth.sphere_packing(n=n, r_min=3.0, r_max=6.0, solid_fraction=0.4, seed=11)
    mask, links = W.packing_geometry(n, c, r)
    dom = G.Domain(lattice.D3Q19, n, n, n)
    sh = [G.Sphere(cc, rr, True) for cc, rr in zip(c, r)]
    fluid = G.classify(dom, sh)
    _compare(mask, links, fluid, G.cut_links(dom, fluid, sh))
    assert 0.55 < fluid.mean() < 0.65


def test_builder_matches_oracle_packing_d3q27(B):
    n = 40
    c, r = synth.sphere_packing(n=n, r_min=3.0, r_max=6.0, solid_fraction=0.4, seed=12)
    g = B.Geometry("D3Q27", n, n, n)
    g.add_spheres(c, r)
    mask, links = g.build()
    g.close()
    dom = G.Domain(lattice.D3Q27, n, n, n)
    sh = [G.Sphere(cc, rr, True) for cc, rr in zip(c, r)]
    fluid = G.classify(dom, sh)
    _compare(mask, links, fluid, G.cut_links(dom, fluid, sh))
    assert (links["dir"] >= 19).any()          # corner links exist



@pytest.mark.parametrize("lat", ["D3Q19", "D3Q27"])
def test_builder_matches_oracle_cylinders(B, lat):
    """Coaxial cylinders along z (the 3D annulus) plus small spheres between them,
    which exercises the candidate lists of bucketed spheres next to cylinders."""
    p = synth.couette_annulus(scale=0.75)
    nz = 10            # a ball and its periodic image stay apart: r + sqrt(3) < nz / 2
    om1 = p["u_inner"] / p["r1"]
    balls = [((p["centre"][0] + 0.5 * (p["r1"] + p["r2"]), p["centre"][1] + 0.3, 2.7), 1.9),
             ((p["centre"][0] - 0.3, p["centre"][1] - 0.5 * (p["r1"] + p["r2"]), 4.1), 2.2)]
    g = B.Geometry(lat, p["nx"], p["ny"], nz)
    g.add_cylinder(p["centre"], p["r1"], True, Omega=(0, 0, om1))
    g.add_cylinder(p["centre"], p["r2"], False)
    for c, r in balls:
        g.add_sphere(c, r, True)
    mask, links = g.build()
    g.close()
    dom = G.Domain(lattice.get(lat), p["nx"], p["ny"], nz)
    sh = [G.Cylinder(p["centre"], p["r1"], True, Omega=(0, 0, om1)), G.Cylinder(p["centre"], p["r2"], False)]
    sh += [G.Sphere(c, r, True) for c, r in balls]
    fluid = G.classify(dom, sh)
    _compare(mask, links, fluid, G.cut_links(dom, fluid, sh))
    assert set(np.unique(links["shape"])) == {0, 1, 2, 3}


def test_binding_loads_torch_before_the_library():
    """The library must bind to the HIP runtime torch loads (torch's streams and
    memory are passed to it); loading it first would pull in a second runtime."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; from paper_2009_04604_amd import binding as B; "
            "assert 'torch' not in sys.modules; B.lib(); assert 'torch' in sys.modules; print('ok')")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr


def test_builder_rejects_bad_shapes(B):
    """Host-only argument checks of the builder's shapes (no GPU needed)."""
    g = B.Geometry("D3Q19", 16, 16, 8, periodic=(True, False, True))
    for r in (0.0, -1.0, float("inf")):
        with pytest.raises(B.LBMError) as e:
            g.add_cylinder((8.0, 8.0, 0.0), r)
        assert e.value.code == B.LBM_EINVAL
    with pytest.raises(B.LBMError) as e:
        g.add_cylinder((8.0, float("nan"), 0.0), 3.0)
    assert e.value.code == B.LBM_EINVAL
    g.close()
