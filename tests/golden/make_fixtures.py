"""Write the stored oracle results used by the full-length parity tests.

    python tests/golden/make_fixtures.py c3       # 64^3 sphere packing, 10000 steps
    python tests/golden/make_fixtures.py c2       # 2048 x 1024 cylinder channel, 2000 steps
    python tests/golden/make_fixtures.py c5 3     # moving-sphere box id 3, 4000 steps
    python tests/golden/make_fixtures.py c4       # 16 served requests with L <= 256, 5000 steps
    python tests/golden/make_fixtures.py e3       # BFL comparator, linear error along the axis
    python tests/golden/make_fixtures.py c3 --extended   # the same in extended precision

Every value written here comes from the FP64 oracle (oracle/) run on the seeded
recipes of ``synth``; nothing is read from the GPU path.  With --extended (c2,
c3, c4) the oracle computes in the host's long double (oracle.precision) and
the file is named *_ext.npz: its results carry the exact solution of the
discrete problem to ~1e-15 of the velocity, where the FP64 oracle's own
rounding of f = w + O(u) leaves ~1e-12 after 1000 steps of the packing.

The full fields are
too large to keep, so each file holds the velocity and density at a fixed,
seeded sample of fluid nodes (uniform over the fluid plus boundary nodes, whose
populations the ELIBB rebuilds), and the full-field norm of u, the mass and the
momentum at each checkpoint (the relative L2 velocity error over the sample is
an unbiased estimate of the full-field one).  Runs print one progress line per
checkpoint; C5 rewrites its file at every checkpoint, so a run that is cut short
leaves the checkpoints it reached.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import geometry as G, lattice as OL, moving, precision, solver  # noqa: E402

SAMPLE_FLUID = 16384
SAMPLE_BND = 4096


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def sample_nodes(fluid, link_nodes, seed, n_fluid=SAMPLE_FLUID, n_bnd=SAMPLE_BND):
    """Sorted node sample: n_fluid uniform fluid nodes plus n_bnd boundary nodes."""
    rng = np.random.default_rng(seed)
    fl = np.flatnonzero(fluid)
    a = rng.choice(fl, size=min(n_fluid, fl.size), replace=False)
    b = np.unique(link_nodes)
    b = rng.choice(b, size=min(n_bnd, b.size), replace=False) if b.size else b
    return np.unique(np.concatenate([a, b]).astype(np.int64))


def snapshot(sim, nodes, dim):
    rho, u = sim.macros()
    fl = sim.fluid
    return {
        "rho": rho[nodes], "u": u[:dim, nodes],
        "norm_u": float(np.sqrt(np.sum(u[:dim, fl] ** 2))),
        "mass": float(rho[fl].sum()),
        "momentum": (rho[fl][None, :] * u[:, fl]).sum(axis=1),
        "n_fluid": int(fl.sum()),
    }


def _out(v):
    """Stored values are float64 (an extended result rounded once)."""
    a = np.asarray(v)
    return a.astype(np.float64) if a.dtype == np.longdouble else a


def fixture_path(name, args):
    return os.path.join(HERE, name + ("_ext" if getattr(args, "extended", False) else "") + ".npz")


def save(path, meta, nodes, snaps):
    arrays = {"nodes": nodes, "meta": np.array(json.dumps(meta))}
    for t, s in snaps.items():
        for k, v in s.items():
            arrays[f"t{t}_{k}"] = _out(v)
    np.savez_compressed(path + ".tmp.npz", **arrays)
    os.replace(path + ".tmp.npz", path)


def run_static(sim, nodes, dim, checkpoints, path, meta):
    snaps = {}
    t = 0
    t0 = time.time()
    for cp in checkpoints:
        sim.run(cp - t)
        t = cp
        snaps[cp] = snapshot(sim, nodes, dim)
        log(f"{meta['case']}: step {cp} ({time.time() - t0:.0f} s)")
        save(path, dict(meta, checkpoints=sorted(snaps)), nodes, snaps)
    return snaps


def c3(args):
    """C3 crop: the packing recipe (largest-first RSA, radii U[6,12], porosity 0.6)
    in a periodic 64^3 box, D3Q19 BGK FP64, tau 0.9, Guo force 1e-6 x, ELIBB-FQ."""
    n = 64
    c, r = synth.sphere_packing(n=n)
    dom = G.Domain(OL.D3Q19, n, n, n)
    sh = [G.Sphere(cc, rr, True) for cc, rr in zip(c, r)]
    fluid = G.classify(dom, sh)
    links = G.cut_links(dom, fluid, sh)
    sim = solver.Simulation(dom, 0.9, force=(1e-6, 0.0, 0.0))
    sim.set_geometry(fluid, links, "FQ")
    sim.init_equilibrium()
    nodes = sample_nodes(fluid.reshape(-1), links["node"], synth.seed_for(3) + 7)
    meta = {"case": "packing64", "lattice": "D3Q19", "n": [n, n, n], "tau": 0.9, "force": [1e-6, 0, 0],
            "variant": "FQ", "steps": 10000, "n_links": int(links["node"].size)}
    meta["precision"] = str(np.dtype(precision.REAL))
    run_static(sim, nodes, 3, [1000, 10000], fixture_path("c3_packing64", args), meta)


def c2(args):
    """C2 at full size: 2048 x 1024 channel, cylinder R = 20 at (400, 512) + seeded
    offset, parabolic inlet u_max 0.05, Re 100 (tau 0.56), walls at y = -1/2 and
    ny - 1/2, zero-gradient outlet, D2Q9 BGK FP64, ELIBB-FQ; E(t) at 1000 and 2000."""
    p = synth.cylinder_channel()
    dom = G.Domain(OL.D2Q9, p["nx"], p["ny"], 1, periodic=(False, False, True), outlet_face=1)
    cyl = G.Sphere(p["centre"], p["radius"], True)
    faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(p["ny"], p["u_max"])), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5)]
    fluid = G.classify(dom, [cyl])
    links = G.cut_links(dom, fluid, [cyl], faces)
    sim = solver.Simulation(dom, p["tau"])
    sim.set_geometry(fluid, links, "FQ")
    sim.init_equilibrium()
    cyl_nodes = links["node"][links["shape"] == 0]
    rng = np.random.default_rng(synth.seed_for(2) + 7)
    nodes = np.unique(np.concatenate([sample_nodes(fluid.reshape(-1), links["node"], rng.integers(1 << 31)),
                                      cyl_nodes]))
    meta = {"case": "channel2048", "lattice": "D2Q9", "n": [p["nx"], p["ny"], 1], "tau": p["tau"],
            "centre": list(p["centre"]), "radius": p["radius"], "u_max": p["u_max"], "variant": "FQ",
            "steps": 2000, "n_links": int(links["node"].size)}
    meta["precision"] = str(np.dtype(precision.REAL))
    run_static(sim, nodes, 2, [1000, 2000], fixture_path("c2_channel2048", args), meta)


def c5(args):
    """C5: one box of the moving-sphere recipe (32 boxes, side U{96..192}, sphere
    r U[10,16], sinusoidal translation and rotation), D3Q19 BGK FP64, ELIBB-FQ,
    links rebuilt and fresh nodes refilled every step, 4000 steps."""
    boxes = synth.moving_boxes()
    b = [x for x in boxes if x["id"] == args.box][0]
    dom = G.Domain(OL.D3Q19, b["nx"], b["ny"], b["nz"])
    kin = moving.Kinematics(b["x0"], b["amplitude"], b["period"], b["direction"], b["omega"])
    m = moving.MovingSphereSim(dom, b["radius"], kin, tau=b["tau"])
    path = os.path.join(HERE, f"c5_box{b['id']}.npz")
    snaps = {}
    rng = np.random.default_rng(synth.seed_for(5) + 7 + b["id"])
    t0 = time.time()
    for cp in (1000, 2000, 3000, 4000):
        m.run(cp - m.t)
        fl = m.sim.fluid
        nodes = sample_nodes(fl, m.sim.links["node"], rng.integers(1 << 31), n_bnd=2048)
        s = snapshot(m.sim, nodes, 3)
        s["nodes"] = nodes
        s["n_links"] = int(m.sim.links["node"].size)
        snaps[cp] = s
        log(f"box {b['id']}: step {cp} ({time.time() - t0:.0f} s)")
        meta = {"case": f"moving_box{b['id']}", "lattice": "D3Q19", "n": [b["nx"], b["ny"], b["nz"]],
                "box": {k: (list(v) if isinstance(v, tuple) else v) for k, v in b.items()}, "variant": "FQ",
                "steps": 4000, "checkpoints": sorted(snaps)}
        save(path, meta, np.zeros(0, np.int64), snaps)


def c4_requests(n_req=16, l_max=256):
    """The first n_req requests of the served stream (256 requests, seed of C4)
    whose side L is at most l_max."""
    reqs = synth.request_stream(256)
    return [r for r in reqs if r["L"] <= l_max][:n_req]


def c4(args):
    """C4 sample: 16 requests of the served stream with L <= 256 (circular Couette
    L x L, tau 0.8; cylinder channel 2L x L, tau 0.6), D2Q9 BGK FP64, ELIBB-FQ,
    5000 steps each."""
    path = fixture_path("c4_requests", args)
    arrays = {}
    meta = {"case": "served_requests", "steps": 5000, "requests": [], "precision": str(np.dtype(precision.REAL))}
    t0 = time.time()
    for req in c4_requests():
        if req["kind"] == "couette":
            dom = G.Domain(OL.D2Q9, req["nx"], req["ny"], 1)
            om1 = req["u_inner"] / req["r1"]
            sh = [G.Sphere(req["centre"], req["r1"], True, Omega=(0, 0, om1)),
                  G.Sphere(req["centre"], req["r2"], False)]
            faces = []
        else:
            dom = G.Domain(OL.D2Q9, req["nx"], req["ny"], 1, periodic=(False, False, True), outlet_face=1)
            sh = [G.Sphere(req["centre"], req["radius"], True)]
            faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(req["ny"], req["u_max"])), G.FaceWall(2, 0.5),
                     G.FaceWall(3, 0.5)]
        fluid = G.classify(dom, sh)
        links = G.cut_links(dom, fluid, sh, faces)
        sim = solver.Simulation(dom, req["tau"])
        sim.set_geometry(fluid, links, "FQ")
        sim.init_equilibrium()
        sim.run(req["steps"])
        nodes = sample_nodes(fluid.reshape(-1), links["node"], synth.seed_for(4) + 7 + req["id"], 4096, 1024)
        s = snapshot(sim, nodes, 2)
        k = f"r{req['id']}_"
        arrays[k + "nodes"] = nodes
        for name, v in s.items():
            arrays[k + name] = _out(v)
        meta["requests"].append({kk: (list(v) if isinstance(v, tuple) else v) for kk, v in req.items()})
        log(f"request {req['id']} ({req['kind']}, L {req['L']}): done ({time.time() - t0:.0f} s)")
        arrays["meta"] = np.array(json.dumps(meta))
        np.savez_compressed(path + ".tmp.npz", **arrays)
        os.replace(path + ".tmp.npz", path)


def e3(args):
    """The oracle-only BFL comparator on the paper's linear-error experiment
    (Sec. III.B: cylindrical Couette, beta = 1/2, TRT with Lambda = 3/16, Re = 10,
    tau 0.8) at r2 - r1 = 10 and 40 lu, two diffusion times: u_y along the
    x-axis through the centre, its closed form, the LE and the rRSE on the axis
    and over the annulus (tests/test_oracle_bfl.py builds the same case)."""
    sys.path.insert(0, ROOT)
    from tests.test_oracle_bfl import _couette_fields
    arrays = {}
    meta = {"case": "e3_bfl", "variant": "BFL", "tau": 0.8, "magic": 3.0 / 16.0, "Re": 10.0, "widths": [10, 40]}
    for w in (10, 40):
        t0 = time.time()
        out = _couette_fields(w, "BFL", magic=3.0 / 16.0)
        for k, v in out.items():
            arrays[f"w{w}_{k}"] = np.asarray(v)
        log(f"e3 width {w}: rRSE axis {out['rrse_axis']:.3e} ({time.time() - t0:.0f} s)")
    arrays["meta"] = np.array(json.dumps(meta))
    path = os.path.join(HERE, "e3_bfl_linear_error.npz")
    np.savez_compressed(path + ".tmp.npz", **arrays)
    os.replace(path + ".tmp.npz", path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=["c2", "c3", "c4", "c5", "e3"])
    ap.add_argument("box", nargs="?", type=int, default=3)
    ap.add_argument("--extended", action="store_true", help="oracle in long double (c2, c3, c4)")
    args = ap.parse_args()
    if args.extended and args.case not in ("c2", "c3", "c4"):
        ap.error("--extended applies to c2, c3 and c4")
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(1)
    except Exception:       # pragma: no cover
        ctx = None
    run = {"c2": c2, "c3": c3, "c4": c4, "c5": c5, "e3": e3}[args.case]
    if args.extended:
        with precision.extended():
            run(args)
    else:
        run(args)
    if ctx is not None:
        ctx.__exit__(None, None, None)


if __name__ == "__main__":
    main()
