"""Benchmark of the fused ELIBB lattice-Boltzmann step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload packing256|channel2048]

Default workload: D3Q19 FP32 body-force-driven flow through a random sphere
packing in a periodic 256^3 box (radii U[6,12], porosity 0.6, tau 0.9, force
1e-6 along x, ELIBB-FQ on every cut link).  A step is one fused collide-stream
+ ELIBB launch over the whole lattice; the timed job is K steps followed by one
FP64 moments/reduction query.  Inputs are resident in HBM before timing starts.

Prints one JSON line:
  value      fluid-node updates per second / 1e6 (MLUPS) of the whole job
  roofline   the step kernel: algorithmic bytes per launch (2 Q sizeof(storage)
             per fluid node) / mean launch duration from HIP events on the
             launch stream, against 8 TB/s
  cpu_baseline  the FP64 oracle timed on the host (one core) on a bounded
             sample of the same workload recipe (a smaller periodic packing)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="packing256", choices=["packing256", "channel2048"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16s", "bf16s"])
    ap.add_argument("--layout", default="compact", choices=["compact", "dense"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="after the measurement, run one plain device copy of this size (for counter scaling)")
    return ap.parse_args()


def traffic_from_profile(workload, storage):
    """HBM bytes per step-kernel launch measured with rocprofv3 counters (FETCH_SIZE
    and WRITE_SIZE scaled by a copy kernel), if the summary in profiles/ was taken
    on the current kernel sources; else None."""
    from paper_2009_04604_amd.profiling import kernel_source_sha
    path = os.path.join(ROOT, "profiles", f"step_kernel_{workload}_{storage}_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_sha():
        return None
    try:
        return float(kv["kernel_bytes_per_launch.FETCH_SIZE"]) + float(kv["kernel_bytes_per_launch.WRITE_SIZE"])
    except (KeyError, ValueError):
        return None


def build_workload(name, storage, layout):
    import synth
    from paper_2009_04604_amd import workloads as W
    if name == "packing256":
        n = 256
        d, mask, links = W.packing_domain(n, storage, layout=layout)
        cfg = {"workload": "sphere_packing_256^3_D3Q19", "lattice": "D3Q19", "n": [n, n, n], "porosity_target": 0.6,
               "tau": 0.9, "force": [1e-6, 0, 0], "variant": "ELIBB-FQ", "storage": storage}
    else:
        p = synth.cylinder_channel()
        d, mask, links = W.channel_domain(p, storage, layout=layout)
        cfg = {"workload": "cylinder_channel_2048x1024_D2Q9", "lattice": "D2Q9", "n": [p["nx"], p["ny"], 1],
               "reynolds": 100, "tau": p["tau"], "variant": "ELIBB-FQ", "storage": storage}
    cfg["layout"] = layout
    return d, cfg


def cpu_baseline(name, seconds):
    """Time the FP64 oracle on one core on a bounded sample of the workload recipe."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:       # pragma: no cover
        threadpool_limits = None
    import numpy as np
    import synth
    from oracle import geometry as G, lattice as OL, solver
    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        if name == "packing256":
            n = 64
            c, r = synth.sphere_packing(n=n)            # same recipe, 64^3 periodic box
            dom = G.Domain(OL.D3Q19, n, n, n)
            sh = [G.Sphere(cc, rr, True) for cc, rr in zip(c, r)]
            fluid = G.classify(dom, sh)
            sim = solver.Simulation(dom, 0.9, force=(1e-6, 0, 0))
            sim.set_geometry(fluid, G.cut_links(dom, fluid, sh), "FQ")
            sample = f"same recipe (largest-first RSA, radii U[6,12], porosity 0.6) in a periodic {n}^3 box, FP64 oracle"
        else:
            p = synth.cylinder_channel(nx=512, ny=256, radius=5.0, centre=(100.0, 128.0))
            dom = G.Domain(OL.D2Q9, p["nx"], p["ny"], 1, periodic=(False, False, True), outlet_face=1)
            cyl = G.Sphere(p["centre"], p["radius"], True)
            faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(p["ny"], p["u_max"])), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5)]
            fluid = G.classify(dom, [cyl])
            sim = solver.Simulation(dom, p["tau"])
            sim.set_geometry(fluid, G.cut_links(dom, fluid, [cyl], faces), "FQ")
            sample = "cylinder channel at 512x256 (same recipe scaled), FP64 oracle"
        sim.init_equilibrium()
        sim.step()
        nfl = int(fluid.sum())
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < seconds:
            sim.step()
            k += 1
        dt = time.perf_counter() - t0
        return {"value": nfl * k / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
                "sample": f"{sample}; {k} steps of {nfl} fluid nodes in {dt:.1f} s"}
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2009_04604_amd import binding as B
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    d, cfg = build_workload(a.workload, a.storage, a.layout)
    info = d.info()
    nfl = info["n_fluid"]
    Q = info["q"]
    sbytes = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}[a.storage]
    bytes_per_update = 2 * Q * sbytes
    stream = torch.cuda.current_stream()

    d.step(a.warmup)
    d.macros(fields=False)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    d.step(a.steps)
    ev1.record(stream)
    _, _, sums, unstable = d.macros(fields=False)       # FP64 reductions (synchronises)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = ev0.elapsed_time(ev1) / a.steps

    mlups = nfl * a.steps / wall / 1e6
    achieved = bytes_per_update * nfl / (kernel_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(a.workload, a.storage),
            "bytes_per_fluid_update": bytes_per_update,
            "link_bytes_per_fluid_update": round(info["link_bytes"] / nfl, 2),
            "kernel_ms": round(kernel_ms, 4)}
    cfg.update({"fluid_nodes": nfl, "cut_links": info["n_links"], "boundary_nodes": info["n_boundary_nodes"],
                "unstable": bool(unstable), "mass": sums[0]})
    out = {
        "metric": "MLUPS (fluid-node updates/s) + % of HBM roofline",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(wall * 1e3 / a.steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"f32": "f32", "f64": "f64", "f16s": "f16", "bf16s": "bf16"}[a.storage],
        "data": "synthetic", "config": cfg, "roofline": roof,
    }
    d.close()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.workload, a.cpu_seconds)
    print(json.dumps(out), flush=True)
    if a.calibration_copy_mib > 0:
        n = a.calibration_copy_mib * 2**20 // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
