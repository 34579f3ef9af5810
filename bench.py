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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="packing256", choices=["packing256", "channel2048"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16s", "bf16s", "f16s-sr", "bf16s-sr"])
    ap.add_argument("--layout", default="compact", choices=["compact", "dense"])
    ap.add_argument("--lattice", default="D3Q19", choices=["D3Q19", "D3Q27"],
                    help="lattice of the packing workload")
    ap.add_argument("--collision", default="BGK", choices=["BGK", "TRT"],
                    help="collision model (TRT with the magic parameter 3/16)")
    ap.add_argument("--wall-neq", default="bounceback", choices=["bounceback", "regularized"],
                    help="wall non-equilibrium estimator of the ELIBB links")
    ap.add_argument("--xcd-remap", type=int, choices=[0, 1], default=None,
                    help="launch option: XCD deal of the step kernel's workgroups: 0 round-robin, 1 contiguous "
                         "eighths; default: the library's")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="only time the FP64 oracle on this host for every configuration (about 10 minutes), "
                         "print one JSON line and exit")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="after the measurement, run one plain device copy of this size (for counter scaling)")
    ap.add_argument("--no-copy-probe", action="store_true",
                    help="skip the device-copy bandwidth measurement (counter runs use their own calibration copy)")
    ap.add_argument("--no-served", action="store_true", help="skip the served-batch section")
    ap.add_argument("--no-boundary-box", action="store_true",
                    help="skip the all-fluid 256^3 box (no-boundary calibration)")
    ap.add_argument("--served-requests", type=int, default=256)
    ap.add_argument("--served-steps", type=int, default=5000)
    ap.add_argument("--served-budget-mib", type=int, default=1024)
    ap.add_argument("--served-load", type=float, default=1.0,
                    help="arrival rate as a multiple of the measured plain FP32 service rate")
    ap.add_argument("--no-moving", action="store_true", help="skip the batched moving-boxes section")
    ap.add_argument("--moving-boxes", type=int, default=32)
    ap.add_argument("--moving-steps", type=int, default=4000)
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


def build_workload(name, storage, layout, lattice="D3Q19", collision="BGK", wall_neq="bounceback"):
    import synth
    from paper_2009_04604_amd import workloads as W
    if name == "packing256":
        n = 256
        d, mask, links = W.packing_domain(n, storage, layout=layout, lattice=lattice, collision=collision,
                                          wall_neq=wall_neq)
        cfg = {"workload": f"sphere_packing_256^3_{lattice}", "lattice": lattice, "n": [n, n, n],
               "porosity_target": 0.6, "tau": 0.9, "force": [1e-6, 0, 0], "variant": "ELIBB-FQ", "storage": storage,
               "collision": collision if collision == "BGK" else "TRT (Lambda 3/16)"}
    else:
        p = synth.cylinder_channel()
        d, mask, links = W.channel_domain(p, storage, layout=layout, wall_neq=wall_neq)
        cfg = {"workload": "cylinder_channel_2048x1024_D2Q9", "lattice": "D2Q9", "n": [p["nx"], p["ny"], 1],
               "reynolds": 100, "tau": p["tau"], "variant": "ELIBB-FQ", "storage": storage, "outlet": "zero-gradient"}
    cfg["layout"] = layout
    cfg["wall_neq"] = wall_neq
    return d, cfg


def copy_bandwidth(gib=2, reps=5):
    """Read + write bandwidth of a plain device-to-device copy (torch), for
    context beside the published peak."""
    import torch
    n = gib * 2**30 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    torch.cuda.empty_cache()
    return round(2.0 * gib * 2**30 / (ms * 1e-3) / 1e9, 1)


def stream_probe(n_elems, arrays=19, reps=10):
    """Practical read + write ceiling: `arrays` FP32 arrays in and `arrays` out,
    n_elems each (the packing's fluid count), one element of every array per
    lane (lbm_stream_probe), on line-aligned runs and on runs shifted by one
    element (every wave straddles lines, as the compact layout's do)."""
    import torch
    from paper_2009_04604_amd import binding as B
    stride = (n_elems + 64 + 63) // 64 * 64
    src = torch.ones(arrays * stride, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {"arrays_in": arrays, "arrays_out": arrays, "elements": n_elems}
    for name, shift in (("aligned", 0), ("shifted", 1)):
        B.lbm_stream_probe(src, dst, n_elems, stride, arrays, shift)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            B.lbm_stream_probe(src, dst, n_elems, stride, arrays, shift)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name + "_GBps"] = round(2 * 4 * arrays * n_elems / (ms * 1e-3) / 1e9, 1)
        out[name + "_ms"] = round(ms, 4)
    del src, dst
    torch.cuda.empty_cache()
    return out


def cpu_baseline(name, seconds, wall_neq="bounceback"):
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
            sim.set_geometry(fluid, G.cut_links(dom, fluid, sh), "FQ", wall_neq=wall_neq)
            sample = f"same recipe (largest-first RSA, radii U[6,12], porosity 0.6) in a periodic {n}^3 box, FP64 oracle"
        else:
            p = synth.cylinder_channel(nx=512, ny=256, radius=5.0, centre=(100.0, 128.0))
            dom = G.Domain(OL.D2Q9, p["nx"], p["ny"], 1, periodic=(False, False, True), outlet_face=1)
            cyl = G.Sphere(p["centre"], p["radius"], True)
            faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(p["ny"], p["u_max"])), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5)]
            fluid = G.classify(dom, [cyl])
            sim = solver.Simulation(dom, p["tau"])
            sim.set_geometry(fluid, G.cut_links(dom, fluid, [cyl], faces), "FQ", wall_neq=wall_neq)
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


# Declared before the served run: the velocity error budget (relative L2 against
# the FP64 oracle) within which a served form counts as delivering the plain
# form's answer.
SERVED_ERROR_BUDGET = 1e-2
# the served form's storage: FP16 shifted populations, stochastically rounded
# stores (unbiased; 7x lower error than nearest rounding on the stored oracle
# sample at ~3% more device time)
SERVED_STORAGE = "f16s-sr"


def _served_fixture():
    """The oracle's FP64 results for the requests of the served stream with
    L <= 256 (tests/golden/c4_requests.npz): id -> (node sample, u (2, n))."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "c4_requests.npz")
    if not os.path.exists(path):
        return {}
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    return {r["id"]: (z[f"r{r['id']}_nodes"], z[f"r{r['id']}_u"][:2]) for r in meta["requests"]}


def _oracle_case(kind, p):
    """An oracle Simulation for one workload recipe (cpu baselines only)."""
    from oracle import geometry as G, lattice as OL, solver
    if kind == "couette":
        dom = G.Domain(OL.D2Q9, p["nx"], p["ny"], 1)
        om1 = p["u_inner"] / p["r1"]
        sh = [G.Sphere(p["centre"], p["r1"], True, Omega=(0, 0, om1)), G.Sphere(p["centre"], p["r2"], False)]
        faces = []
    else:
        dom = G.Domain(OL.D2Q9, p["nx"], p["ny"], 1, periodic=(False, False, True), outlet_face=1)
        sh = [G.Sphere(p["centre"], p["radius"], True)]
        faces = [G.FaceWall(0, 0.5, G.parabolic_inlet(p["ny"], p["u_max"])), G.FaceWall(2, 0.5), G.FaceWall(3, 0.5)]
    fluid = G.classify(dom, sh)
    sim = solver.Simulation(dom, p["tau"])
    sim.set_geometry(fluid, G.cut_links(dom, fluid, sh, faces), "FQ")
    sim.init_equilibrium()
    return sim


def _time_oracle_steps(sim, k, log=None, every=0):
    sim.step()
    t0 = time.perf_counter()
    for j in range(k):
        sim.step()
        if log and every and (j + 1) % every == 0:
            log(f"cpu full: {j + 1} of {k} steps ({time.perf_counter() - t0:.0f} s)")
    return (time.perf_counter() - t0) / k


def _worker_init():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:       # pragma: no cover
        pass


def _request_seconds(args):
    """Oracle seconds per step of one served request (one core)."""
    req, k = args
    sim = _oracle_case(req["kind"], req)
    return _time_oracle_steps(sim, k)


def _box_seconds(args):
    """Oracle seconds per step of one moving-sphere box (one core)."""
    from oracle import geometry as G, lattice as OL, moving
    b, k = args
    dom = G.Domain(OL.D3Q19, b["nx"], b["ny"], b["nz"])
    kin = moving.Kinematics(b["x0"], b["amplitude"], b["period"], b["direction"], b["omega"])
    m = moving.MovingSphereSim(dom, b["radius"], kin, tau=b["tau"])
    m.step()
    t0 = time.perf_counter()
    m.run(k)
    return (time.perf_counter() - t0) / k


def cpu_baseline_full(log):
    """The FP64 oracle on the host of this run, per workload: one core for the
    single-domain configurations (the 48^2 annulus in full; 200 steps of the
    2048 x 1024 channel; 20 steps of the 256^3 packing; 20 steps of the
    smallest moving box, projected to its 4000), and every core of the host,
    one process per request or box, for the served stream and the moving
    boxes (a sample of 16 requests and 8 boxes, a few steps each, projected to
    their full step counts)."""
    import multiprocessing as mp
    import numpy as np
    import synth
    from oracle import geometry as G, lattice as OL, solver
    _worker_init()
    cores = len(os.sched_getaffinity(0))
    out = {"cores_all": cores, "kind": "oracle"}
    # C1 in full
    p = synth.couette_annulus()
    sim = _oracle_case("couette", p)
    t0 = time.perf_counter()
    sim.run(p["steps"])
    dt = time.perf_counter() - t0
    nfl = int(sim.fluid.sum())
    out["C1_annulus48_5000_steps"] = {"seconds": round(dt, 2), "MLUPS": round(nfl * p["steps"] / dt / 1e6, 3), "cores": 1}
    log(f"cpu full: C1 {dt:.1f} s")
    # C2: 200 steps
    p = synth.cylinder_channel()
    sim = _oracle_case("channel", p)
    s = _time_oracle_steps(sim, 200, log, 20)
    nfl = int(sim.fluid.sum())
    out["C2_channel2048_200_steps"] = {"s_per_step": round(s, 3), "MLUPS": round(nfl / s / 1e6, 3), "cores": 1,
                                       "projected_20000_steps_h": round(20000 * s / 3600, 2)}
    del sim
    log(f"cpu full: C2 {s:.3f} s/step")
    # C3 at full size: 20 steps
    n = 256
    c, r = synth.sphere_packing(n=n)
    dom = G.Domain(OL.D3Q19, n, n, n)
    sh = [G.Sphere(cc, rr, True) for cc, rr in zip(c, r)]
    t0 = time.perf_counter()
    fluid = G.classify(dom, sh)
    log(f"cpu full: C3 classified ({time.perf_counter() - t0:.0f} s)")
    links = G.cut_links(dom, fluid, sh)
    log(f"cpu full: C3 {links['node'].size} cut links ({time.perf_counter() - t0:.0f} s)")
    sim = solver.Simulation(dom, 0.9, force=(1e-6, 0, 0))
    sim.set_geometry(fluid, links, "FQ")
    sim.init_equilibrium()
    del links
    setup = time.perf_counter() - t0
    log(f"cpu full: C3 set up ({setup:.0f} s)")
    s = _time_oracle_steps(sim, 20, log, 2)
    nfl = int(fluid.sum())
    out["C3_packing256_20_steps"] = {"s_per_step": round(s, 3), "MLUPS": round(nfl / s / 1e6, 3), "cores": 1,
                                     "setup_s": round(setup, 1), "projected_10000_steps_h": round(10000 * s / 3600, 2)}
    del sim, fluid
    log(f"cpu full: C3 256^3 {s:.2f} s/step")
    # C5: the smallest box, 20 steps
    boxes = synth.moving_boxes()
    small = min(boxes, key=lambda b: b["nx"])
    s = _box_seconds((small, 20))
    out["C5_smallest_box_20_steps"] = {"box": small["id"], "side": small["nx"], "s_per_step": round(s, 3), "cores": 1,
                                       "projected_4000_steps_h": round(4000 * s / 3600, 2)}
    log(f"cpu full: C5 box {small['id']} {s:.2f} s/step")
    # all cores: served requests and moving boxes
    reqs = synth.request_stream(256)
    sample = reqs[::16]
    with mp.get_context("fork").Pool(processes=cores, initializer=_worker_init) as pool:
        t0 = time.perf_counter()
        sec = []
        for x in pool.imap_unordered(_request_seconds, [(q, 10) for q in sample]):
            sec.append(x)
            log(f"cpu full: C4 request {len(sec)} of {len(sample)} timed")
        wall = time.perf_counter() - t0
        per_req = float(np.mean(sec)) * 5000
        out["C4_served_all_cores"] = {"sample": f"{len(sample)} requests (every 16th of the 256), 10 steps each",
                                      "mean_request_s_at_5000_steps": round(per_req, 1),
                                      "solves_per_s": round(cores / per_req, 5), "cores": cores,
                                      "sample_wall_s": round(wall, 1)}
        log(f"cpu full: C4 {cores / per_req:.5f} solves/s on {cores} cores")
        bsample = boxes[::4]
        sec = []
        for x in pool.imap_unordered(_box_seconds, [(b, 3) for b in bsample]):
            sec.append(x)
            log(f"cpu full: C5 box {len(sec)} of {len(bsample)} timed")
        per_box = float(np.mean(sec)) * 4000
        out["C5_boxes_all_cores"] = {"sample": f"{len(bsample)} boxes (every 4th of the 32), 3 steps each",
                                     "mean_box_s_at_4000_steps": round(per_box, 1),
                                     "boxes_per_s": round(cores / per_box, 6), "cores": cores}
        log(f"cpu full: C5 {cores / per_box:.6f} boxes/s on {cores} cores")
    return out


def served_section(a, log):
    """Served D2Q9 requests (circular Couette L x L and cylinder channel 2L x L,
    L ~ U{64..1024}, Poisson arrivals): continuously batched FP16-shifted form,
    and the same batching in FP32 (results identical to the plain form's), against
    the plain FP32 one-request-at-a-time form on the same arrivals.  Every form
    builds the geometry of arrived requests on the same 4-thread pool while
    earlier requests run; device-busy time is the HIP-event time of the step
    launches."""
    import numpy as np
    import torch
    import synth
    from paper_2009_04604_amd import serve
    reqs = synth.request_stream(n_requests=a.served_requests, rate=1.0, steps=a.served_steps)
    sample = sorted(set(range(0, len(reqs), max(1, len(reqs) // 16))))
    # plain service rate from a sample of requests run alone in FP32
    log(f"served: {len(reqs)} requests; plain service-time sample")
    ex = serve.GpuExecutor(storage="f32")
    t_serv = []
    for k in sample[:8]:
        q = dict(reqs[k])
        t0 = time.perf_counter()
        h = ex.admit(ex.prepare(q))
        ex.step_alone(h, q["steps"])
        ex.sync()
        ex.finish(h, q)
        ex.free(h)
        t_serv.append(time.perf_counter() - t0)
    ex.close()
    mu = 1.0 / float(np.mean(t_serv))
    lam = a.served_load * mu
    for r in reqs:
        r["arrival"] = r["arrival"] / lam          # unit-rate Poisson times scaled to rate lam
    log(f"served: plain sample service {np.mean(t_serv):.4f} s/request, arrival rate {lam:.2f}/s")
    budget = a.served_budget_mib * 2**20
    fix = _served_fixture() if a.served_steps == 5000 else {}
    ids = sorted(set(reqs[k]["id"] for k in sample) | set(fix))
    exs = serve.GpuExecutor(storage=SERVED_STORAGE, keep_fields=ids)
    srv = serve.Server(exs, hbm_budget=budget, chunk=100, prepare_workers=4)
    log("served: batched run")
    served = srv.run(reqs)
    busy_served = exs.busy_s
    exs.close()
    log("served: done")
    # the served form at exactly the plain form's error: FP32 storage, same batching
    exs32 = serve.GpuExecutor(storage="f32", keep_fields=ids)
    srv32 = serve.Server(exs32, hbm_budget=budget, chunk=100, prepare_workers=4)
    log("served: batched FP32 run")
    served32 = srv32.run(reqs)
    busy_served32 = exs32.busy_s
    exs32.close()
    exp = serve.GpuExecutor(storage="f32", keep_fields=ids)
    plain = serve.run_plain(exp, reqs, prepare_workers=4)
    busy_plain = exp.busy_s
    exp.close()
    log("served: plain done")
    # velocity error of each sampled request against the same request in FP64
    # capacity: every request queued at t = 0 (served), server busy time (plain)
    log("served: capacity run (all requests at t = 0)")
    reqs0 = [dict(r, arrival=0.0) for r in reqs]
    exc = serve.GpuExecutor(storage=SERVED_STORAGE)
    srv0 = serve.Server(exc, hbm_budget=budget, chunk=100, prepare_workers=4)
    cap_served = serve.summarize(srv0.run(reqs0))["solves_per_s"]
    exc.close()
    exc = serve.GpuExecutor(storage="f32")
    srv0 = serve.Server(exc, hbm_budget=budget, chunk=100, prepare_workers=4)
    cap_served32 = serve.summarize(srv0.run(reqs0))["solves_per_s"]
    exc.close()
    cap_plain = serve.busy_capacity(plain)
    log("served: FP64 references")
    ref = serve.GpuExecutor(storage="f64", keep_fields=ids)
    e_s, e_p, e_s32 = [], [], []
    same32 = True
    for k in sample:
        q = reqs[k]
        h = ref.admit(ref.prepare(q))
        ref.step_alone(h, q["steps"])
        u = ref.finish(h, q)["u"]
        ref.free(h)
        nrm = np.linalg.norm(u)
        e_s.append(float(np.linalg.norm(served[k]["result"]["u"] - u) / nrm))
        e_p.append(float(np.linalg.norm(plain[k]["result"]["u"] - u) / nrm))
        e_s32.append(float(np.linalg.norm(served32[k]["result"]["u"] - u) / nrm))
        same32 = same32 and np.array_equal(served32[k]["result"]["u"], plain[k]["result"]["u"])
    ref.close()
    torch.cuda.synchronize()
    # against the FP64 oracle on the stored node samples
    eo = {"served": [], "plain": [], "served_f32": []}
    for rid, (nodes, uref) in fix.items():
        nrm = np.linalg.norm(uref)
        for name, recs in (("served", served), ("plain", plain), ("served_f32", served32)):
            u = recs[rid]["result"]["u"][nodes].T
            eo[name].append(float(np.linalg.norm(u - uref) / nrm))
    ss, sp, s32 = serve.summarize(served), serve.summarize(plain), serve.summarize(served32)

    def oracle_err(name):
        if not eo[name]:
            return None
        return {"max": max(eo[name]), "median": float(np.median(eo[name])),
                "within_budget": bool(max(eo[name]) <= SERVED_ERROR_BUDGET)}
    nodes = sum(r["nx"] * r["ny"] for r in reqs)
    return {
        "workload": f"{len(reqs)} D2Q9 requests (circular Couette LxL / cylinder channel 2LxL, L~U{{64..1024}}), "
                    f"{a.served_steps} steps each, Poisson arrivals",
        "arrival_rate_per_s": round(lam, 3), "load_vs_plain_rate": a.served_load, "hbm_budget_bytes": budget,
        "lattice_nodes_total": nodes,
        "served": {"storage": SERVED_STORAGE + " (FP16 f - w with stochastic rounding, FP32 compute, FP64 reductions)",
                   "solves_per_s": round(ss["solves_per_s"], 3),
                   "p50_s": round(ss["p50_s"], 4), "p99_s": round(ss["p99_s"], 4), "makespan_s": round(ss["makespan_s"], 3),
                   "peak_resident": srv.peak_active, "peak_bytes": srv.peak_bytes, "chunks": srv.chunks,
                   "host_phase_s": {k: round(v, 3) for k, v in sorted(srv.phase.items())},
                   "device_busy_s": round(busy_served, 3),
                   "E_vs_oracle": oracle_err("served"),
                   "E_vs_f64_max": max(e_s), "E_vs_f64_median": float(np.median(e_s))},
        "plain": {"storage": "f32, one request at a time (FIFO), geometry prefetched on the same 4-thread pool",
                  "solves_per_s": round(sp["solves_per_s"], 3),
                  "p50_s": round(sp["p50_s"], 4), "p99_s": round(sp["p99_s"], 4), "makespan_s": round(sp["makespan_s"], 3),
                  "device_busy_s": round(busy_plain, 3), "E_vs_oracle": oracle_err("plain"),
                  "E_vs_f64_max": max(e_p), "E_vs_f64_median": float(np.median(e_p))},
        "served_f32": {"storage": "f32, continuous batching (the plain form's arithmetic)",
                       "solves_per_s": round(s32["solves_per_s"], 3), "p50_s": round(s32["p50_s"], 4),
                       "p99_s": round(s32["p99_s"], 4), "makespan_s": round(s32["makespan_s"], 3),
                       "peak_resident": srv32.peak_active, "device_busy_s": round(busy_served32, 3),
                       "E_vs_oracle": oracle_err("served_f32"), "E_vs_f64_max": max(e_s32),
                       "E_vs_f64_median": float(np.median(e_s32)), "fields_identical_to_plain": bool(same32)},
        "equal_error_speedup_solves_per_s": round(s32["solves_per_s"] / sp["solves_per_s"], 3),
        "equal_error_p99_ratio_plain_over_served": round(sp["p99_s"] / s32["p99_s"], 3),
        "capacity_solves_per_s": {"served": round(cap_served, 3), "served_f32": round(cap_served32, 3),
                                  "plain": round(cap_plain, 3), "ratio": round(cap_served / cap_plain, 3),
                                  "ratio_f32": round(cap_served32 / cap_plain, 3),
                                  "how": "served: all requests queued at t = 0, over the makespan; "
                                         "plain: requests per second of busy time in the run above"},
        "speedup_solves_per_s": round(ss["solves_per_s"] / sp["solves_per_s"], 3),
        "p99_ratio_plain_over_served": round(sp["p99_s"] / ss["p99_s"], 3),
        "error_budget": {"relative_L2_velocity_vs_fp64_oracle": SERVED_ERROR_BUDGET, "declared": "before the run"},
        "error_sample": f"E_vs_oracle: the {len(fix)} requests with L <= 256 stored by the FP64 oracle "
                        f"(tests/golden/c4_requests.npz, node samples); E_vs_f64: {len(sample)} requests "
                        f"(every {max(1, len(reqs) // 16)}th) against the FP64 GPU path",
    }


def no_boundary_section(a, log):
    """All-fluid periodic 256^3 D3Q19 box, FP32, compact layout, with the packing's
    tau and force and no links: the step kernel without boundary work, every
    segment's slots starting on a 128 B line (the no-boundary calibration)."""
    import torch
    from paper_2009_04604_amd import binding as B
    n = 256
    g = B.Geometry("D3Q19", n, n, n, periodic=(True, True, True))
    mask, links = g.build()
    g.close()
    d = B.Domain("D3Q19", n, n, n, mask, 0.9, storage="f32", force=(1e-6, 0.0, 0.0), layout="compact")
    d.set_boundary_links(links)
    nfl = d.info()["n_fluid"]
    stream = torch.cuda.current_stream()
    log("no-boundary box: timed steps")
    d.step(a.warmup)
    d.macros(fields=False)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    d.step(a.steps)
    ev1.record(stream)
    _, _, _, unstable = d.macros(fields=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = ev0.elapsed_time(ev1) / a.steps
    d.close()
    achieved = 152 * nfl / (kernel_ms * 1e-3) / 1e9
    return {"workload": "all-fluid periodic 256^3 D3Q19 box, FP32, compact layout, tau 0.9, Guo force (1e-6, 0, 0), "
                        "no links", "fluid_nodes": nfl, "cut_links": int(len(links["q"])), "steps": a.steps,
            "ms_per_step": round(wall * 1e3 / a.steps, 4), "kernel_ms": round(kernel_ms, 4),
            "mlups": round(nfl * a.steps / wall / 1e6, 1), "achieved_GBps": round(achieved, 1),
            "frac": round(achieved / HBM_PEAK_GBS, 4), "unstable": bool(unstable)}


def moving_section(a, log):
    """Batched D3Q19 BF16 periodic boxes, each with a sphere in prescribed
    motion, links rebuilt on the device every step."""
    import torch
    import synth
    from paper_2009_04604_amd import binding as B, workloads as W
    boxes = synth.moving_boxes(n_boxes=a.moving_boxes, steps=a.moving_steps)
    log(f"moving: {len(boxes)} boxes, building")
    ds = [W.moving_box_domain(b, storage="bf16s") for b in boxes]
    bt = B.Batch()
    log("moving: autotune")
    choice = bt.autotune(ds, steps_per_candidate=4)
    log(f"moving: choice {choice}; timed run of {a.moving_steps} steps")
    torch.cuda.synchronize()
    nodes = sum(b["nx"] * b["ny"] * b["nz"] for b in boxes)
    fluid0 = sum(d.info()["n_fluid"] for d in ds)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    bt.step(ds, a.moving_steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    fluid1 = sum(d.info()["n_fluid"] for d in ds)
    links = sum(d.info()["n_links"] for d in ds)
    unstable = False
    for d in ds:
        unstable = unstable or d.macros(fields=False)[3]
    log("moving: batched done")
    # the same boxes one after another with lbm_step, a few steps each
    k = 50
    log("moving: one box at a time")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for d in ds:
        d.step(k)
    torch.cuda.synchronize()
    one = (time.perf_counter() - t1) / k
    bt.close()
    for d in ds:
        d.close()
    fl = 0.5 * (fluid0 + fluid1)
    mlups = fl * a.moving_steps / wall / 1e6
    achieved = 2 * 19 * 2 * fl * a.moving_steps / gpu_s / 1e9
    return {
        "workload": f"{len(boxes)} periodic D3Q19 boxes, side U{{96..192}}, moving sphere r U[10,16], BF16 shifted, "
                    f"{a.moving_steps} steps, links rebuilt on the GPU every step",
        "lattice_nodes": nodes, "fluid_nodes_mean": int(fl), "cut_links_final": links, "unstable": bool(unstable),
        "mlups": round(mlups, 1), "ms_per_step": round(wall * 1e3 / a.moving_steps, 4),
        "boxes_per_s": round(len(boxes) * a.moving_steps / wall / a.moving_steps, 3),
        "hbm_frac_population_bytes": round(achieved / HBM_PEAK_GBS, 4), "achieved_GBps": round(achieved, 1),
        "autotune_choice": choice, "one_at_a_time_ms_per_step": round(one * 1e3, 4),
        "batched_speedup_vs_one_at_a_time": round(one / (wall / a.moving_steps), 3),
    }


def main():
    a = parse()
    if a.cpu_baseline_full:
        print(json.dumps({"cpu_baseline_full": cpu_baseline_full(log)}), flush=True)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2009_04604_amd import binding as B
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    log(f"main: building {a.workload} ({a.storage}, {a.layout})")
    d, cfg = build_workload(a.workload, a.storage, a.layout, a.lattice, a.collision, a.wall_neq)
    if a.xcd_remap is not None:
        d.set_launch_option(0, a.xcd_remap)
        cfg["xcd_remap"] = a.xcd_remap
    log("main: timed steps")
    info = d.info()
    nfl = info["n_fluid"]
    Q = info["q"]
    sbytes = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2, "f16s-sr": 2, "bf16s-sr": 2}[a.storage]
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
    traffic = traffic_from_profile(a.workload, a.storage) if (a.lattice, a.collision, a.wall_neq) == ("D3Q19", "BGK", "bounceback") else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_fluid_update": bytes_per_update,
            "link_bytes_per_fluid_update": round(info["link_bytes"] / nfl, 2),
            "kernel_ms": round(kernel_ms, 4),
            "traffic_GBps": None if traffic is None else round(traffic / (kernel_ms * 1e-3) / 1e9, 1),
            "device_copy_GBps": None if a.no_copy_probe else copy_bandwidth()}
    if not a.no_copy_probe:
        sp = stream_probe(nfl, arrays=Q)
        roof["stream_probe"] = sp
        # the practical ceiling of this access pattern: the achieved rate against
        # the aligned and the shifted 2Q-array stream measured in the same run
        roof["frac_of_aligned_stream"] = round(achieved / sp["aligned_GBps"], 4)
        roof["frac_of_shifted_stream"] = round(achieved / sp["shifted_GBps"], 4)
    cfg.update({"fluid_nodes": nfl, "cut_links": info["n_links"], "boundary_nodes": info["n_boundary_nodes"],
                "unstable": bool(unstable), "mass": sums[0]})
    out = {
        "metric": "MLUPS (fluid-node updates/s) + % of HBM roofline",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(wall * 1e3 / a.steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"f32": "f32", "f64": "f64", "f16s": "f16", "bf16s": "bf16", "f16s-sr": "f16", "bf16s-sr": "bf16"}[a.storage],
        "data": "synthetic", "config": cfg, "roofline": roof,
    }
    d.close()

    if not a.no_boundary_box:
        out["no_boundary_box"] = no_boundary_section(a, log)
    if not a.no_moving:
        out["moving_batch"] = moving_section(a, log)
    if not a.no_served:
        out["served_batch"] = served_section(a, log)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.workload, a.cpu_seconds, a.wall_neq)
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
