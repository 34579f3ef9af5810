"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module holds only input recipes -- lattice sizes, obstacle positions and
radii, relaxation times, request streams -- and none of the method's
arithmetic (no equilibria, no link distances, no interpolation).  Both the
oracle and the HIP library derive everything else from these descriptions on
their own.  All randomness comes from numpy's PCG64 seeded per workload.

Workloads (shapes of the paper's test cases; the paper publishes no datasets):

* ``couette_annulus``   circular Couette between an inner rotating and an outer
                        resting cylinder (Sec. III.B), D2Q9.
* ``cylinder_channel``  channel flow past a circular cylinder, parabolic inlet,
                        zero-gradient outlet, walls at y = -1/2 and ny - 1/2.
* ``sphere_packing``    random non-overlapping spheres placed largest-first by
                        random sequential addition in a periodic box.
* ``request_stream``    a Poisson stream of served requests (Couette / channel).
* ``moving_boxes``      periodic boxes each holding one sphere in prescribed
                        sinusoidal translation plus rotation.
"""
import math

import numpy as np

BASE_SEED = 2009


def seed_for(k):
    """Per-workload seed: 2009 * 10 + k."""
    return BASE_SEED * 10 + int(k)


def couette_annulus(scale=1.0, u_inner=0.01, tau=0.8, steps=5000):
    """48x48 annulus at scale 1: centre (24, 24), r1 = 8, r2 = 20 (all x scale)."""
    n = int(round(48 * scale))
    return {
        "lattice": "D2Q9", "nx": n, "ny": n, "nz": 1,
        "centre": (n / 2.0, n / 2.0, 0.0),
        "r1": 8.0 * scale, "r2": 20.0 * scale,
        "u_inner": float(u_inner), "tau": float(tau), "steps": int(steps),
        "rho0": 1.0,
    }


def cylinder_channel(nx=2048, ny=1024, radius=20.0, centre=(400.0, 512.0), u_max=0.05,
                     reynolds=100.0, tau=None, steps=20000, seed=None):
    """Channel with a cylinder; centre offset by U[0,1)^2 drawn from the seed.

    Re = u_max D / nu with D = 2 radius  =>  tau = 3 nu + 1/2 unless given.
    """
    rng = np.random.default_rng(seed_for(2) if seed is None else seed)
    dx, dy = rng.random(2)
    nu = u_max * 2.0 * radius / reynolds
    t = 3.0 * nu + 0.5 if tau is None else float(tau)
    return {
        "lattice": "D2Q9", "nx": int(nx), "ny": int(ny), "nz": 1,
        "centre": (centre[0] + dx, centre[1] + dy, 0.0), "radius": float(radius),
        "u_max": float(u_max), "tau": t, "steps": int(steps), "rho0": 1.0,
    }


def sphere_packing(n=256, r_min=6.0, r_max=12.0, solid_fraction=0.4, seed=None, max_attempts=200000):
    """Largest-first random sequential addition of non-overlapping spheres in a
    periodic n^3 box.  Radii are pre-drawn U[r_min, r_max] until the analytic solid
    fraction reaches the target, sorted descending, and each sphere is placed at a
    uniform random centre that does not overlap any placed sphere (periodic minimum
    image, strict non-overlap).  Returns (centres (k,3), radii (k,))."""
    rng = np.random.default_rng(seed_for(3) if seed is None else seed)
    vol = float(n) ** 3
    radii = []
    total = 0.0
    while total / vol < solid_fraction:
        r = rng.uniform(r_min, r_max)
        radii.append(r)
        total += 4.0 / 3.0 * math.pi * r ** 3
    radii = np.sort(np.array(radii))[::-1]
    centres = np.zeros((0, 3))
    placed_r = np.zeros(0)
    # coarse cell grid for neighbour candidates
    cell = 2.0 * r_max
    ncell = max(1, int(n // cell))
    cs = n / ncell
    buckets = {}
    for r in radii:
        for _ in range(max_attempts // 256 + 1):
            cand = rng.random((256, 3)) * n
            ok = np.ones(256, dtype=bool)
            if placed_r.size:
                # test every candidate against placed spheres in nearby cells
                cidx = np.floor(cand / cs).astype(int) % ncell
                for k in range(256):
                    near = []
                    cx, cy, cz = cidx[k]
                    for ox in (-1, 0, 1):
                        for oy in (-1, 0, 1):
                            for oz in (-1, 0, 1):
                                near.extend(buckets.get(((cx + ox) % ncell, (cy + oy) % ncell, (cz + oz) % ncell), ()))
                    if near:
                        near = np.array(near)
                        d = cand[k] - centres[near]
                        d -= n * np.round(d / n)
                        if np.any((d * d).sum(axis=1) <= (r + placed_r[near]) ** 2):
                            ok[k] = False
                            continue
                    break
            good = np.flatnonzero(ok)
            if good.size:
                c = cand[good[0]]
                key = tuple(np.floor(c / cs).astype(int) % ncell)
                buckets.setdefault(key, []).append(centres.shape[0])
                centres = np.vstack([centres, c])
                placed_r = np.append(placed_r, r)
                break
        else:
            raise RuntimeError("random sequential addition stalled")
    return centres, placed_r


def request_stream(n_requests=256, rate=None, seed=None, l_min=64, l_max=1024, steps=5000):
    """Served requests: half circular Couette (L x L), half cylinder channel (2L x L).

    Each request: {"kind", "L", "arrival", ...geometry}.  Arrival times are a
    Poisson process of the given rate (requests per second), drawn from a
    generator of their own so that the requests themselves do not depend on the
    rate; rate None gives all arrivals at t = 0.
    """
    base = seed_for(4) if seed is None else seed
    rng = np.random.default_rng(base)
    arrivals = np.random.default_rng(base + 1)
    reqs = []
    t = 0.0
    for k in range(n_requests):
        L = int(rng.integers(l_min, l_max + 1))
        kind = "couette" if k % 2 == 0 else "channel"
        if rate is not None:
            t += arrivals.exponential(1.0 / rate)
        if kind == "couette":
            s = L / 48.0
            req = {"kind": kind, "L": L, "nx": L, "ny": L, "centre": (L / 2.0, L / 2.0, 0.0),
                   "r1": L / 6.0, "r2": 5.0 * L / 12.0, "u_inner": 0.01, "tau": 0.8}
            del s
        else:
            R = max(3.0, 20.0 * L / 1024.0)
            off = rng.random(2)
            req = {"kind": kind, "L": L, "nx": 2 * L, "ny": L,
                   "centre": (400.0 * L / 1024.0 + off[0], 512.0 * L / 1024.0 + off[1], 0.0),
                   "radius": R, "u_max": 0.05, "tau": 0.6}
        req.update({"id": k, "arrival": t, "steps": int(steps), "lattice": "D2Q9"})
        reqs.append(req)
    return reqs


def moving_boxes(n_boxes=32, seed=None, side_min=96, side_max=192, r_min=10.0, r_max=16.0,
                 amplitude=8.0, period=2000.0, surface_speed=0.02, tau=0.8, steps=4000):
    """Periodic D3Q19 boxes, each with a sphere at the box centre moving as
    x_c(t) = x_0 + A sin(2 pi t / T) e, rotating at |Omega| = surface_speed / r about
    a random axis; e and the axis are random unit vectors from the seed."""
    rng = np.random.default_rng(seed_for(5) if seed is None else seed)
    boxes = []
    for k in range(n_boxes):
        side = int(rng.integers(side_min, side_max + 1))
        r = float(rng.uniform(r_min, r_max))
        e = rng.normal(size=3)
        e /= np.linalg.norm(e)
        ax = rng.normal(size=3)
        ax /= np.linalg.norm(ax)
        boxes.append({
            "id": k, "lattice": "D3Q19", "nx": side, "ny": side, "nz": side,
            "x0": (side / 2.0, side / 2.0, side / 2.0), "radius": r,
            "amplitude": float(amplitude), "period": float(period), "direction": tuple(e),
            "omega": tuple(ax * surface_speed / r), "tau": float(tau), "steps": int(steps),
            "rho0": 1.0,
        })
    return boxes
