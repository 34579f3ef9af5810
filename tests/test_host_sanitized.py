"""The host side of the library under the address and undefined-behaviour
sanitizers, on the CPU: the geometry builder (geometry.cpp) and the cut-link
validation and planning (hostplan.cpp) are compiled with g++
-fsanitize=address,undefined together with a driver (tests/sanitize/
host_driver.cpp) that builds the workloads' geometries, plans their links,
checks every planned record, checks the compact layout's source-row table by
forming every pull's slot the way the step kernel does and comparing it with
the source node's slot counted directly, and feeds corrupted link lists that
must be refused.  Any sanitizer report aborts the driver.  The builder's output is
also compared, to the bit, with the production library's (hipcc build) on the
same shapes."""
import os
import shutil
import re
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_04604_amd", "csrc")
LAT = {"D2Q9": 0, "D3Q19": 1, "D3Q27": 2}
VARIANT = {"FQ": 0, "F": 1, "UQ": 2, "U": 3, "HWBB": 4}


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("san") / "host_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Werror",
           "-I" + os.path.join(ROOT, "include"), "-o", exe, os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
           os.path.join(CSRC, "geometry.cpp"), os.path.join(CSRC, "hostplan.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _h(x):
    return float(x).hex()


class Script:
    """Commands for the driver and the same shapes for the production builder."""

    def __init__(self, tmp):
        self.lines, self.cases, self.tmp = [], [], tmp

    def geom(self, lat, nx, ny, nz, periodic=(True, True, True), outlet=-1):
        per = sum(int(bool(p)) << a for a, p in enumerate(periodic))
        self.lines.append(f"geom {LAT[lat]} {nx} {ny} {nz} {per} {outlet}")
        self.cur = {"args": (lat, nx, ny, nz, periodic, None if outlet < 0 else outlet), "shapes": []}

    def round(self, kind, c, r, inside=True, V=(0, 0, 0), Om=(0, 0, 0)):
        vals = " ".join(_h(v) for v in (*c, r))
        self.lines.append(f"{kind} {vals} {int(inside)} " + " ".join(_h(v) for v in (*V, *Om)))
        self.cur["shapes"].append((kind, c, r, inside, V, Om))

    def spheres(self, c, r):
        self.lines.append(f"spheres {len(r)}")
        self.lines += [" ".join(_h(v) for v in (*cc, rr)) for cc, rr in zip(c, r)]
        self.cur["shapes"].append(("spheres", c, r))

    def face(self, f, q=0.5, uw=(0, 0, 0), profile=0):
        self.lines.append(f"face {f} {_h(q)} " + " ".join(_h(v) for v in uw) + f" {profile}")
        self.cur["shapes"].append(("face", f, q, uw, profile))

    def build(self, plans=(("FQ", 0.01, 1),)):
        prefix = os.path.join(self.tmp, f"case{len(self.cases)}")
        self.lines.append(f"build {prefix}")
        for v, qc, f64 in plans:
            self.lines.append(f"plan {VARIANT[v]} {_h(qc)} {f64}")
        self.lines.append("end")
        self.cases.append((prefix, self.cur))


def _production(B, case):
    lat, nx, ny, nz, periodic, outlet = case["args"]
    g = B.Geometry(lat, nx, ny, nz, periodic=periodic, outlet_face=outlet)
    for s in case["shapes"]:
        if s[0] == "sphere":
            g.add_sphere(s[1], s[2], s[3], V=s[4], Omega=s[5])
        elif s[0] == "cylinder":
            g.add_cylinder(s[1], s[2], s[3], V=s[4], Omega=s[5])
        elif s[0] == "spheres":
            g.add_spheres(s[1], s[2])
        else:
            g.add_face_wall(s[1], s[2], uw=s[3], profile=s[4])
    mask, links = g.build()
    g.close()
    return mask, links


def test_host_library_under_sanitizers(driver, tmp_path):
    from paper_2009_04604_amd import binding as B
    s = Script(str(tmp_path))
    # annulus with a rotating inner wall (moving-wall planning, FP64 and FP32 weights)
    p = synth.couette_annulus()
    s.geom("D2Q9", p["nx"], p["ny"], 1)
    s.round("sphere", p["centre"], p["r1"], True, Om=(0, 0, p["u_inner"] / p["r1"]))
    s.round("sphere", p["centre"], p["r2"], False)
    s.build((("FQ", 0.01, 1), ("U", 0.01, 0), ("HWBB", 0.0, 1)))
    # cylinder channel: parabolic inlet, walls, zero-gradient outlet
    p = synth.cylinder_channel(nx=300, ny=120, radius=9.0, centre=(60.0, 60.0))
    s.geom("D2Q9", p["nx"], p["ny"], 1, periodic=(False, False, True), outlet=1)
    s.round("sphere", p["centre"], p["radius"], True)
    s.face(0, 0.5, (p["u_max"], 0, 0), 1)
    s.face(2, 0.5)
    s.face(3, 0.5)
    s.build()
    # sphere packing (bucketed spheres), D3Q19 and D3Q27
    c, r = synth.sphere_packing(n=40, r_min=3.0, r_max=6.0, solid_fraction=0.4, seed=11)
    for lat in ("D3Q19", "D3Q27"):
        s.geom(lat, 40, 40, 40)
        s.spheres(c, r)
        s.build((("FQ", 0.01, 1), ("F", 0.01, 0)))
    # coaxial cylinders with a ball between them; a moving sphere across a periodic corner
    s.geom("D3Q27", 48, 48, 10)
    s.round("cylinder", (24.0, 24.0, 0.0), 8.0, True, Om=(0, 0, 0.004))
    s.round("cylinder", (24.0, 24.0, 0.0), 20.0, False)
    s.round("sphere", (38.1, 24.3, 2.7), 1.9, True)
    s.build()
    s.geom("D3Q19", 24, 20, 16)
    s.round("sphere", (1.2, 19.5, 15.0), 4.3, True, V=(0.01, -0.02, 0.005), Om=(0.001, 0.002, -0.003))
    s.build((("UQ", 0.01, 1),))
    # rows of several segments with a periodic x-wrap (the source-row table's row
    # ends), and an outlet on a y face (source rows clamped onto it)
    s.geom("D3Q19", 150, 12, 10)
    s.round("sphere", (3.0, 4.0, 3.0), 2.6, True)
    s.round("sphere", (148.5, 1.0, 6.0), 2.2, True)
    s.round("sphere", (70.0, 5.0, 2.0), 2.5, True)
    s.build()
    s.geom("D2Q9", 130, 40, 1, periodic=(True, False, True), outlet=3)
    s.round("sphere", (64.5, 20.0, 0.0), 6.0, True)
    s.face(2, 0.5)
    s.build()
    # degenerate lattices: one node, all solid, nodes exactly on the wall
    s.geom("D3Q19", 1, 1, 1)
    s.build()
    s.geom("D3Q19", 3, 3, 3)
    s.round("sphere", (1.0, 1.0, 1.0), 10.0, True)
    s.build()
    s.geom("D2Q9", 9, 9, 1)
    s.round("sphere", (4.0, 4.0, 0.0), 2.0, True)
    s.build()
    s.lines.append("bad")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([driver], input="\n".join(s.lines) + "\n", capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0 and r.stdout.rstrip().endswith("ALL OK"), r.stdout[-3000:] + r.stderr[-3000:]
    assert "FAIL" not in r.stdout
    assert r.stdout.count("plan ok") == 15
    assert r.stdout.count("source rows ok") == 15
    # every lane of every segment pulls inside the population array (the
    # compact step lets lanes that are not fluid pull as well)
    assert len(re.findall(r"source rows ok \d+ in range [1-9]\d*", r.stdout)) == 15
    # the sanitized build agrees with the production library to the bit
    for prefix, case in s.cases:
        mask, links = _production(B, case)
        got_mask = np.fromfile(prefix + ".mask", np.uint8)
        assert np.array_equal(got_mask, mask)
        assert np.array_equal(np.fromfile(prefix + ".node", np.int64), links["node"])
        assert np.array_equal(np.fromfile(prefix + ".dir", np.int8).astype(np.int64), links["dir"])
        assert np.array_equal(np.fromfile(prefix + ".q", np.float64), links["q"])
        assert np.array_equal(np.fromfile(prefix + ".uw", np.float64).reshape(-1, 3), links["uw_t"])
        assert np.array_equal(np.fromfile(prefix + ".uw1", np.float64).reshape(-1, 3), links["uw_t1"])
        assert np.array_equal(np.fromfile(prefix + ".shape", np.int32).astype(np.int64), links["shape"])
    # the degenerate cases did what they should
    counts = [ln.split()[1:] for ln in r.stdout.splitlines() if ln.startswith("built")]
    assert counts[-3] == ["1", "0"] and counts[-2] == ["0", "0"]
    q = np.fromfile(s.cases[-1][0] + ".q", np.float64)
    assert (q == 1.0).any()
