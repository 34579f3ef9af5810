"""Build liblbm.so (the HIP kernels and the C-ABI) for gfx950 in-tree.

    python -m paper_2009_04604_amd.build        # or build() from Python

Every build recompiles from source into paper_2009_04604_amd/liblbm.so.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liblbm.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-I" + os.path.join(HERE, "..", "include")]
# device code: gfx950 only; packed FP32 instructions disabled
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

# (source, object name, extra flags): the lattice kernels are built once per
# lattice; the D2Q9 build also holds the lattice-independent kernels and the
# lattice dispatch
SOURCES = [
    ("kernels.hip", "kernels_d2q9.o", ["-DLBM_LATTICE=D2Q9", "-DLBM_COMMON"]),
    ("kernels.hip", "kernels_d3q19.o", ["-DLBM_LATTICE=D3Q19"]),
    ("kernels.hip", "kernels_d3q27.o", ["-DLBM_LATTICE=D3Q27"]),
    ("moving.hip", "moving.o", []),
    ("noalloc.hip", "noalloc.o", []),
    ("api.cpp", "api.o", []),
    ("batch.cpp", "batch.o", []),
    ("geometry.cpp", "geometry.o", []),
    ("hostplan.cpp", "hostplan.o", []),
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout)
        raise RuntimeError(f"compilation failed: {os.path.basename(cmd[-1])}")
    return r.stdout


def build(verbose=False):
    """Compile every source (in parallel) and link liblbm.so."""
    import concurrent.futures
    os.makedirs(BUILD_DIR, exist_ok=True)
    cmds, objs = [], []
    for src, oname, extra in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD_DIR, oname)
        cmd = [HIPCC, *COMMON, *DEVICE, *extra, "-x", "hip", "-c", "-o", obj, path]
        if src.endswith(".cpp"):
            # host builder: no FMA contraction, so that the geometry arithmetic
            # rounds exactly like the plain double-precision definition
            cmd.insert(1, "-ffp-contract=off")
        cmds.append(cmd)
        objs.append(obj)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as pool:
        for out in pool.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs])
    os.replace(tmp, OUT)
    return OUT


def clean():
    shutil.rmtree(BUILD_DIR, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose=True))
