"""Summaries of rocprofv3 output for the step kernel.

    python -m paper_2009_04604_amd.profiling stats  <kernel_stats.csv>  [--match step_kernel]
    python -m paper_2009_04604_amd.profiling pmc    <counter_collection.csv> --match step_kernel \\
            --copy-kernel copy --copy-bytes B

``stats`` prints the per-kernel call count and mean duration from
``rocprofv3 --kernel-trace --stats`` (the ``*_kernel_stats.csv`` file).
``pmc`` prints, per counter, the mean value per dispatch of the matching kernel
and of a plain copy kernel of known size (bytes read = bytes written = B), and
the HBM bytes per launch of the kernel after scaling each counter by what it
reads for the copy (FETCH_SIZE and WRITE_SIZE are reported in KiB).
"""
import argparse
import collections
import csv
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/kernels.hip", "csrc/elibb.hpp", "csrc/storage.hpp", "csrc/lattice.hpp", "csrc/internal.hpp"]


def kernel_source_sha():
    """sha256 over the sources the step kernel is compiled from."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stats(path, match=None):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        name = r.get("Name") or r.get("KernelName") or r.get("Kernel_Name")
        if match and match not in name:
            continue
        calls = int(float(r["Calls"]))
        avg_ns = float(r["AverageNs"])
        out.append((name, calls, avg_ns, float(r.get("TotalDurationNs", avg_ns * calls))))
    return out


def pmc(path, match, copy_match=None):
    """Mean counter value per dispatch of the kernel; summed over all dispatches
    of the copy (the runtime may split one copy into several dispatches)."""
    rows = list(csv.DictReader(open(path)))
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        name = r["Kernel_Name"]
        key = "kernel" if match in name else ("copy" if copy_match and copy_match in name else None)
        if key is None:
            continue
        acc[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = {}
    for k, d in acc.items():
        out[k] = {c: (sum(v) if k == "copy" else sum(v) / len(v)) for c, v in d.items()}
        out[k]["dispatches"] = float(max(len(v) for v in d.values()))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "pmc", "sha"])
    ap.add_argument("path", nargs="?", help="csv file (pmc: comma-separated list, one per counter run)")
    ap.add_argument("--match", default="step_kernel")
    ap.add_argument("--copy-kernel", default=None)
    ap.add_argument("--copy-bytes", type=float, default=None)
    a = ap.parse_args()
    if a.mode == "sha":
        print(kernel_source_sha())
        return
    if a.mode == "stats":
        for name, calls, avg, tot in stats(a.path, a.match):
            print(f"{name[:90]:90s} calls={calls:6d} mean_us={avg / 1e3:10.3f} total_ms={tot / 1e6:10.3f}")
        return
    res = {}
    for path in a.path.split(","):
        for key, d in pmc(path, a.match, a.copy_kernel).items():
            res.setdefault(key, {}).update(d)
    print(f"kernel_source_sha256: {kernel_source_sha()}")
    for key, d in res.items():
        for c, v in sorted(d.items()):
            print(f"{key}.{c}: {v:.1f}")
    if a.copy_bytes and "copy" in res and "kernel" in res:
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            if c in res["copy"] and c in res["kernel"]:
                factor = res["copy"][c] * 1024.0 / a.copy_bytes
                print(f"copy_factor.{c}: {factor:.4f}")
                print(f"kernel_bytes_per_launch.{c}: {res['kernel'][c] * 1024.0 / factor:.0f}")


if __name__ == "__main__":
    main()
