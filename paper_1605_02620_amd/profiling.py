"""Summaries of rocprofv3 counter runs of the sweep kernel.

`summarize_traffic` reads the CSV output of two `rocprofv3 --pmc` runs of
`bench.py --copy-probe` (one with FETCH_SIZE, one with WRITE_SIZE), scales
each counter by what it reads for the probe's plain 1 GiB device copy, and
returns the HBM bytes per block_sweep launch.  The result is stamped with a
hash of the kernel source so that a stale measurement is never reported for
a changed kernel.

    python -m paper_1605_02620_amd.profiling <fetch_dir> <write_dir> <out.json> [instance]

(instance: the kernel instance in the form rsos_kernel_name reports, e.g.
block_sweep<8,32,8,256,int8,int16,0>; default: the instance that moves the
most bytes per launch).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(PKG, "csrc", "rsos_kernels.hpp")
COPY_BYTES = 1 << 30  # the probe copies one int32[16384^2] buffer


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def kernel_instance(rocprof_name: str) -> str:
    """A rocprofv3 kernel name in the form rsos_kernel_name reports, e.g.
    'void rsosk::block_sweep<8, 32, 8, 256, signed char, short, 0>(...)' ->
    'block_sweep<8,32,8,256,int8,int16,0>'."""
    n = rocprof_name.split("(")[0].strip()
    if n.startswith("void "):
        n = n[5:]
    n = n.replace("rsosk::", "").replace(" ", "")
    if "<" not in n:
        return n
    base, args = n.split("<", 1)
    types = {"signedchar": "int8", "unsignedchar": "uint8", "short": "int16", "int": "int32"}
    return base + "<" + ",".join(types.get(a, a) for a in args.rstrip(">").split(",")) + ">"


def _counter(dirname: str, name: str, instance: str | None = None):
    rows = list(csv.DictReader(open(os.path.join(dirname, "run_counter_collection.csv"))))
    per_kernel = {}
    for r in rows:
        if r["Counter_Name"] == name and "block_sweep" in r["Kernel_Name"]:
            if instance is None or kernel_instance(r["Kernel_Name"]) == instance:
                per_kernel.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    copies = sorted(float(r["Counter_Value"]) for r in rows
                    if r["Counter_Name"] == name and "copyBuffer" in r["Kernel_Name"])
    if not per_kernel or len(copies) < 5:
        raise ValueError(f"{dirname}: no block_sweep or probe-copy dispatches for {name}")
    # the given instance, else the one that moves the most bytes per launch
    kernel = max(per_kernel, key=lambda k: sum(per_kernel[k]) / len(per_kernel[k]))
    sweep = per_kernel[kernel]
    probe = sum(copies[-5:]) / 5.0  # the five 1 GiB copies are the largest
    scale = (COPY_BYTES / 1024.0) / probe
    return kernel, sum(sweep) / len(sweep) * 1024.0 * scale, scale


def summarize_traffic(fetch_dir: str, write_dir: str, instance: str | None = None) -> dict:
    kernel, fetch, sf = _counter(fetch_dir, "FETCH_SIZE", instance)
    _, write, sw = _counter(write_dir, "WRITE_SIZE", instance)
    return {"kernel": kernel, "kernel_source_sha256_16": kernel_hash(),
            "fetch_bytes_per_launch": round(fetch), "write_bytes_per_launch": round(write),
            "traffic_bytes_per_launch": round(fetch + write),
            "fetch_scale": round(sf, 4), "write_scale": round(sw, 4)}


def current_traffic(json_path: str):
    """Bytes per launch from a stored summary, or None if the kernel source
    changed since the counters were taken."""
    try:
        d = json.load(open(json_path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return d


if __name__ == "__main__":
    if len(sys.argv) not in (4, 5):
        print(__doc__)
        sys.exit(2)
    out = summarize_traffic(sys.argv[1], sys.argv[2], sys.argv[4] if len(sys.argv) == 5 else None)
    json.dump(out, open(sys.argv[3], "w"), indent=1)
    print(json.dumps(out))
