"""HBM traffic of the hot kernels from rocprofv3 hardware counters.

Two counter runs of the native runner (one with FETCH_SIZE, one with
WRITE_SIZE; the counters cannot share a pass) each also time a plain
device-to-device copy of known size (`irgl_run --calibrate MB`).  The copy's
counter readings give the scale from counter units to bytes; the scaled
per-dispatch averages of the kernel are its measured HBM traffic per launch.

  python -m paper_1607_05707_amd.profiling traffic \\
      --fetch-db F_results.db --write-db W_results.db --calib-mb 1024 \\
      --kernel 'persistent_kernel<256, irgl::SsspOp>' --workload rmat22 \\
      --command '...' --out profiles/traffic_rmat22_sssp.json

The JSON records a digest of the HIP sources; bench.py reports the traffic
only while the sources still have that digest (a changed kernel makes the
old counters stale).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import subprocess
import sys
import tempfile
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_KERNEL = "__amd_rocclr_copyBuffer"


# The translation unit that defines and launches the profiled kernels: every
# header under csrc/ and irgl.hip (other .hip / .cpp files, such as the
# native runner, hold other kernels or the harness and do not change these).
def digest_files():
    return sorted(glob.glob(os.path.join(CSRC, "*.h"))) + [os.path.join(CSRC, "irgl.hip")]


def source_digest() -> str:
    """sha256 over the sources of the profiled kernels (file names and contents)."""
    h = hashlib.sha256()
    for path in digest_files():
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_rows(db: str, counter: str):
    """(kernel name, value) of every dispatch's `counter` in a rocpd database."""
    with tempfile.TemporaryDirectory() as tmp:
        subprocess.run(["rocpd2csv", "-i", db, "-d", tmp, "-o", "c"], check=True,
                       stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        paths = glob.glob(os.path.join(tmp, "*counter_collection*.csv"))
        if not paths:
            raise SystemExit(f"no counter table in {db}")
        out = []
        with open(paths[0]) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    out.append((r["Kernel_Name"], float(r["Counter_Value"])))
        return out


def per_kernel(rows, kernel_substr: str):
    vals = [v for k, v in rows if kernel_substr in k]
    return vals


def traffic(args) -> int:
    calib_kib = args.calib_mb * 1024.0
    res = {}
    for name, db, counter in (("fetch", args.fetch_db, "FETCH_SIZE"), ("write", args.write_db, "WRITE_SIZE")):
        rows = counter_rows(db, counter)
        copy = max(v for k, v in rows if COPY_KERNEL in k)  # the calibration copy is the largest copy
        vals = per_kernel(rows, args.kernel)
        if not vals:
            raise SystemExit(f"kernel {args.kernel!r} not found in {db}")
        factor = calib_kib / copy
        res[name] = {"counter": counter, "dispatches": len(vals), "avg_kib": sum(vals) / len(vals),
                     "calib_copy_kib": copy, "factor": factor,
                     "bytes_per_launch": sum(vals) / len(vals) * 1024.0 * factor}
    out = {
        "kernel": args.kernel,
        "workload": args.workload,
        "fetch": res["fetch"],
        "write": res["write"],
        "traffic_bytes_per_launch": res["fetch"]["bytes_per_launch"] + res["write"]["bytes_per_launch"],
        "source_digest": source_digest(),
        "command": args.command,
        "calibration": f"device-to-device copy of {args.calib_mb} MiB (reads and writes {args.calib_mb} MiB)",
    }
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
    return 0


def load_traffic(path: str):
    """The recorded traffic per launch, or None when missing or stale."""
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest():
        return None
    return rec


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch-db", required=True)
    t.add_argument("--write-db", required=True)
    t.add_argument("--calib-mb", type=float, required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--command", required=True, help="the profiled command, recorded in the JSON")
    t.add_argument("--out", required=True)
    sub.add_parser("digest")
    args = ap.parse_args(argv)
    if args.cmd == "digest":
        print(source_digest())
        return 0
    return traffic(args)


if __name__ == "__main__":
    sys.exit(main())
