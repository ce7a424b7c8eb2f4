"""Turn rocprofv3 counter and trace CSVs into per-kernel figures.

HBM traffic: `FETCH_SIZE` and `WRITE_SIZE` (KiB per dispatch) are scaled by
what the same counters read for a plain device copy of known size run in the
same process (bench.py --calib-copy: 4 GiB read + 4 GiB written by the
runtime's copy kernel).  The result is bytes per launch, keyed by the hash of
the kernel source it was measured on, so a stale figure is never reported.

    python -m paper_2505_22313_amd.profiling traffic <fetch_dir> <write_dir>
    python -m paper_2505_22313_amd.profiling stats <trace_dir>
"""

import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "asm_kernels.hip")
CALIB_KERNEL = "__amd_rocclr_copyBuffer"
CALIB_BYTES = 4 * 1024 ** 3

PASS_NAMES = {"k_pass_a_fwd": "pass_a_fwd", "k_pass_b_fwd": "pass_b_fwd", "k_pass_c": "pass_c",
              "k_pass_b_inv": "pass_b_inv", "k_pass_a_inv": "pass_a_inv"}


def kernel_source_hash():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def pass_name(kernel_name):
    for k, v in PASS_NAMES.items():
        if "dop::" + k + "<" in kernel_name:
            return v
    return None


def _csv(directory, suffix):
    files = glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def counters(directory):
    """{kernel name: {counter: [value per dispatch]}}"""
    out = defaultdict(lambda: defaultdict(list))
    for r in _csv(directory, "counter_collection.csv"):
        out[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def traffic(fetch_dir, write_dir):
    f = counters(fetch_dir)
    w = counters(write_dir)
    fk = [v for k, v in f.items() if k.startswith(CALIB_KERNEL)]
    wk = [v for k, v in w.items() if k.startswith(CALIB_KERNEL)]
    if not fk or not wk:
        raise RuntimeError("calibration copy kernel not found: run bench.py with --calib-copy")
    f_factor = CALIB_BYTES / (1024.0 * max(fk[0]["FETCH_SIZE"]))
    w_factor = CALIB_BYTES / (1024.0 * max(wk[0]["WRITE_SIZE"]))
    res = {"source_sha": kernel_source_hash(), "fetch_factor": round(f_factor, 4),
           "write_factor": round(w_factor, 4), "kernels": {}}
    for k, v in f.items():
        name = pass_name(k)
        if not name or k not in w:
            continue
        fb = sum(v["FETCH_SIZE"]) / len(v["FETCH_SIZE"]) * 1024.0 * f_factor
        wb = sum(w[k]["WRITE_SIZE"]) / len(w[k]["WRITE_SIZE"]) * 1024.0 * w_factor
        res["kernels"][name] = {"kernel": k, "dispatches": len(v["FETCH_SIZE"]),
                                "fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb}
    return res


def stats(trace_dir):
    rows = _csv(trace_dir, "kernel_stats.csv")
    return [{"name": r["Name"], "calls": int(r["Calls"]), "avg_ms": float(r["AverageNs"]) / 1e6,
             "min_ms": float(r["MinNs"]) / 1e6, "max_ms": float(r["MaxNs"]) / 1e6,
             "share": float(r["Percentage"])} for r in rows]


def main(argv):
    if len(argv) >= 3 and argv[0] == "traffic":
        print(json.dumps(traffic(argv[1], argv[2]), indent=1))
    elif len(argv) >= 2 and argv[0] == "stats":
        print(json.dumps(stats(argv[1]), indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
