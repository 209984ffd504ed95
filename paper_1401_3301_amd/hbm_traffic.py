"""Turn rocprofv3 FETCH_SIZE / WRITE_SIZE counter files into HBM bytes.

    python -m paper_1401_3301_amd.hbm_traffic <fetch_dir> <write_dir> \\
        <copy_fetch_dir> <copy_write_dir> <kernel_substring> <op> <out.json>

Each directory is a rocprofv3 ``--pmc ... --output-format csv`` output.
FETCH_SIZE and WRITE_SIZE are read in KiB per dispatch, averaged over the
dispatches of the named kernel on the measured workload (those of the small
warm-up mesh are left out), and scaled by the ratio of the true bytes of
a plain device copy (``bench.py --copy-calibration``: 2^29 bytes read and
written per copy) to what the same counters report for that copy.  The
result, with the hash of the kernel sources the counters were taken on, is
written as JSON for bench.py.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import sys


def counter_mean(d: str, counter: str, kernel_sub: str) -> float:
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    per = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter or kernel_sub not in r["Kernel_Name"]:
                continue
            per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for kernel '{kernel_sub}' under {d}")
    # bench.py first runs the kernel on a small warm-up mesh: keep the
    # dispatches of the measured workload only (within 4x of the largest)
    top = max(per.values())
    vals = [v for v in per.values() if v >= 0.25 * top]
    return sum(vals) / len(vals)


def main(argv):
    fd, wd, cfd, cwd, ksub, op, out = argv[1:8]
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from bench import kernel_sha

    copy_bytes = 1 << 29
    f_kib = counter_mean(fd, "FETCH_SIZE", ksub)
    w_kib = counter_mean(wd, "WRITE_SIZE", ksub)
    cf_kib = counter_mean(cfd, "FETCH_SIZE", "copy")
    cw_kib = counter_mean(cwd, "WRITE_SIZE", "copy")
    f_scale = copy_bytes / (cf_kib * 1024.0)
    w_scale = copy_bytes / (cw_kib * 1024.0)
    res = {
        "kernel": ksub, "op": op, "kernel_sha": kernel_sha(), "n": 128,
        "fetch_kib": f_kib, "write_kib": w_kib,
        "copy_fetch_kib": cf_kib, "copy_write_kib": cw_kib,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "fetch_bytes": f_kib * 1024.0 * f_scale, "write_bytes": w_kib * 1024.0 * w_scale,
    }
    res["traffic_bytes"] = res["fetch_bytes"] + res["write_bytes"]
    json.dump(res, open(out, "w"), indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main(sys.argv)
