"""Turns rocprofv3 memory-counter runs into the traffic summary bench.py reads.

Usage (after the two counter runs of the bench and of its copy probe):
  python traffic_summary.py <fetch_bench_dir> <write_bench_dir> \
      <fetch_copy_dir> <write_copy_dir> <kernel> <workload> <launches_per_step>

FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch.  Each is scaled by
the ratio (bytes actually copied) / (counter reading) of the copy probe, a
1 GiB device-to-device copy, so the result is in HBM bytes as the copy kernel
would count them.  Writes profiles/<kernel>_<workload>_traffic.json and .md.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30


def counter_per_dispatch(d: str, counter: str, name_part: str) -> float:
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    vals = []
    for fn in files:
        for r in csv.DictReader(open(fn)):
            if name_part in r.get("Kernel_Name", "") and r.get("Counter_Name") == counter:
                vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} rows for {name_part} under {d}")
    return sum(vals) / len(vals)


def main(argv) -> int:
    fb, wb, fc, wc, kernel, workload, _launches = argv
    kname = {"pass_a": "k_pass_a", "pass_b": "k_pass_b", "pass_c": "k_pass_c"}[kernel]
    fetch = counter_per_dispatch(fb, "FETCH_SIZE", kname) * 1024
    write = counter_per_dispatch(wb, "WRITE_SIZE", kname) * 1024
    copy_f = counter_per_dispatch(fc, "FETCH_SIZE", "copy") * 1024
    copy_w = counter_per_dispatch(wc, "WRITE_SIZE", "copy") * 1024
    kf, kw = COPY_BYTES / copy_f, COPY_BYTES / copy_w
    sys.path.insert(0, ROOT)
    from bench import kernel_source_sha1
    out = {"kernel": kernel, "workload": workload,
           "fetch_bytes_per_dispatch_raw": fetch, "write_bytes_per_dispatch_raw": write,
           "copy_probe_fetch_factor": kf, "copy_probe_write_factor": kw,
           "hbm_bytes_per_launch": int(fetch * kf + write * kw),
           "source_sha1": kernel_source_sha1(kernel)}
    base = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic")
    with open(base + ".json", "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
