"""Summaries of rocprofv3 output for the committed profiles.

kernel_stats(csv)                     -> per-kernel calls / average ns
traffic(fetch_csv, write_csv, ...)    -> HBM bytes per dispatch of a kernel,
                                         scaled by the counters of a copy
                                         kernel of known size

FETCH_SIZE and WRITE_SIZE are read in KiB per dispatch from two separate
`rocprofv3 --pmc` runs of the same command.  The copy kernel
(`copy_kernel`, launched by bench.py on 4 GiB buffers) moves a known number
of bytes, so bytes_known / counter_KiB is the scale factor of each counter.
"""
from __future__ import annotations

import csv
import collections
import hashlib
import json
import os
import re
import sys


def kernel_stats(path):
    out = {}
    for r in csv.DictReader(open(path)):
        out[r["Name"]] = dict(calls=int(r["Calls"]), avg_ns=float(r["AverageNs"]),
                              total_ns=float(r["TotalDurationNs"]), pct=float(r["Percentage"]))
    return out


def counter_per_dispatch(path, counter):
    """{kernel name: [value per dispatch, ...]} for one counter."""
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return per


def _match(d, pattern):
    return {k: v for k, v in d.items() if re.search(pattern, k)}


def traffic(fetch_csv, write_csv, kernel_pattern, copy_pattern="copy_kernel", copy_bytes=4 << 30):
    fetch = counter_per_dispatch(fetch_csv, "FETCH_SIZE")
    write = counter_per_dispatch(write_csv, "WRITE_SIZE")

    def mean(vals):
        return sum(vals) / len(vals)

    cf = [v for k, vs in _match(fetch, copy_pattern).items() for v in vs]
    cw = [v for k, vs in _match(write, copy_pattern).items() for v in vs]
    kf = [v for k, vs in _match(fetch, kernel_pattern).items() for v in vs]
    kw = [v for k, vs in _match(write, kernel_pattern).items() for v in vs]
    scale_f = copy_bytes / (mean(cf) * 1024.0)
    scale_w = copy_bytes / (mean(cw) * 1024.0)
    return dict(fetch_kib_per_dispatch=mean(kf), write_kib_per_dispatch=mean(kw),
                copy_fetch_kib=mean(cf), copy_write_kib=mean(cw),
                scale_fetch=scale_f, scale_write=scale_w,
                bytes_per_launch=mean(kf) * 1024.0 * scale_f + mean(kw) * 1024.0 * scale_w,
                dispatches=(len(kf), len(kw)))


def sweep_source_sha(root):
    src = os.path.join(root, "paper_1702_08521_amd", "csrc", "sweep.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


if __name__ == "__main__":
    print(json.dumps(kernel_stats(sys.argv[1]), indent=1))
