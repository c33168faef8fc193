"""Summaries of rocprofv3 output for profiles/: per-kernel trace statistics
and calibrated HBM traffic (FETCH_SIZE / WRITE_SIZE per dispatch, scaled by
the same counters on a plain device copy of known size).

    python -m paper_1210_7774_amd.profile_summary trace <run_kernel_stats.csv>
    python -m paper_1210_7774_amd.profile_summary traffic <fetch dir> <write dir> <cal fetch dir> <cal write dir>
        <out.json> <n> <kernel sources...>

The traffic record keeps, per timing class of the library ("pre_rr n=511",
"post n=4095", ...), the calibrated read and write bytes of one launch at the
finest level (the dispatches of each kernel that move the most data), and
the hash of the kernel sources they were taken on; bench.py reports them only
while the sources are unchanged.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
# kernel instantiation of the fused 3D passes -> the library's timing class
M3_CLASS = {("0", "0"): "pre_sweep", ("1", "0"): "pre_sweep", ("0", "1"): "pre_rr", ("1", "1"): "pre_rr",
            ("2", "0"): "post_corr", ("2", "2"): "post_norm", ("0", "2"): "post_norm"}


def short(name):
    m = re.search(r"k_march3d<(\w+), (\w+), (\d), (\d),", name)
    if m:
        return "k_march3d<%s,%s,head %s,tail %s>" % m.groups()
    m = re.search(r"k_march3dw<(\w+), (\w+), (\d), (\d), (\d)>", name)
    if m:
        return "k_march3dw<%s,%s,%s sweeps,head %s,tail %s>" % m.groups()
    return re.sub(r"\(.*", "", name)[:90]


def trace(path):
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    print("| kernel | calls | average | min | max | share |")
    print("|---|---|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        if float(r["TotalDurationNs"]) < 0.001 * tot:
            continue
        print("| `%s` | %s | %.2f us | %.2f us | %.2f us | %.1f %% |"
              % (short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                 float(r["MaxNs"]) / 1e3, 100 * float(r["TotalDurationNs"]) / tot))
    print("\ntotal kernel time %.2f ms" % (tot / 1e6))


def per_kernel(d, counter):
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
        if r["Counter_Name"] == counter:
            out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return out


def finest(vals):
    """Dispatches of the finest level: several levels share a kernel (and can
    share a grid size), the finest one moves the most data by far."""
    top = max(vals)
    sel = [v for v in vals if v >= 0.5 * top]
    return sum(sel) / len(sel)


def copy_kib(d, counter):
    return max(finest(x) for k, x in per_kernel(d, counter).items() if "elementwise" in k or "copy" in k.lower())


def traffic(fdir, wdir, cfdir, cwdir, out, n, sources):
    # 256 MiB copy: read and written once
    fs = 262144.0 / copy_kib(cfdir, "FETCH_SIZE")
    ws = 262144.0 / copy_kib(cwdir, "WRITE_SIZE")
    fk, wk = per_kernel(fdir, "FETCH_SIZE"), per_kernel(wdir, "WRITE_SIZE")
    kernels = {}
    for name in sorted(fk):
        m = re.search(r"k_march3d<\w+, \w+, (\d), (\d),", name)
        mw = re.search(r"k_march3dw<\w+, \w+, (\d), (\d), (\d)>", name)
        m2 = re.search(r"k_march2d<double, double, \d+, \d+, \d+, \d+, \w+, (\d), 1,", name)
        if m and m.groups() in M3_CLASS:
            cls = "%s n=%d" % (M3_CLASS[m.groups()], n)
        elif mw and mw.groups()[1:] in M3_CLASS:  # the wavefront passes: "w<sweeps>" + the class
            cls = "w%s%s n=%d" % (mw.group(1), M3_CLASS[mw.groups()[1:]], n)
        elif m2:
            cls = "%s n=%d" % ("pre" if m2.group(1) == "0" else "post", n)  # the finest FP64 march kernels
        else:
            continue
        rd = finest(fk[name]) * fs * 1024
        wr = finest(wk[name]) * ws * 1024
        if cls in kernels and kernels[cls]["read_bytes"] >= rd:
            continue
        kernels[cls] = {"read_bytes": rd, "write_bytes": wr, "kernel": short(name)}
    # (a kernel that runs only below the given level would be mislabelled
    # with its largest dispatch: keep the classes that move finest-level data)
    top = max(k["read_bytes"] + k["write_bytes"] for k in kernels.values())
    kernels = {c: k for c, k in kernels.items() if k["read_bytes"] + k["write_bytes"] >= 0.25 * top}
    for cls, k in sorted(kernels.items()):
        print("%-16s read %8.1f MB  write %8.1f MB  (%s)" % (cls, k["read_bytes"] / 1e6, k["write_bytes"] / 1e6,
                                                          k["kernel"]))
    h = hashlib.sha256()
    for fn in sources:
        h.update(open(os.path.join(CSRC, fn), "rb").read())
    rec = {"source_hash": h.hexdigest()[:16], "kernels": kernels, "fetch_scale": fs, "write_scale": ws,
           "note": "per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the finest-level kernels, scaled by a 256 MiB "
                   "device copy"}
    json.dump(rec, open(out, "w"), indent=1)
    print("scale: fetch %.3f write %.3f; source hash %s" % (fs, ws, rec["source_hash"]))


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2])
    else:
        traffic(*sys.argv[2:7], int(sys.argv[7]), sys.argv[8:])
