"""Summaries of rocprofv3 output for the apply kernels (used to write profiles/).

  python -m paper_1004_3354_amd.profsum stats <kernel_stats.csv>
      per-kernel dispatch count and average duration (from --kernel-trace --stats)
  python -m paper_1004_3354_amd.profsum traffic <fetch counter_collection.csv>
          <write counter_collection.csv> <pmc-pass json line file> <workload>
      HBM bytes per apply launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
      each scaled by the factor that makes the same counter read the known
      4 D bytes for the plain copy kernel in the same run.
"""
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

APPLY_KERNELS = ("k_apply", "k_cs<", "k_csb<", "k_rt<", "k_upb<")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def source_hash():
    h = hashlib.sha256()
    for f in ("apply.hip", "ed_internal.h", "tables.hip"):
        h.update(open(os.path.join(ROOT, "paper_1004_3354_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def stats(path):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        name = r.get("Name") or r.get("KernelName") or r.get("Kernel_Name")
        calls = int(r.get("Calls", 0))
        avg_ns = float(r.get("AverageNs", r.get("Average_Ns", 0.0)))
        out.append((name, calls, avg_ns))
    out.sort(key=lambda t: -t[1] * t[2])
    return out


def _per_dispatch(path, counter):
    vals = defaultdict(list)
    for r in csv.DictReader(open(path)):
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or r.get("KernelName")
        cn = r.get("Counter_Name") or r.get("Counter-Name")
        if cn != counter:
            continue
        did = int(r.get("Dispatch_Id") or r.get("Dispatch-Id") or 0)
        vals[name].append((did, float(r.get("Counter_Value") or r.get("Counter-Value"))))
    return vals


def traffic(fetch_csv, write_csv, info_json, workload):
    info = json.loads([l for l in open(info_json) if l.startswith("{")][-1])
    steps, cb = info["steps"], info["copy_bytes_each_way"]
    res = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        v = _per_dispatch(path, counter)
        copy = [x for n, l in v.items() if "copy" in n.lower() or "elementwise" in n.lower() for x in l]
        copy = sorted(copy)[-steps:]
        apply_names = [n for n in v if any(k in n for k in APPLY_KERNELS)]
        # the last `steps` dispatches of each apply kernel are the timed ones
        per_launch = 0.0
        for n in apply_names:
            l = sorted(v[n])[-steps:]
            per_launch += sum(c for _, c in l) / len(l)
        copy_kib = sum(c for _, c in copy) / max(len(copy), 1)
        factor = (cb / 1024.0) / copy_kib if copy_kib > 0 else float("nan")
        res[counter] = {"apply_kib_per_launch": per_launch, "copy_kib": copy_kib, "factor": factor,
                        "bytes": per_launch * 1024.0 * factor, "kernels": apply_names}
    total = res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"]
    return {workload: {"source_hash": source_hash(), "bytes_per_launch": total,
                       "fetch_bytes": res["FETCH_SIZE"]["bytes"], "write_bytes": res["WRITE_SIZE"]["bytes"],
                       "fetch_factor": res["FETCH_SIZE"]["factor"], "write_factor": res["WRITE_SIZE"]["factor"],
                       "algorithmic_bytes": 8 * info["D"], "schedule": info["schedule"],
                       "kernels": res["FETCH_SIZE"]["kernels"]}}


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        for n, c, a in stats(sys.argv[2])[:25]:
            print("%6d  %12.2f us  %s" % (c, a / 1e3, n[:120]))
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(*sys.argv[2:6]), indent=1))
