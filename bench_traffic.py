"""Turn two rocprofv3 counter runs of bench.py into per-launch HBM traffic of the 2D stage kernel.

Usage: python bench_traffic.py <fetch_counter_collection.csv> <write_counter_collection.csv>
Counters are KiB per dispatch.  Each is scaled by what it reads for the plain copy kernel
of known size that bench.py runs (torch copy_ of a 1 GiB float64 tensor: 1 GiB read and
1 GiB written), then averaged over all stage launches of each precision.
"""
import collections
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
GIB = float(1 << 30)
KEYS = {"f64": ["stage2d_kernel<double, double, double"], "f32": ["stage2d_kernel<float, float, float"],
        "mixed": ["stage2d_kernel<double, float, double", "stage2d_kernel<float, float, double"]}


def per_kernel(path, cname):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == cname:
            d[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
    return d


def main(fetch_csv, write_csv):
    F, W = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    big = lambda vals: [v for v in vals if v > 0.25 * GIB]
    cf, cw = big(F["__amd_rocclr_copyBuffer"]), big(W["__amd_rocclr_copyBuffer"])
    fF, fW = GIB / (sum(cf) / len(cf)), GIB / (sum(cw) / len(cw))
    res, raw = {}, {}
    for prec, keys in KEYS.items():
        fv = [v for k in F for key in keys if key in k for v in F[k]]
        wv = [v for k in W for key in keys if key in k for v in W[k]]
        if not fv:
            continue
        raw[prec] = {"fetch_bytes": sum(fv) / len(fv), "write_bytes": sum(wv) / len(wv)}
        res[prec] = fF * raw[prec]["fetch_bytes"] + fW * raw[prec]["write_bytes"]
    src = os.path.join(ROOT, "paper_1109_1027_amd", "csrc", "stage2d.hip")
    out = {"kernel": "nlse::stage2d_kernel (mean over the four RK4-stage launches)",
           "workload": "2D GP, 2049^2 nodes, bench.py defaults",
           "source_sha": hashlib.sha256(open(src, "rb").read()).hexdigest()[:16],
           "per_launch_bytes": res, "raw_counter_bytes": raw,
           "scale_factors": {"FETCH_SIZE": fF, "WRITE_SIZE": fW,
                             "calibration": "torch copy_ of a 1 GiB float64 tensor: 1 GiB read, 1 GiB written"},
           "commands": [
               "cd /tmp && rocprofv3 --pmc FETCH_SIZE -d $R/gpurun_out/prof_fetch -o fetch --output-format csv "
               "-- python3 $R/bench.py --steps 5 --warmup 1 --no-cpu-baseline",
               "cd /tmp && rocprofv3 --pmc WRITE_SIZE -d $R/gpurun_out/prof_write -o write --output-format csv "
               "-- python3 $R/bench.py --steps 5 --warmup 1 --no-cpu-baseline"]}
    json.dump(out, open(os.path.join(ROOT, "profiles", "traffic_stage2d_gp2d_2048.json"), "w"), indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2])
