"""Turn two rocprofv3 counter runs of bench.py into per-launch HBM traffic of a 2D kernel.

Usage: python bench_traffic.py <step2d|stage2d> <variant2d> <stage_variant> <fetch_collection.csv> <write_collection.csv>
       python bench_traffic.py pair3d <variant3d> - <fetch_collection.csv> <write_collection.csv> [<calibration.json>]
       python bench_traffic.py valu <variant2d> <valu_counter_collection.csv>   (VALU issue of the whole-step kernel)
       python bench_traffic.py valu_stencils <valu_counter_collection.csv>   (the same per Laplacian and instance)

<variant2d>, <stage_variant> and <variant3d> are the per-precision kernel variants the counter runs
of bench.py were given (--variant2d, --stage-variant, --variant3d), e.g. f64:6,f32:3,mixed:3.

Counters are KiB per dispatch.  Each is scaled by what it reads for the plain copy kernel of
known size that bench.py runs (torch copy_ of a 1 GiB float64 tensor: 1 GiB read and 1 GiB
written), then averaged over all launches of the kernel for each precision.  A run whose own
large copies include other transfers (the 3D run uploads 1-2 GB fields) takes the factors from
the JSON of a 2D counter run of the same session instead (optional last argument).  The result goes
to profiles/traffic_<kind>_gp2d_2048.json together with a hash of the kernel's sources;
bench.py reports it only while the sources still match.
"""
import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_1109_1027_amd", "csrc")
GIB = float(1 << 30)

# source files each kernel is compiled from (its .hip and every header it includes)
SOURCES = {"stage2d": ["stage2d.hip", "tile2d.h", "point.h", "common.h", "kernels.h"],
           "step2d": ["step2d.hip", "step2d_impl.h", "step2d_f64.hip", "step2d_f32.hip", "step2d_mixed.hip", "wave2d.h",
                      "dpp.h", "point.h", "common.h", "kernels.h"],
           "pair3d": ["step3d.hip", "point.h", "common.h", "kernels.h"]}
KEYS = {"stage2d": {"f64": ["stage2d_kernel<double, double, double"], "f32": ["stage2d_kernel<float, float, float"],
                    "mixed": ["stage2d_kernel<double, float, double", "stage2d_kernel<float, float, double"]},
        "step2d": {"f64": ["step2d_kernel<double, double"], "f32": ["step2d_kernel<float, float"],
                   "mixed": ["step2d_kernel<float, double"]},
        "pair3d": {"f64": ["pair3d_kernel<double, double, double"], "f32": ["pair3d_kernel<float, float, float"],
                   "mixed": ["pair3d_kernel<double, float, double", "pair3d_kernel<float, float, double"]}}
NAMES = {"stage2d": "nlse::stage2d_kernel (mean over the four RK4-stage launches)",
         "step2d": "nlse::step2d_kernel (one launch per RK4 step)",
         "pair3d": "nlse::pair3d_kernel (mean over the two launches of an RK4 step)"}
WORKLOADS = {"stage2d": ("gp2d_2048", "2D GP, 2049^2 nodes, bench.py defaults"),
             "step2d": ("gp2d_2048", "2D GP, 2049^2 nodes, bench.py defaults"),
             "pair3d": ("gp3d_512", "3D GP, 513^3 nodes, bench.py defaults")}


def traffic_file(kind):
    return os.path.join(ROOT, "profiles", f"traffic_{kind}_{WORKLOADS[kind][0]}.json")


def _code_only(text):
    """Source text without comments and blank space: a comment edit does not change the kernel."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(" ".join(line.split()) for line in text.splitlines() if line.strip())


def source_sha(kind, root=CSRC):
    h = hashlib.sha256()
    for f in SOURCES[kind]:
        h.update(_code_only(open(os.path.join(root, f), encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def per_kernel(path, cname):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == cname:
            d[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
    return d


def main(kind, variant2d, stage_variant, fetch_csv, write_csv, calib_json=None):
    variants = stage_variant if kind == "stage2d" else variant2d
    var = {k: int(v) for k, v in (item.split(":") for item in variants.split(","))}
    F, W = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    if calib_json:
        sf = json.load(open(calib_json))["scale_factors"]
        fF, fW = sf["FETCH_SIZE"], sf["WRITE_SIZE"]
        calib = f"factors of {os.path.basename(calib_json)} (same session): " + sf["calibration"]
    else:
        big = lambda vals: [v for v in vals if v > 0.25 * GIB]
        cf, cw = big(F["__amd_rocclr_copyBuffer"]), big(W["__amd_rocclr_copyBuffer"])
        fF, fW = GIB / (sum(cf) / len(cf)), GIB / (sum(cw) / len(cw))
        calib = "torch copy_ of a 1 GiB float64 tensor: 1 GiB read, 1 GiB written"
    res, raw = {}, {}
    for prec, keys in KEYS[kind].items():
        fv = [v for k in F for key in keys if key in k for v in F[k]]
        wv = [v for k in W for key in keys if key in k for v in W[k]]
        if not fv:
            continue
        raw[prec] = {"fetch_bytes": sum(fv) / len(fv), "write_bytes": sum(wv) / len(wv), "launches": len(fv)}
        res[prec] = {"bytes": fF * raw[prec]["fetch_bytes"] + fW * raw[prec]["write_bytes"],
                     "variant": var.get(prec)}
    if kind == "pair3d":
        args = (f"--precs f32 --steps 5 --warmup 1 --no-cpu-baseline --batch-steps 0 --no-learned --no-stencils "
                f"--no-msd --no-stage3d --steps3d 3 --variant3d {variant2d}")
        d = "prof3d"
    else:
        args = (f"--steps 5 --warmup 1 --no-cpu-baseline --n3d 0 --batch-steps 0 --no-learned --no-stencils "
                f"--no-msd --variant2d {variant2d} --stage-variant {stage_variant}")
        d = "prof"
    out = {"kernel": NAMES[kind], "workload": WORKLOADS[kind][1],
           "source_sha": source_sha(kind), "sources": SOURCES[kind],
           "per_launch_bytes": res, "raw_counter_bytes": raw,
           "scale_factors": {"FETCH_SIZE": fF, "WRITE_SIZE": fW, "calibration": calib},
           "commands": [f"cd /tmp && rocprofv3 --pmc {c} -d /tmp/{d}_{c} -o pmc --output-format csv "
                        f"-- python3 $R/bench.py {args}" for c in ("FETCH_SIZE", "WRITE_SIZE")]}
    json.dump(out, open(traffic_file(kind), "w"), indent=1)
    print(json.dumps(out, indent=1))


def valu_file():
    return os.path.join(ROOT, "profiles", "valu_step2d_gp2d_2048.json")


def valu(variant2d, csv_path, simds=1024, xcds=8):
    """VALU issue of the whole-step kernel from one counter run (SQ_INSTS_VALU, SQ_INSTS_SALU,
    SQ_INSTS_VALU_FLOPS_FP64/FP32, SQ_WAVES, GRBM_GUI_ACTIVE): issue = SQ_INSTS_VALU x 4 cycles
    (a wave64 instruction on a 16-lane SIMD) / (SIMDs x GRBM_GUI_ACTIVE per XCD)."""
    var = {k: int(v) for k, v in (item.split(":") for item in variant2d.split(","))}
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(csv_path)):
        agg[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    res = {}
    for prec, keys in KEYS["step2d"].items():
        names = [k for k in agg for key in keys if key in k]
        if not names:
            continue
        c = {n: sum(v) / len(v) for n, v in agg[names[0]].items()}
        cycles = c["GRBM_GUI_ACTIVE"] / xcds
        res[prec] = {"variant": var.get(prec), "valu_issue": c["SQ_INSTS_VALU"] * 4 / (simds * cycles),
                     "insts_valu": c["SQ_INSTS_VALU"], "insts_salu": c["SQ_INSTS_SALU"], "waves": c["SQ_WAVES"],
                     "cycles_per_xcd": cycles,
                     "executed_flops": 64 * (c["SQ_INSTS_VALU_FLOPS_FP64"] + c["SQ_INSTS_VALU_FLOPS_FP32"])}
    out = {"kernel": NAMES["step2d"], "source_sha": source_sha("step2d"), "per_launch": res,
           "command": "cd /tmp && rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_VALU_FLOPS_FP64 "
                      "SQ_INSTS_VALU_FLOPS_FP32 SQ_ACTIVE_INST_VALU SQ_BUSY_CU_CYCLES SQ_WAVES GRBM_GUI_ACTIVE "
                      "-d /tmp/prof_valu -o pmc --output-format csv -- python3 $R/bench.py --steps 5 "
                      "--warmup 1 --no-cpu-baseline --n3d 0 --batch-steps 0 --no-learned --no-stencils --no-msd "
                      f"--variant2d {variant2d}"}
    json.dump(out, open(valu_file(), "w"), indent=1)
    print(json.dumps(out, indent=1))


def valu_stencils(csv_path, simds=1024, xcds=8):
    """VALU counters of the whole-step kernel for each Laplacian (template argument ST: 0 2SHOC,
    1 non-compact, 2 CD) and each kernel instance of a counter run of bench.py with its stencil
    section on; the same counters and issue formula as valu()."""
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(csv_path)):
        if "step2d_kernel<" in r["Kernel_Name"]:
            agg[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lap = {"0": "2shoc", "1": "noncompact", "2": "cd"}
    res = {}
    for name, cs in sorted(agg.items()):
        m = re.search(r"step2d_kernel<(\w+), (\w+), (\d+), (\d+), (\d+), false>", name)
        if not m:
            continue
        c = {n: sum(v) / len(v) for n, v in cs.items()}
        cycles = c["GRBM_GUI_ACTIVE"] / xcds
        key = f"<{m.group(1)}, {m.group(2)}, Q={m.group(3)}, rows in flight {m.group(4)}> {lap[m.group(5)]}"
        res[key] = {"dispatches": len(cs["SQ_WAVES"]), "valu_issue": c["SQ_INSTS_VALU"] * 4 / (simds * cycles),
                    "insts_valu": c["SQ_INSTS_VALU"], "insts_salu": c["SQ_INSTS_SALU"], "waves": c["SQ_WAVES"],
                    "cycles_per_xcd": cycles}
    out = {"kernel": "nlse::step2d_kernel, 2SHOC / non-compact / CD Laplacians", "source_sha": source_sha("step2d"),
           "per_launch": res,
           "command": "cd /tmp && rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_VALU_FLOPS_FP64 "
                      "SQ_INSTS_VALU_FLOPS_FP32 SQ_ACTIVE_INST_VALU SQ_BUSY_CU_CYCLES SQ_WAVES GRBM_GUI_ACTIVE "
                      "-d /tmp/prof_valu_st -o pmc --output-format csv -- python3 $R/bench.py --steps 5 "
                      "--warmup 1 --no-cpu-baseline --n3d 0 --batch-steps 0 --no-learned --no-msd --precs f64,f32"}
    json.dump(out, open(os.path.join(ROOT, "profiles", "valu_step2d_stencils_gp2d_2048.json"), "w"), indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    if sys.argv[1] == "valu":
        valu(sys.argv[2], sys.argv[3])
    elif sys.argv[1] == "valu_stencils":
        valu_stencils(sys.argv[2])
    else:
        main(*sys.argv[1:7])
