"""Summaries of rocprofv3 output for the committed profiles.

- ``stats``: the kernel statistics of a ``rocprofv3 --kernel-trace --stats``
  run (``*_kernel_stats.csv``) as a markdown table, with the command that
  produced it.
- ``pmc``: HBM traffic of one kernel per dispatch from two counter runs
  (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``, KiB per dispatch), each
  scaled by what the same counter reads for a plain device copy of known
  size (the copy's bytes divided by its counter reading), as JSON.  The JSON
  records the hash of the step kernel's sources (``kernel_source_hash``) so
  that a reader can tell when the counters no longer describe the kernel.
- ``valu``: vector, transcendental, FP64 and matrix-core instruction counts
  of the f*_M solver and network-start kernels per 64 sites, from counter
  runs over the 4096 x 2048 moment field, as JSON (with the hash of those
  kernels' sources): per kernel the median over the field's dispatches
  (those with at least half the largest vector count).

Usage (from the repository root):
  python -m paper_0705_4371_amd.profiling stats DIR --command "..." --title "..."
  python -m paper_0705_4371_amd.profiling pmc --kernel k_step --fetch DIR --write DIR \\
      --copy-fetch DIR --copy-write DIR --algorithmic-bytes B --workload "..." --command "..."
  python -m paper_0705_4371_amd.profiling valu --dirs DIR [DIR ...] --sites N --command "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STEP_SOURCES = ("lbm_step.hpp", "lbm_step_f32q9.hip", "lbm_step_f64q9.hip", "lbm_device.hpp", "lbm_launch.hpp",
                "lbm_fstar.hpp", "lbm_fstar_dev.hpp", "lbm_fstar_site.hpp")


FSTAR_SOURCES = ("lbm_fstar.hip", "lbm_fstar.hpp", "lbm_fstar_dev.hpp", "lbm_fstar_site.hpp", "lbm_device.hpp",
                 "lbm_mlp_infer.hip", "lbm_mlp_dev.hpp")
# the solver kernels by start, and the network start
FSTAR_KERNELS = {"plain_newton": "k_fstar<4>(", "rest": "k_fstar<0>(", "closed_form": "k_fstar<1>(", "mlp": "k_fstar<2>(",
                 "exact_start": "k_fstar<3>(", "mlp_forward": "k_mlp_warm("}
VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VALU_FMA_F64",
                 "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_MFMA")


def _hash(names) -> str:
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_0705_4371_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_source_hash() -> str:
    """Hash of the sources the fused step kernel is compiled from."""
    return _hash(STEP_SOURCES)


def fstar_source_hash() -> str:
    """Hash of the sources of the f*_M solver and network-start kernels."""
    return _hash(FSTAR_SOURCES)


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def _rows(path: str) -> list:
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def stats_markdown(directory: str, command: str, title: str, top: int = 30) -> str:
    rows = _rows(_one(os.path.join(directory, "**", "*kernel_stats.csv")))
    out = ["# %s" % title, "", "Command (repository root REPO on the GPU machine, after "
           "`cd /tmp && export TMPDIR=/tmp`):", "", "    " + command, "",
           "| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"].replace("|", "\\|")
        if len(name) > 90:
            name = name[:90] + "..."
        out.append("| `%s` | %s | %.1f | %.1f | %.1f | %.2f%% |" % (
            name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    return "\n".join(out) + "\n"


def counter_per_dispatch(directory: str, kernel: str, counter: str, skip_first: int = 0):
    """Mean counter value (KiB) over the dispatches whose name contains `kernel`."""
    rows = _rows(_one(os.path.join(directory, "**", "*counter_collection.csv")))
    vals = [float(r["Counter_Value"]) for r in rows
            if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter]
    vals = vals[skip_first:]
    if not vals:
        raise ValueError("no %s dispatches of %s in %s" % (counter, kernel, directory))
    return sum(vals) / len(vals), len(vals)


def pmc_summary(a) -> dict:
    fetch, nf = counter_per_dispatch(a.fetch, a.kernel_match, "FETCH_SIZE", a.skip_first)
    write, nw = counter_per_dispatch(a.write, a.kernel_match, "WRITE_SIZE", a.skip_first)
    cf, _ = counter_per_dispatch(a.copy_fetch, a.copy_kernel, "FETCH_SIZE")
    cw, _ = counter_per_dispatch(a.copy_write, a.copy_kernel, "WRITE_SIZE")
    copy_bytes = float(a.copy_bytes)
    ff, fw = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    rd, wr = fetch * 1024.0 * ff, write * 1024.0 * fw
    return {
        "kernel": a.kernel, "workload": a.workload, "kernel_source_hash": kernel_source_hash(),
        "fetch_size_kib_per_dispatch": round(fetch, 1), "write_size_kib_per_dispatch": round(write, 1),
        "dispatches_averaged": min(nf, nw),
        "copy_calibration": {"what": a.copy_what, "fetch_size_kib": cf, "write_size_kib": cw,
                             "fetch_factor": round(ff, 5), "write_factor": round(fw, 5)},
        "hbm_read_bytes_per_launch": int(rd), "hbm_write_bytes_per_launch": int(wr),
        "hbm_bytes_per_launch": int(rd + wr), "algorithmic_bytes_per_launch": int(a.algorithmic_bytes),
        "ratio_to_algorithmic": round((rd + wr) / float(a.algorithmic_bytes), 5),
        "commands": a.command,
    }


def valu_summary(a) -> dict:
    # dispatch (run, id) -> (kernel name, {counter: value}); the runs need
    # not dispatch in the same order, so each counter is taken as the median
    # over the dispatches of a kernel in the run that counted it
    per = {}
    for k, d in enumerate(a.dirs):
        for r in _rows(_one(os.path.join(d, "**", "*counter_collection.csv"))):
            name, cnt = per.setdefault((k, int(r["Dispatch_Id"])), (r["Kernel_Name"], {}))
            cnt[r["Counter_Name"]] = float(r["Counter_Value"])
    waves = a.sites / 64.0
    out = {"workload": a.workload, "sites": a.sites, "fstar_source_hash": fstar_source_hash(),
           "step_source_hash": kernel_source_hash(),
           "unit": "instructions per wavefront of 64 sites", "commands": a.command, "kernels": {}}
    kernels = dict(kv.split("=", 1) for kv in a.kernel) if a.kernel else FSTAR_KERNELS
    for key, match in kernels.items():
        c, nd = {}, 0
        for k in VALU_COUNTERS:
            vals = [cnt[k] for name, cnt in per.values() if match in name and k in cnt]
            if not vals:
                break
            # the field's dispatches (the largest), not the smaller training-pair solve
            top = max(vals)
            vals = [v for v in vals if v >= 0.5 * top]
            c[k] = statistics.median(vals)
            if k == "SQ_INSTS_VALU":  # the dispatches counted (a zero counter selects them all)
                nd = len(vals)
        if len(c) != len(VALU_COUNTERS):
            continue
        out["kernels"][key] = {
            "kernel": match.rstrip("("), "dispatches": nd,
            "valu": round(c["SQ_INSTS_VALU"] / waves, 1),
            "transcendental": round((c["SQ_INSTS_VALU_TRANS_F32"] + c["SQ_INSTS_VALU_TRANS_F64"]) / waves, 1),
            "fp64": round((c["SQ_INSTS_VALU_FMA_F64"] + c["SQ_INSTS_VALU_ADD_F64"] + c["SQ_INSTS_VALU_MUL_F64"])
                          / waves, 1),
            "mfma": round(c["SQ_INSTS_MFMA"] / waves, 1)}
        # HBM counters, when a run counted them: raw KiB per dispatch (median)
        for k in ("FETCH_SIZE", "WRITE_SIZE"):
            vals = [cnt[k] for name, cnt in per.values() if match in name and k in cnt]
            if vals:
                top = max(vals)
                out["kernels"][key][k.lower() + "_kib"] = round(statistics.median([v for v in vals if v >= 0.5 * top]), 1)
    return out


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--command", required=True)
    s.add_argument("--title", required=True)
    p = sub.add_parser("pmc")
    p.add_argument("--kernel", required=True, help="name written into the summary")
    p.add_argument("--kernel-match", required=True, help="substring of the dispatch name")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--copy-fetch", required=True)
    p.add_argument("--copy-write", required=True)
    p.add_argument("--copy-kernel", default="copyBuffer")
    p.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    p.add_argument("--copy-what", default="torch copy of 2^28 float32 (1 GiB read, 1 GiB written)")
    p.add_argument("--algorithmic-bytes", type=float, required=True)
    p.add_argument("--workload", required=True)
    p.add_argument("--skip-first", type=int, default=0)
    p.add_argument("--command", action="append", required=True)
    v = sub.add_parser("valu")
    v.add_argument("--dirs", nargs="+", required=True, help="counter runs (any split of the counters)")
    v.add_argument("--sites", type=int, default=4096 * 2048)
    v.add_argument("--workload", default="f*_M moment field 4096x2048 (rho in [0.5, 1.5], |u| <= 0.1, "
                                          "2E/rho within 5% of isothermal), residual <= 1e-10")
    v.add_argument("--command", action="append", required=True)
    v.add_argument("--kernel", action="append", default=[],
                   help="KEY=SUBSTRING of a dispatch name (repeatable; default: the solver and network kernels)")
    a = ap.parse_args(argv)
    if a.what == "valu":
        json.dump(valu_summary(a), sys.stdout, indent=1)
        sys.stdout.write("\n")
    elif a.what == "stats":
        sys.stdout.write(stats_markdown(a.dir, a.command, a.title))
    else:
        json.dump(pmc_summary(a), sys.stdout, indent=1)
        sys.stdout.write("\n")


if __name__ == "__main__":
    main()
