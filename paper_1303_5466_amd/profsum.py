"""Summaries of rocprofv3 CSV output (the text kept under profiles/).

    python -m paper_1303_5466_amd.profsum trace DIR [--title T] [--command C]
        per-kernel statistics of a --kernel-trace run, per factor build, and
        the level-pipeline GEMM launches on their own
    python -m paper_1303_5466_amd.profsum traffic --fetch D --write D \
            --cal-fetch D --cal-write D --copy-bytes B [--command C ...]
        HBM bytes per level-pipeline GEMM launch from FETCH_SIZE / WRITE_SIZE
        (KiB per dispatch), each scaled by what the same counter reads for a
        plain copy of B bytes (read B, write B)

A factor build starts at its leaf_F_kernel dispatch.  The factor's level
GEMMs (Schur products, Gauss-Jordan updates, E blocks, root) are the
gemm_kernel instantiations with role 0 (either tile width, product and
split-K reduce dispatches alike); interpolation, solve and library GEMMs are
roles 1, 2 and 3 of the same code.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
GEMM = "gemm_kernel<double, 0"      # name prefix: gemm_kernel<double, 0, 64> and <double, 0, 128>


def _short(name: str) -> str:
    n = name.replace("void ", "").replace("rsd::(anonymous namespace)::", "")
    return re.sub(r"\(.*", "", n).strip()


def _rows(d: str, suffix: str):
    files = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    with open(files[0], newline="") as fh:
        return list(csv.DictReader(fh))


def _dispatches(rows):
    out = []
    for r in rows:
        out.append(dict(name=_short(r["Kernel_Name"]), queue=r["Queue_Id"],
                        start=int(r["Start_Timestamp"]), end=int(r["End_Timestamp"]),
                        dispatch=r.get("Dispatch_Id"), row=r))
    out.sort(key=lambda x: x["start"])
    return out


def level_gemm_ids(disp, gemm: str = GEMM):
    """Dispatch ids of the factor's level GEMM launches, and the number of builds."""
    starts = [d["start"] for d in disp if d["name"].startswith("leaf_F_kernel")]
    return {d["dispatch"] for d in disp if d["name"].startswith(gemm + ",")}, len(starts)


def trace_summary(d: str, title: str, command: str, gemm: str = GEMM) -> str:
    disp = _dispatches(_rows(d, "kernel_trace.csv"))
    ids, nb = level_gemm_ids(disp, gemm)
    agg = defaultdict(lambda: [0, 0.0])
    for x in disp:
        a = agg[x["name"]]
        a[0] += 1
        a[1] += (x["end"] - x["start"]) / 1e3
    lv = [(x["end"] - x["start"]) / 1e3 for x in disp if x["dispatch"] in ids]
    nb = max(nb, 1)
    out = [f"# {title}", "", "Command (repository root, one MI355X):", "", "```", command, "```", "",
           f"{nb} factor builds in the trace (per-build columns divide by {nb}).", "",
           "| kernel | calls/build | ms/build | avg us |", "|---|---:|---:|---:|"]
    for k, (n, us) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| `{k}` | {n / nb:.0f} | {us / 1e3 / nb:.3f} | {us / n:.1f} |")
    if lv:
        out += ["", f"Level GEMM dispatches (`{gemm}, *>`: the factor's Schur, Gauss-Jordan, E and root products):",
                "", f"- launches: {len(lv)} ({len(lv) / nb:.0f} per build)",
                f"- average duration: {sum(lv) / len(lv):.2f} us",
                f"- total per build: {sum(lv) / 1e3 / nb:.3f} ms"]
    return "\n".join(out) + "\n"


def _counter_avg(d: str, counter: str, select):
    rows = [r for r in _rows(d, "counter_collection.csv") if r["Counter_Name"] == counter]
    disp = _dispatches(rows)
    vals = [float(x["row"]["Counter_Value"]) for x in disp if select(x, disp)]
    return (sum(vals) / len(vals), len(vals)) if vals else (float("nan"), 0)


def traffic_summary(a) -> str:
    def level(x, disp, cache={}):
        key = id(disp)
        if key not in cache:
            cache[key] = level_gemm_ids(disp)[0]
        return x["dispatch"] in cache[key]

    def copy(x, disp):
        return re.search(a.copy_kernel, x["name"]) is not None

    f_kib, nf = _counter_avg(a.fetch, "FETCH_SIZE", level)
    w_kib, nw = _counter_avg(a.write, "WRITE_SIZE", level)
    cf_kib, _ = _counter_avg(a.cal_fetch, "FETCH_SIZE", copy)
    cw_kib, _ = _counter_avg(a.cal_write, "WRITE_SIZE", copy)
    sf = cf_kib * 1024 / a.copy_bytes
    sw = cw_kib * 1024 / a.copy_bytes
    fetch_b = f_kib * 1024 / sf
    write_b = w_kib * 1024 / sw
    with open(os.path.join(HERE, "csrc", "k_gemm.hip"), "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    out = ["# HBM traffic of the level GEMM launches — 256x256 Laplace, float64", "",
           "Commands (repository root, one MI355X; one counter per run):", "", "```"]
    out += a.command
    out += ["```", "",
            f"Copy calibration: a {a.copy_bytes:.0f} B elementwise copy reads FETCH_SIZE = {cf_kib:.0f} KiB "
            f"and WRITE_SIZE = {cw_kib:.0f} KiB, so the scale factors are {sf:.3f} (fetch) and "
            f"{sw:.3f} (write); per-launch counter values are divided by them.", "",
            f"- level GEMM launches sampled: {nf} (fetch), {nw} (write)",
            f"- FETCH_SIZE per launch: {f_kib:.1f} KiB -> {fetch_b:.0f} B",
            f"- WRITE_SIZE per launch: {w_kib:.1f} KiB -> {write_b:.0f} B", "",
            f"traffic_bytes_per_launch = {fetch_b + write_b:.0f}",
            f"k_gemm.hip sha256 = {digest}"]
    return "\n".join(out) + "\n"


def read_traffic(path: str):
    """(bytes per launch, k_gemm.hip digest) recorded in a traffic summary, or None."""
    try:
        txt = open(path).read()
    except OSError:
        return None
    m1 = re.search(r"traffic_bytes_per_launch = ([0-9.e+]+)", txt)
    m2 = re.search(r"k_gemm.hip sha256 = ([0-9a-f]+)", txt)
    if not (m1 and m2):
        return None
    return float(m1.group(1)), m2.group(1)


def gemm_source_digest() -> str:
    with open(os.path.join(HERE, "csrc", "k_gemm.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", default="Kernel statistics")
    t.add_argument("--command", default="")
    t.add_argument("--gemm", default=GEMM, help="kernel name prefix of the level GEMM to summarise")
    f = sub.add_parser("traffic")
    f.add_argument("--fetch", required=True)
    f.add_argument("--write", required=True)
    f.add_argument("--cal-fetch", required=True)
    f.add_argument("--cal-write", required=True)
    f.add_argument("--copy-bytes", type=float, required=True)
    f.add_argument("--copy-kernel", default="elementwise")
    f.add_argument("--command", action="append", default=[])
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        sys.stdout.write(trace_summary(a.dir, a.title, a.command, a.gemm))
    else:
        sys.stdout.write(traffic_summary(a))


if __name__ == "__main__":
    main()
