"""Summaries of rocprofv3 output for the solver's kernels.

    python -m paper_2008_08825_amd.profsummary stats DIR [--top 20]
        markdown table of the kernel statistics (``--kernel-trace --stats``
        run writing CSV under DIR)
    python -m paper_2008_08825_amd.profsummary traffic FETCH_DIR WRITE_DIR \\
            --copy-mib 1024 --key n8192_clustered/fp64 [--json profiles/traffic.json]
        average FETCH_SIZE / WRITE_SIZE per dispatch (one ``--pmc`` run per
        counter), scaled by what the same counters read for the plain
        device copy of COPY_MIB MiB in the same run; merged into the JSON
        file the benchmark reads (keyed by workload/form/kernel and the hash
        of the Jacobi kernel source, so the figures are ignored once the
        kernels change).
    python -m paper_2008_08825_amd.profsummary mfma PMC_DIR [--bench BENCH_JSON]
        executed MFMA flops per dispatch from a ``--pmc
        SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_INSTS_VALU_MFMA_MOPS_F32`` run (each
        count is 512 flops), and for the Jacobi kernels the benchmark's
        kernel-side figure (exec_flops_per_launch in BENCH_JSON, the JSON line
        the same run printed) beside it.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# op name in the kernel symbol -> name used by the benchmark
BENCH_NAMES = {"GramOp": "jacobi_gram", "EigOp": "jacobi_eig", "RotOp": "jacobi_rotate"}


def jacobi_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_2008_08825_amd", "csrc", "jacobi.hip"), "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def short_name(name: str) -> str:
    """'void bse::k_grp<bse::(anonymous namespace)::RotOp<float> >(...)' -> 'RotOp<float> [grouped]'."""
    m = re.search(r"k_(one|grp)<(?:bse::)?(?:\(anonymous namespace\)::)?([A-Za-z0-9_]+)(<[^>]*>)?", name)
    if m:
        kind = "grouped" if m.group(1) == "grp" else "single"
        return f"{m.group(2)}{m.group(3) or ''} [{kind}]"
    m = re.search(r"(k_[A-Za-z0-9_]+|__amd_rocclr_[A-Za-z0-9_]+)", name)
    return m.group(1) if m else name[:60]


def bench_key(name: str):
    m = re.search(r"(GramOp|EigOp|RotOp)<(double|float)>", name)
    if not m:
        return None
    return BENCH_NAMES[m.group(1)], ("fp64" if m.group(2) == "double" else "mixed")


def find(pattern_dir: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(pattern_dir, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise SystemExit(f"no *{suffix} under {pattern_dir}")
    return sorted(hits)[0]


def stats(dirname: str, top: int = 20):
    path = find(dirname, "kernel_stats.csv")
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["| kernel | calls | total ms | average us | share |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        t = float(r["TotalDurationNs"])
        out.append(f"| {short_name(r['Name'])} | {r['Calls']} | {t / 1e6:.1f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {100.0 * t / total:.2f}% |")
    out.append(f"| (all kernels) | {sum(int(r['Calls']) for r in rows)} | {total / 1e6:.1f} | | 100% |")
    return "\n".join(out)


def counters(dirname: str):
    path = find(dirname, "counter_collection.csv")
    per = defaultdict(list)
    for r in csv.DictReader(open(path)):
        per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return per


def traffic(fetch_dir, write_dir, copy_mib, key, json_path=None):
    fetch = counters(fetch_dir)
    write = counters(write_dir)
    copy = [k for k in fetch if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no copy kernel in the FETCH_SIZE run (use --copy-calibration)")
    kib = copy_mib * 1024.0
    cf = max(fetch[copy[0]])
    cw = max(write[copy[0]])
    f_scale = kib / cf
    w_scale = kib / cw
    lines = [f"Calibration: the {copy_mib} MiB device copy reads FETCH_SIZE = {cf:,.0f} KiB and "
             f"WRITE_SIZE = {cw:,.0f} KiB per dispatch for {kib:,.0f} KiB moved each way: "
             f"FETCH_SIZE x {f_scale:.2f}, WRITE_SIZE x {w_scale:.2f}.", "",
             "| kernel | dispatches | FETCH_SIZE KiB / dispatch (raw) | read MiB / dispatch | "
             "WRITE_SIZE KiB / dispatch | written MiB / dispatch |", "|---|---|---|---|---|---|"]
    result = {}
    for name in sorted(fetch, key=lambda k: -sum(fetch[k])):
        if name in copy or name not in write:
            continue
        fv, wv = fetch[name], write[name]
        fa = sum(fv) / len(fv)
        wa = sum(wv) / len(wv)
        rd = fa * f_scale / 1024.0
        wr = wa * w_scale / 1024.0
        lines.append(f"| {short_name(name)} | {len(fv)} | {fa:,.0f} | {rd:,.2f} | {wa:,.0f} | {wr:,.2f} |")
        bk = bench_key(name)
        if bk:
            result[f"{key.split('/')[0]}/{bk[1]}/{bk[0]}"] = {
                "read_bytes_per_launch": rd * 2 ** 20, "write_bytes_per_launch": wr * 2 ** 20,
                "bytes_per_launch": (rd + wr) * 2 ** 20, "dispatches": len(fv),
                "fetch_scale": f_scale, "write_scale": w_scale}
    if json_path:
        try:
            data = json.load(open(json_path))
        except (OSError, ValueError):
            data = {}
        h = jacobi_source_hash()
        if data.get("source_sha1") != h:
            data = {"source_sha1": h, "kernels": {}}
        data["kernels"].update(result)
        with open(json_path, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    return "\n".join(lines)


def mfma(dirname: str, bench_json=None):
    path = find(dirname, "counter_collection.csv")
    per = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        per[name][r["Counter_Name"]] += float(r["Counter_Value"])
        disp[name].add(r.get("Dispatch_Id") or r.get("Correlation_Id") or len(disp[name]))
    formula = {}
    if bench_json:
        with open(bench_json) as f:
            line = [ln for ln in f if ln.strip().startswith("{")][-1]
        b = json.loads(line)
        for form in ("fp64", "mixed", "mixed_polish"):
            if form not in b:
                continue
            for sect, prec in (("kernels", "fp64" if form == "fp64" else "mixed"), ("polish_kernels", "fp64")):
                for k, v in b[form].get(sect, {}).items():
                    if v.get("exec_flops_per_launch"):
                        formula[(k, prec)] = v["exec_flops_per_launch"]
    out = ["| kernel | dispatches | MFMA F64 GFLOP / dispatch | MFMA F32 GFLOP / dispatch | "
           "kernel-side formula GFLOP / launch | counter / formula |", "|---|---|---|---|---|---|"]
    rows = sorted(per, key=lambda k: -(per[k].get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)
                                       + per[k].get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0)))
    for name in rows:
        d = max(1, len(disp[name]))
        f64 = per[name].get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512 / d
        f32 = per[name].get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) * 512 / d
        if f64 == 0.0 and f32 == 0.0:
            continue
        bk = bench_key(name)
        fm = formula.get(bk) if bk else None
        ratio = f"{(f64 + f32) / fm:.3f}" if fm else ""
        out.append(f"| {short_name(name)} | {d} | {f64 / 1e9:,.2f} | {f32 / 1e9:,.2f} | "
                   f"{fm / 1e9:,.2f} | {ratio} |" if fm else
                   f"| {short_name(name)} | {d} | {f64 / 1e9:,.2f} | {f32 / 1e9:,.2f} | | |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--top", type=int, default=20)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--key", required=True, help="workload/form the runs measured")
    t.add_argument("--json", default=None)
    m = sub.add_parser("mfma")
    m.add_argument("dir")
    m.add_argument("--bench", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats(a.dir, a.top))
    elif a.cmd == "mfma":
        print(mfma(a.dir, a.bench))
    else:
        print(traffic(a.fetch_dir, a.write_dir, a.copy_mib, a.key, a.json))


if __name__ == "__main__":
    sys.exit(main())
