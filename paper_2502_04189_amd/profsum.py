"""Summaries of rocprofv3 runs: per-kernel average duration from a
kernel-trace run (``--kernel-trace --stats --output-format csv``) and HBM
bytes per dispatch from two counter runs (``--pmc FETCH_SIZE`` and
``--pmc WRITE_SIZE``), written as a short markdown table and a JSON file
that bench.py reads for its roofline's ``traffic``.

The byte counters are calibrated in the same runs against kernels of known
traffic: ``pcx::k_min_slot`` (the density minimum) reads exactly one FP64 field,
and torch's fill kernel writes exactly one FP64 field of the workload (its
size is given on the command line).

    python -m paper_2502_04189_amd.profsum --name fp64_512cube_step \\
        --trace DIR --fetch DIR --write DIR --field-bytes 1073741824 \\
        --cmd "rocprofv3 ..." [--cmd ...] --out profiles

With --counters DIR (repeatable) and --kernel NAME (repeatable) it writes a
table of SQ instruction and wait counters per kernel instead.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")


def src_hash(prefix: str = "pcx_") -> str:
    """sha256 (first 16 hex) of the kernel sources whose name starts with
    prefix: pcx_ for the pressure-correction step and its batch, flow_ for
    the substep, varcoef_ for the variable-coefficient projection."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(CSRC, prefix + "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def _csv(d: str, suffix: str):
    fs = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not fs:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    rows = []
    for f in fs:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def kernel_stats(d: str):
    """name -> (calls, average ms) from a --stats run."""
    out = {}
    for r in _csv(d, "kernel_stats.csv"):
        out[r["Name"]] = (int(r["Calls"]), float(r["AverageNs"]) * 1e-6)
    return out


def counter_means(d: str, counter: str):
    """name -> mean per dispatch of one counter (the values rocprofv3 prints;
    a counter summed over several instances is added up per dispatch)."""
    per = {}
    for r in _csv(d, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        key = (r["Kernel_Name"], r.get("Dispatch_Id", r.get("Correlation_Id")))
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    acc = {}
    for (name, _), v in per.items():
        s, n = acc.get(name, (0.0, 0))
        acc[name] = (s + v, n + 1)
    return {k: s / n for k, (s, n) in acc.items()}


def _ref(vals: dict, prefix_or_part: str):
    for k, v in vals.items():
        if k.startswith(prefix_or_part) or prefix_or_part in k:
            return k, v
    raise KeyError(f"calibration kernel {prefix_or_part!r} not in the counter run")


def summarize(name, trace, fetch, write, field_bytes, cmds, out_dir, prefix="pcx_", notes="", top=12):
    ks = kernel_stats(trace)
    fe = counter_means(fetch, "FETCH_SIZE") if fetch else {}
    wr = counter_means(write, "WRITE_SIZE") if write else {}
    lines = [f"# rocprofv3 summary: {name}", "", "Commands (from the repository root, on one MI355X):", "", "```"]
    lines += list(cmds) + ["```", ""]
    lines.append(f"Kernel sources hash (sha256 of csrc/{prefix}*, first 16 hex): `{src_hash(prefix)}`")
    lines.append("")
    kernels = {}
    if fe and wr:
        fk, fv = _ref(fe, "pcx::k_min_slot")
        wk, wv = _ref(wr, "FillFunc")
        ffac = field_bytes / (fv * 1024.0)
        wfac = field_bytes / (wv * 1024.0)
        lines.append("Byte counters are KiB per dispatch, calibrated in the same runs: "
                     f"`{fk}` reads exactly {field_bytes / 2**30:.3f} GiB and reports FETCH_SIZE = "
                     f"{fv:.0f} KiB (factor {ffac:.3f}); a torch fill writes exactly {field_bytes / 2**30:.3f} GiB "
                     f"and reports WRITE_SIZE = {wv:.0f} KiB (factor {wfac:.3f}).")
        lines.append("")
        lines.append("| Kernel | calls | avg ms | fetched GiB | written GiB | TB/s (counted bytes) |")
        lines.append("|---|---|---|---|---|---|")
    else:
        ffac = wfac = None
        lines.append("| Kernel | calls | avg ms | total ms |")
        lines.append("|---|---|---|---|")
    for kname, (calls, ms) in sorted(ks.items(), key=lambda kv: -kv[1][0] * kv[1][1])[:top]:
        short = kname if len(kname) <= 90 else kname[:87] + "..."
        if ffac is not None and kname in fe and kname in wr:
            fb = fe[kname] * 1024.0 * ffac
            wb = wr[kname] * 1024.0 * wfac
            kernels[kname] = {"ms": ms, "fetch_bytes": fb, "write_bytes": wb}
            lines.append(f"| `{short}` | {calls} | {ms:.4f} | {fb / 2**30:.3f} | {wb / 2**30:.3f} | "
                         f"{(fb + wb) / (ms * 1e-3) / 1e12:.2f} |")
        elif ffac is not None:
            lines.append(f"| `{short}` | {calls} | {ms:.4f} | | | |")
        else:
            lines.append(f"| `{short}` | {calls} | {ms:.4f} | {calls * ms:.2f} |")
    if notes:
        lines += ["", notes.strip()]
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, name + ".md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if kernels:
        with open(os.path.join(out_dir, name + "_traffic.json"), "w") as fh:
            json.dump({"src_hash": src_hash(prefix), "kernels": kernels}, fh, indent=1)
    return kernels


def counter_table(name, trace, runs, kernels, cmds, out_dir, prefix="pcx_", notes="", simds=1024, ghz=2.4):
    """Instruction and wait counters per dispatch of the given kernels (name
    substrings) from --pmc runs of SQ counters, with the VALU busy fraction
    they imply: SQ_INSTS_VALU x 4 cycles (a wave64 VALU instruction holds its
    SIMD for 4 cycles) over the SIMD cycles of the kernel's average duration
    from the kernel-trace run (1024 SIMDs at 2.4 GHz)."""
    ks = kernel_stats(trace)
    vals = {}
    for d in runs:
        names = {r["Counter_Name"] for r in _csv(d, "counter_collection.csv")}
        for c in sorted(names):
            for k, v in counter_means(d, c).items():
                vals.setdefault(k, {})[c] = v
    lines = [f"# rocprofv3 counters: {name}", "", "Commands (from the repository root, on one MI355X):", "", "```"]
    lines += list(cmds) + ["```", ""]
    lines.append(f"Kernel sources hash (sha256 of csrc/{prefix}*, first 16 hex): `{src_hash(prefix)}`")
    lines.append("")
    lines.append("| Kernel | avg ms | waves | VALU / wave | VMEM rd / wave | LDS / wave | "
                 "VALU busy | wait / wave cycles |")
    lines.append("|---|---|---|---|---|---|---|---|")
    out = {}
    for part in kernels:
        hits = [k for k in vals if part in k]
        if not hits:
            continue
        k = hits[0]
        v = vals[k]
        ms = next((m for kn, (_, m) in ks.items() if part in kn), None)
        waves = v.get("SQ_WAVES", 0.0)
        per = lambda c: v[c] / waves if waves and c in v else float("nan")
        busy = v["SQ_INSTS_VALU"] * 4 / (simds * ghz * 1e9 * ms * 1e-3) if ms and "SQ_INSTS_VALU" in v else float("nan")
        wait = v["SQ_WAIT_INST_ANY"] / v["SQ_WAVE_CYCLES"] if v.get("SQ_WAVE_CYCLES") else float("nan")
        out[k] = {"ms": ms, "counters": v, "valu_busy": busy, "wait_frac": wait}
        short = k if len(k) <= 70 else k[:67] + "..."
        lines.append(f"| `{short}` | {ms:.4f} | {waves:.0f} | {per('SQ_INSTS_VALU'):.0f} | "
                     f"{per('SQ_INSTS_VMEM_RD'):.1f} | {per('SQ_INSTS_LDS'):.1f} | {busy:.2f} | {wait:.2f} |")
    if notes:
        lines += ["", notes.strip()]
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, name + ".md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--name", required=True)
    ap.add_argument("--trace", required=True, help="directory of the --kernel-trace --stats run")
    ap.add_argument("--fetch", help="directory of the --pmc FETCH_SIZE run")
    ap.add_argument("--write", help="directory of the --pmc WRITE_SIZE run")
    ap.add_argument("--field-bytes", type=float, default=float(1 << 30))
    ap.add_argument("--cmd", action="append", default=[])
    ap.add_argument("--prefix", default="pcx_")
    ap.add_argument("--notes", default="")
    ap.add_argument("--top", type=int, default=12)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(HERE), "profiles"))
    ap.add_argument("--counters", action="append", default=[],
                    help="directory of a --pmc run of SQ counters (repeatable); with --kernel, "
                         "writes the counter table instead of the byte summary")
    ap.add_argument("--kernel", action="append", default=[], help="kernel name substring for --counters")
    a = ap.parse_args(argv)
    if a.counters:
        counter_table(a.name, a.trace, a.counters, a.kernel, a.cmd, a.out, a.prefix, a.notes)
        return 0
    summarize(a.name, a.trace, a.fetch, a.write, a.field_bytes, a.cmd, a.out, a.prefix, a.notes, a.top)
    return 0


if __name__ == "__main__":
    sys.exit(main())
