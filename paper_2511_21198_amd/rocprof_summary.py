"""Summarise rocprofv3 output of a solver run per kernel kind.

    python -m paper_2511_21198_amd.rocprof_summary --trace DIR [--fetch DIR]
        [--write DIR] [--sq DIR] [--mfma DIR] --np NP [--json OUT.json]
        [--md OUT.md] [--cmd "..."]

DIR is a rocprofv3 ``-d`` directory written with ``-f csv``: ``--trace`` one
of ``--kernel-trace --stats``, ``--fetch`` / ``--write`` one of
``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` (KiB per dispatch).

Kernel dispatches are mapped to the kinds the library's own hipEvent
profiler reports (toep_x_f32, dst_y_f64, gm_maxpy_f32, ...).  The strided
Toeplitz kernel serves the y and the z pass of a matvec; a dispatch is the
y pass when the previous Toeplitz dispatch was an x pass.  Dispatches that
returned at once because the solve had already stopped (Krylov iterations
are enqueued ahead of the convergence test) are left out: in the trace
those shorter than ``--skip-us`` microseconds, in the counter runs those
that fetched less than 1 MiB.

HBM bytes: FETCH_SIZE and WRITE_SIZE are scaled by the factors that make
the float64 -> float32 cast kernel (k_cast, NP elements: reads 8 NP bytes,
writes 4 NP bytes) read and write exactly its own size.  NP is the padded
vector length of the run (n3 * n2 * round_up(n1, 32)).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))


# Device sources behind each kernel kind (the structures they read included).
_LINE_SRC = ["fsd_internal.h", "fsd_lines.hpp", "fsd_wave.hpp", "fsd_cols.hpp", "fsd_passes.hpp",
             "fsd_lines_f32.hip", "fsd_lines_f64.hip"]
_SOURCES = {"toep": _LINE_SRC, "dst": _LINE_SRC, "dsts": _LINE_SRC,
            "gm": ["fsd_internal.h", "fsd_gmres.h", "fsd_gmres.hip"],
            "pcg": ["fsd_internal.h", "fsd_vec.h", "fsd_vec.hip"],
            "cast": ["fsd_internal.h", "fsd_vec.h", "fsd_vec.hip"],
            "resid": ["fsd_internal.h", "fsd_vec.h", "fsd_vec.hip"],
            "circ": ["fsd_internal.h", "fsd_circ.h", "fsd_circ.hip"],
            "gdst": ["fsd_internal.h", "fsd_gdst.hip"], "gdsts": ["fsd_internal.h", "fsd_gdst.hip"]}


def source_hash(kind: str | None = None) -> str:
    """Hash of the device sources of a kernel kind (all device sources when
    kind is None), to detect counters taken on other kernels."""
    if kind is None:
        names = sorted({n for v in _SOURCES.values() for n in v})
    else:
        names = _SOURCES[kind.split("_")[0]]
    h = hashlib.sha256()
    for n in names:
        h.update(n.encode())
        with open(os.path.join(HERE, "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


_KINDS = [
    (re.compile(r"k_col_toep\b"), "toep_s"),
    (re.compile(r"k_col_dsth?\s*<\s*true"), "dsts"),
    (re.compile(r"k_col_dsth?\b"), "dst_y"),
    (re.compile(r"k2?_toep_x\b"), "toep_x"),
    (re.compile(r"k2?_toep_s\b"), "toep_s"),
    (re.compile(r"k2?_dst_x\b"), "dst_x"),
    (re.compile(r"k_dstsh?_s\b"), "dsts"),
    (re.compile(r"k2_dst_s\s*<\s*\w+\s*,\s*\d+\s*,\s*(true|1)\b"), "dsts"),
    (re.compile(r"k2?_dst_s\b"), "dst_y"),
    (re.compile(r"k_mdot\b"), "gm_mdot"),
    (re.compile(r"k_maxpy\b"), "gm_maxpy"),
    (re.compile(r"k_gm_update\b"), "gm_update"),
    (re.compile(r"k_update_xr\b"), "pcg_update"),
    (re.compile(r"k_cast\b"), "cast"),
    (re.compile(r"k_resid_prev\b"), "resid_prev_f64"),
    (re.compile(r"k_circ\b"), "circ_f64"),
    (re.compile(r"k_gdst_row\b"), "gdst_x"),
    (re.compile(r"k_gdst_col\b"), "gdst_col"),
]


def _dtype(name: str) -> str:
    m = re.search(r"<\s*(float|double)", name)
    if not m:
        return ""
    return "f32" if m.group(1) == "float" else "f64"


def classify(rows, dim=3):
    """rows: dispatches in submission order with 'Kernel_Name'.  Returns the
    kind of each (None for kernels outside the table)."""
    out = []
    last_toep = None
    cols = 0   # matrix-core DST column passes since the last row pass: y, last axis, y
    for r in rows:
        name = r["Kernel_Name"]
        kind = None
        for rx, k in _KINDS:
            if rx.search(name):
                kind = k
                break
        if kind is None:
            out.append(None)
            continue
        if kind == "toep_s":
            kind = "toep_y" if (last_toep == "toep_x" or dim == 2) else "toep_z"
        if kind == "dsts":
            kind = "dsts_z" if dim == 3 else "dsts_y"
        if kind.startswith("toep"):
            last_toep = kind
        if kind == "gdst_x":
            cols = 0
        elif kind == "gdst_col":
            cols += 1
            kind = ("gdsts_z" if dim == 3 else "gdsts_y") if (cols == 2 or dim == 2) else "gdst_y"
        dt = _dtype(name)
        if kind.startswith("gdst"):
            dt = "f32"
        out.append(f"{kind}_{dt}" if dt and kind not in ("cast", "resid_prev_f64", "circ_f64") else kind)
    return out


def _read(path_dir, pattern):
    files = glob.glob(os.path.join(path_dir, "**", pattern), recursive=True)
    if not files:
        raise FileNotFoundError(f"no {pattern} under {path_dir}")
    rows = list(csv.DictReader(open(files[0])))
    key = "Dispatch_Id" if "Dispatch_Id" in rows[0] else "Correlation_Id"
    rows.sort(key=lambda r: int(r[key]))
    return rows


def summarise(trace_dir, fetch_dir=None, write_dir=None, np_len=None, skip_us=8.0, dim=3,
              scale_from=None):
    tr = _read(trace_dir, "*kernel_trace.csv")
    kinds = classify(tr, dim)
    dur = collections.defaultdict(list)
    skipped = collections.Counter()
    for r, k in zip(tr, kinds):
        if k is None:
            continue
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        if us < skip_us:
            skipped[k] += 1
        else:
            dur[k].append(us)
    res = {k: {"dispatches": len(v), "skipped": skipped[k], "avg_us": sum(v) / len(v),
               "total_ms": sum(v) / 1e3} for k, v in dur.items()}
    factors = {}
    for label, d, cname in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        if not d:
            continue
        rows = [r for r in _read(d, "*counter_collection.csv") if r["Counter_Name"] == cname]
        ks = classify(rows, dim)
        per = collections.defaultdict(list)
        for r, k in zip(rows, ks):
            v = float(r["Counter_Value"]) * 1024.0
            if k is None or (k != "cast" and label == "fetch" and v < 1 << 20):
                continue
            per[k].append(v)
        if "cast" in per and np_len:
            expect = (8.0 if label == "fetch" else 4.0) * np_len
            factors[label] = expect / (sum(per["cast"]) / len(per["cast"]))
        elif scale_from and label in scale_from:
            factors[label] = scale_from[label]
        f = factors.get(label, 1.0)
        for k, v in per.items():
            if k in res:
                res[k][f"{label}_bytes_per_dispatch"] = f * sum(v) / len(v)
    for k, e in res.items():
        e["source_hash"] = source_hash(k)
        if "fetch_bytes_per_dispatch" in e and "write_bytes_per_dispatch" in e:
            e["hbm_bytes_per_dispatch"] = e["fetch_bytes_per_dispatch"] + e["write_bytes_per_dispatch"]
            e["hbm_gbps"] = e["hbm_bytes_per_dispatch"] / (e["avg_us"] * 1e-6) / 1e9
    return res, factors


MFMA_COUNTERS = ("SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_BUSY_CYCLES",
                 "GRBM_GUI_ACTIVE")


def mfma_summary(mfma_dir, res, dim=3):
    """Per kind: the MFMA counters per dispatch (averaged over the
    dispatches that issued matrix-core work; the ones enqueued after the
    solve had stopped return at once) and the bf16 TFLOP/s they imply (a
    MOPS unit is 512 flops) over the kind's average traced duration."""
    rows = _read(mfma_dir, "*counter_collection.csv")
    key = "Dispatch_Id" if "Dispatch_Id" in rows[0] else "Correlation_Id"
    by_id = collections.OrderedDict()
    for r in rows:
        if r["Counter_Name"] in MFMA_COUNTERS:
            d = by_id.setdefault(r[key], {"Kernel_Name": r["Kernel_Name"]})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
    disp = list(by_id.values())
    per = collections.defaultdict(list)
    for d, k in zip(disp, classify(disp, dim)):
        if k is not None and d.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) > 0:
            per[k].append(d)
    out = {}
    for k, ds in per.items():
        e = {c: sum(d.get(c, 0.0) for d in ds) / len(ds) for c in MFMA_COUNTERS}
        e["dispatches"] = len(ds)
        if k in res:
            e["bf16_tflops"] = e["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512.0 / (res[k]["avg_us"] * 1e-6) / 1e12
        out[k] = e
    return out


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_ACTIVE_INST_VALU",
               "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES",
               "GRBM_GUI_ACTIVE")
SIMDS = 1024   # 256 compute units x 4 SIMDs
CUS = 256
XCDS = 8       # GRBM_GUI_ACTIVE is summed over the accelerator dies


def sq_summary(sq_dir, dim=3):
    """Per kind: the shader counters per dispatch, averaged over the
    dispatches that did their work (those enqueued after the solve had
    stopped return at once: below a quarter of the kind's largest VALU
    instruction count), and the fractions derived from them:

      valu_busy  = 4 SQ_ACTIVE_INST_VALU / (SIMDS C)
      lds_busy   = 4 SQ_ACTIVE_INST_LDS  / (SIMDS C)
      bank_conflict = SQ_LDS_BANK_CONFLICT / (CUS C)

    with C = GRBM_GUI_ACTIVE / XCDS the dispatch's busy cycles (the GRBM
    counter is summed over the 8 dies: it reads about 8 x clock x duration)
    and the ACTIVE_INST counters in quad-cycles summed over all SIMDs; and
    VALU / LDS instructions per wavefront."""
    rows = _read(sq_dir, "*counter_collection.csv")
    key = "Dispatch_Id" if "Dispatch_Id" in rows[0] else "Correlation_Id"
    by_id = collections.OrderedDict()
    for r in rows:
        if r["Counter_Name"] in SQ_COUNTERS:
            d = by_id.setdefault(r[key], {"Kernel_Name": r["Kernel_Name"]})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    disp = list(by_id.values())
    per = collections.defaultdict(list)
    for d, k in zip(disp, classify(disp, dim)):
        if k is not None:
            per[k].append(d)
    out = {}
    for k, ds in per.items():
        top = max(d.get("SQ_INSTS_VALU", 0.0) for d in ds)
        ds = [d for d in ds if d.get("SQ_INSTS_VALU", 0.0) >= 0.25 * top]
        if not ds:
            continue
        e = {c: sum(d.get(c, 0.0) for d in ds) / len(ds) for c in SQ_COUNTERS}
        e["dispatches"] = len(ds)
        g = e["GRBM_GUI_ACTIVE"] / XCDS
        w = e["SQ_WAVES"]
        if g > 0:
            e["valu_busy"] = 4.0 * e["SQ_ACTIVE_INST_VALU"] / (SIMDS * g)
            e["lds_busy"] = 4.0 * e["SQ_ACTIVE_INST_LDS"] / (SIMDS * g)
            e["bank_conflict"] = e["SQ_LDS_BANK_CONFLICT"] / (CUS * g)
        if w > 0:
            e["valu_per_wave"] = e["SQ_INSTS_VALU"] / w
            e["lds_per_wave"] = e["SQ_INSTS_LDS"] / w
        out[k] = e
    return out


def _stats_table(trace_dir: str, top: int):
    """Markdown rows of the rocprofv3 --stats kernel summary in trace_dir."""
    paths = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not paths:
        return []
    with open(paths[0]) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | total ms | avg us | min us | max us | % |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["Name"]
        if len(name) > 110:
            name = name[:110]
        out.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--np", type=int, help="padded vector length of the run")
    ap.add_argument("--dim", type=int, default=3)
    ap.add_argument("--skip-us", type=float, default=8.0)
    ap.add_argument("--json")
    ap.add_argument("--md")
    ap.add_argument("--cmd", default="", help="the profiled command, recorded in the outputs")
    ap.add_argument("--title", default="")
    ap.add_argument("--mfma", help="rocprofv3 -d directory of a --pmc run of " + " ".join(MFMA_COUNTERS))
    ap.add_argument("--sq", help="rocprofv3 -d directory of a --pmc run of " + " ".join(SQ_COUNTERS))
    ap.add_argument("--scale-from", help="summary JSON whose k_cast counter scale factors to use "
                                         "when this run launched no k_cast")
    a = ap.parse_args(argv)
    scale_from = None
    if a.scale_from:
        with open(a.scale_from) as f:
            scale_from = json.load(f).get("counter_scale")
    res, factors = summarise(a.trace, a.fetch, a.write, a.np, a.skip_us, a.dim, scale_from)
    doc = {"command": a.cmd, "source_hash": source_hash(), "np": a.np,
           "counter_scale": factors, "kinds": res}
    mf = mfma_summary(a.mfma, res, a.dim) if a.mfma else None
    if mf:
        doc["mfma"] = mf
    sq = sq_summary(a.sq, a.dim) if a.sq else None
    if sq:
        doc["sq"] = sq
    if a.json:
        with open(a.json, "w") as f:
            json.dump(doc, f, indent=1, sort_keys=True)
    lines = []
    if a.title:
        lines += [f"# {a.title}", ""]
    lines += ["Command:", "", "```", a.cmd, "```", "",
              f"Library source hash: `{doc['source_hash']}`.  Counter scale factors "
              + (f"(k_cast calibration, {a.np} elements): " if not scale_from else
                 f"(k_cast calibration taken from `{a.scale_from}`): ")
              + ", ".join(f"{k} x{v:.4f}" for k, v in factors.items()), "",
              f"Dispatches shorter than {a.skip_us:g} us (enqueued after the solve had "
              "stopped; they return at once) are listed as skipped and excluded.", "",
              "| kind | dispatches | skipped | avg us | total ms | HBM MB/dispatch | HBM GB/s |",
              "|---|---:|---:|---:|---:|---:|---:|"]
    for k, e in sorted(res.items(), key=lambda kv: -kv[1]["total_ms"]):
        hb = e.get("hbm_bytes_per_dispatch")
        lines.append(f"| {k} | {e['dispatches']} | {e['skipped']} | {e['avg_us']:.2f} | "
                     f"{e['total_ms']:.3f} | {hb / 1e6:.2f} | {e['hbm_gbps']:.0f} |" if hb else
                     f"| {k} | {e['dispatches']} | {e['skipped']} | {e['avg_us']:.2f} | "
                     f"{e['total_ms']:.3f} | - | - |")
    if mf:
        lines += ["", "Matrix-core counters (per dispatch, averaged; bf16 TFLOP/s = 512 x "
                  "SQ_INSTS_VALU_MFMA_MOPS_BF16 / average duration, dense bf16 peak 2500):", "",
                  "| kind | MFMA MOPS (bf16) | GFLOP | MFMA busy cycles | SQ busy cycles | GRBM active | bf16 TFLOP/s |",
                  "|---|---:|---:|---:|---:|---:|---:|"]
        for k, e in sorted(mf.items()):
            m = e.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0)
            if not m:
                continue
            lines.append(f"| {k} | {m:.4g} | {m * 512 / 1e9:.2f} | {e.get('SQ_VALU_MFMA_BUSY_CYCLES', 0):.4g} | "
                         f"{e.get('SQ_BUSY_CYCLES', 0):.4g} | {e.get('GRBM_GUI_ACTIVE', 0):.4g} | "
                         f"{e.get('bf16_tflops', 0):.1f} |")
    if sq:
        lines += ["", "Shader counters (per dispatch, averaged over the dispatches that did their "
                  "work): VALU busy = 4 SQ_ACTIVE_INST_VALU / (1024 SIMDs x C), LDS busy likewise "
                  "from SQ_ACTIVE_INST_LDS, bank conflict = SQ_LDS_BANK_CONFLICT / (256 CUs x C), "
                  "with C = GRBM_GUI_ACTIVE / 8 (the GRBM counter sums the 8 dies):", "",
                  "| kind | waves | VALU instr/wave | LDS instr/wave | VALU busy | LDS busy | bank conflict | GRBM active |",
                  "|---|---:|---:|---:|---:|---:|---:|---:|"]
        order = sorted(sq, key=lambda k: -res.get(k, {}).get("total_ms", 0.0))
        for k in order:
            e = sq[k]
            lines.append(f"| {k} | {e['SQ_WAVES']:.0f} | {e.get('valu_per_wave', 0):.0f} | "
                         f"{e.get('lds_per_wave', 0):.0f} | {e.get('valu_busy', 0):.2f} | "
                         f"{e.get('lds_busy', 0):.2f} | {e.get('bank_conflict', 0):.3f} | "
                         f"{e['GRBM_GUI_ACTIVE']:.4g} |")
    stats = _stats_table(a.trace, 25)
    if stats:
        lines += ["", "rocprofv3 `--stats` kernel summary of the same run (`*_kernel_stats.csv`, "
                  "top 25 by total time; averages include the skipped dispatches):", ""] + stats
    text = "\n".join(lines) + "\n"
    if a.md:
        with open(a.md, "w") as f:
            f.write(text)
    print(text)


if __name__ == "__main__":
    main()
