"""Turn rocprofv3 output of the benchmark into the short summaries kept with
the library: a per-kernel table (launches, durations, counter bytes) in
Markdown, and the measured bytes per launch beyond the L2 that the benchmark
reports beside its roofline.

Inputs are rocprofv3 runs of the same benchmark command:
  --kernel-trace --stats --output-format csv      (durations)
  --pmc FETCH_SIZE --output-format csv            (KiB read per dispatch)
  --pmc WRITE_SIZE --output-format csv            (KiB written per dispatch)
  --pmc SQ_INSTS_VALU SQ_INSTS_SALU ... (optional: instruction counts, summed
    over the device's shader engines)
  --pmc TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum ... (optional: read requests by
    size)
The benchmark runs an untimed device copy of a known size (the run's largest
copy); its counter readings give the factor that turns each counter into bytes (on gfx950
FETCH_SIZE reads half the bytes a streaming copy moves; WRITE_SIZE reads them
all).  Counter bytes are what the L2 exchanged with the memory side (HBM, or
the last-level cache in front of it).

    python -m paper_2112_13169_amd.prof_summary --kt DIR --fetch DIR --write DIR \\
        --workload plain-medium --cal-bytes 67108864 --command "..." \\
        --md profiles/NAME.md --json profiles/traffic.json
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
KERNEL_SOURCES = ["csrc/vg_kernels.hip", "csrc/vg_walk.h", "csrc/vg_internal.h",
                  "csrc/vg_frustum.h"]


def code_only(text):
    """C/C++ source without its comments and blank space (a comment edit does
    not change a kernel)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(read=None):
    """Hash of the kernel sources' code: counter readings taken on other code
    are stale.  `read(rel)` may supply a file's text (default: this tree)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        if read is None:
            with open(os.path.join(HERE, rel)) as fh:
                text = fh.read()
        else:
            text = read(rel)
        h.update(code_only(text).encode())
    return h.hexdigest()[:16]


def short_name(name):
    name = name.replace("vg::(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0]


def _one(pattern):
    hits = sorted(glob.glob(pattern))
    if not hits:
        raise SystemExit(f"no file matches {pattern}")
    return hits[0]


def read_stats(kt_dir):
    out = {}
    with open(_one(os.path.join(kt_dir, "*kernel_stats.csv"))) as fh:
        for r in csv.DictReader(fh):
            out[short_name(r["Name"])] = dict(calls=int(r["Calls"]), avg_ns=float(r["AverageNs"]),
                                              min_ns=float(r["MinNs"]), max_ns=float(r["MaxNs"]),
                                              pct=float(r["Percentage"]))
    return out


# MI355X HBM3E peak, GB/s (vendor figure)
HBM_PEAK_GBS = 8000.0
# MI355X: 256 CUs x 4 SIMDs; a wave64 VALU instruction occupies a 16-lane
# SIMD for 4 cycles; 2.4 GHz
SIMDS = 1024
VALU_CYCLES = 4
CLOCK_GHZ = 2.4
SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD",
               "SQ_INSTS_VMEM_WR", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES")


def read_sq(pmc_dir):
    """Per-kernel mean of each SQ counter over its dispatches."""
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    with open(_one(os.path.join(pmc_dir, "*counter_collection.csv"))) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] in SQ_COUNTERS:
                vals[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(
                    float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} | {"dispatches": len(next(iter(
        d.values())))} for k, d in vals.items()}


RDREQ_COUNTERS = ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum",
                  "TCC_EA0_RDREQ_128B_sum")


def read_rdreq(pmc_dir):
    """Per-kernel mean of the L2's read requests to the memory side by size,
    over its dispatches."""
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    with open(_one(os.path.join(pmc_dir, "*counter_collection.csv"))) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] in RDREQ_COUNTERS:
                vals[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(
                    float(r["Counter_Value"]))
    return {k: {c[len("TCC_EA0_"):-len("_sum")]: sum(v) / len(v) for c, v in d.items()}
            for k, d in vals.items()}


def read_counter(pmc_dir, counter):
    """Per-kernel list of (grid size, KiB) of each dispatch, in dispatch order."""
    rows = []
    with open(_one(os.path.join(pmc_dir, "*counter_collection.csv"))) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                rows.append((int(r["Dispatch_Id"]), short_name(r["Kernel_Name"]),
                             int(r["Grid_Size"]), float(r["Counter_Value"])))
    rows.sort()
    per = collections.defaultdict(list)
    for _, k, grid, kib in rows:
        per[k].append((grid, kib))
    return per, rows


def calibration(rows, cal_bytes):
    """Counter KiB of the calibration copy: the largest plain copy kernel
    dispatch of the run (the benchmark's copy is many times larger than its
    frame uploads and grid reads)."""
    copies = [r for r in rows if "copyBuffer" in r[1] and "Rect" not in r[1]]
    if not copies:
        raise SystemExit("no calibration copy in the counter run")
    kib = max(r[3] for r in copies)
    return (cal_bytes / 1024.0) / kib, kib


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--kt", required=True)
    ap.add_argument("--fetch", help="FETCH_SIZE run (optional: no counter columns)")
    ap.add_argument("--write", help="WRITE_SIZE run")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--cal-bytes", type=int, required=True)
    ap.add_argument("--command", required=True, help="the profiled command, for the record")
    ap.add_argument("--md", required=True)
    ap.add_argument("--json", help="traffic summary to write (needs both counter runs)")
    ap.add_argument("--sq", help="SQ counter run (optional: instruction table)")
    ap.add_argument("--rdreq", help="run of the read request counters by size (optional)")
    ap.add_argument("--walk-kernel", help="kernel whose VALU per walk step is reported")
    ap.add_argument("--walk-steps", type=float,
                    help="in-grid walk steps per launch of --walk-kernel (from the benchmark)")
    a = ap.parse_args(argv)

    stats = read_stats(a.kt)
    counters = bool(a.fetch and a.write)
    fetch, write = {}, {}
    f_fac = w_fac = f_cal = w_cal = None
    if counters:
        fetch, frows = read_counter(a.fetch, "FETCH_SIZE")
        write, wrows = read_counter(a.write, "WRITE_SIZE")
        f_fac, f_cal = calibration(frows, a.cal_bytes)
        w_fac, w_cal = calibration(wrows, a.cal_bytes)

    kernels = {}
    lines = [f"# Kernel durations and memory-side bytes: {a.workload}", "",
             "Commands (one MI355X; REPO is the repository root):", "", "```"]
    lines += a.command.strip().splitlines()
    lines += ["```", ""]
    if counters:
        lines += [f"Calibration: a {a.cal_bytes} B device copy read FETCH_SIZE {f_cal:.1f} KiB "
                  f"and WRITE_SIZE {w_cal:.1f} KiB, so bytes = FETCH_SIZE x {f_fac:.4f} KiB + "
                  f"WRITE_SIZE x {w_fac:.4f} KiB.", ""]
    lines += [f"Kernel sources hash (code without comments): `{kernel_source_hash()}`", "",
              "| kernel | launches | avg us | min us | max us | % time | FETCH KiB | WRITE KiB "
              "| bytes/launch (calibrated) | GB/s | of HBM peak |",
              "|---|---|---|---|---|---|---|---|---|---|---|"]
    for k, s in sorted(stats.items(), key=lambda kv: -kv[1]["pct"]):
        fk = [v for _, v in fetch.get(k, [])]
        wk = [v for _, v in write.get(k, [])]
        fr = sum(fk) / len(fk) if fk else None
        wr = sum(wk) / len(wk) if wk else None
        nbytes = gbs = None
        if fr is not None and wr is not None:
            nbytes = 1024.0 * (fr * f_fac + wr * w_fac)
            gbs = nbytes / s["avg_ns"]          # bytes per ns = GB/s
            if k.startswith(("k_", "kb_")):
                kernels[k] = dict(hbm_bytes_per_launch=round(nbytes), launches=s["calls"],
                                  fetch_kib=round(fr, 1),
                                  write_kib=round(wr, 1), avg_us=round(s["avg_ns"] / 1e3, 3),
                                  gb_per_s=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
        lines.append(f"| `{k}` | {s['calls']} | {s['avg_ns'] / 1e3:.2f} | {s['min_ns'] / 1e3:.2f} | "
                     f"{s['max_ns'] / 1e3:.2f} | {s['pct']:.1f} | "
                     f"{'-' if fr is None else f'{fr:.1f}'} | {'-' if wr is None else f'{wr:.1f}'} | "
                     f"{'-' if nbytes is None else f'{nbytes / 1e6:.3f} MB'} | "
                     f"{'-' if gbs is None else f'{gbs:.0f}'} | "
                     f"{'-' if gbs is None else f'{gbs / HBM_PEAK_GBS:.3f}'} |")
    lines.append("")
    sq_rows = {}
    if a.sq:
        sq = read_sq(a.sq)
        lines += ["Instruction counters (one `rocprofv3 --pmc` pass of SQ counters; values are summed "
                  "over the device's shader engines and averaged over a kernel's dispatches). "
                  "`VALU busy` is SQ_INSTS_VALU x 4 cycles over the SIMD cycles of the "
                  "kernel's trace average (1 024 SIMDs x 2.4 GHz): the share of the chip's VALU "
                  "issue slots the kernel used.", "",
                  "| kernel | waves | VALU / wave | SALU / wave | VMEM rd / wave | VMEM wr / wave "
                  "| VALU busy |", "|---|---|---|---|---|---|---|"]
        for k, s in sorted(stats.items(), key=lambda kv: -kv[1]["pct"]):
            q = sq.get(k)
            if not q or not k.startswith(("k_", "kb_")) or not q.get("SQ_WAVES"):
                continue
            w = q["SQ_WAVES"]
            busy = q["SQ_INSTS_VALU"] * VALU_CYCLES / (SIMDS * s["avg_ns"] * CLOCK_GHZ)
            sq_rows[k] = dict(waves=round(w), valu_per_wave=round(q["SQ_INSTS_VALU"] / w, 1),
                              salu_per_wave=round(q["SQ_INSTS_SALU"] / w, 1),
                              valu_busy=round(busy, 3), valu_insts=q["SQ_INSTS_VALU"])
            lines.append(f"| `{k}` | {w:.0f} | {q['SQ_INSTS_VALU'] / w:.1f} | "
                         f"{q['SQ_INSTS_SALU'] / w:.1f} | {q['SQ_INSTS_VMEM_RD'] / w:.1f} | "
                         f"{q['SQ_INSTS_VMEM_WR'] / w:.1f} | {busy:.3f} |")
        lines.append("")
        if a.walk_kernel and a.walk_steps and a.walk_kernel in sq:
            q = sq[a.walk_kernel]
            per = 64.0 * q["SQ_INSTS_VALU"] / a.walk_steps
            lines += [f"`{a.walk_kernel}`: {q['SQ_INSTS_VALU']:.4g} VALU wave-instructions per "
                      f"launch for {a.walk_steps:.4g} in-grid walk steps, i.e. {per:.1f} VALU "
                      f"lane-slots per step (64 per wave-instruction, idle lanes of partly "
                      f"finished wavefronts included), against the 20 algorithmic operations "
                      f"of a step.", ""]
    rd_rows = {}
    if a.rdreq:
        rq = read_rdreq(a.rdreq)
        lines += ["Read requests by size (one `rocprofv3 --pmc` pass of TCC_EA0_RDREQ, "
                  "TCC_EA0_RDREQ_32B, _64B and _128B, summed over the L2 channels, mean per "
                  "dispatch): the share of 128-byte requests tells whether a kernel's scattered "
                  "loads fetch the same 128-byte lines as the streaming copy the FETCH_SIZE "
                  "factor comes from.", "",
                  "| kernel | read requests | 32 B | 64 B | 128 B | share 128 B | bytes requested |",
                  "|---|---|---|---|---|---|---|"]
        for k, s in sorted(stats.items(), key=lambda kv: -kv[1]["pct"]):
            q = rq.get(k)
            if not q or not q.get("RDREQ"):
                continue
            n32, n64, n128 = q.get("RDREQ_32B", 0.0), q.get("RDREQ_64B", 0.0), q.get("RDREQ_128B", 0.0)
            nbytes = 32 * n32 + 64 * n64 + 128 * n128
            share = n128 / q["RDREQ"]
            if k.startswith(("k_", "kb_")):
                rd_rows[k] = dict(requests=round(q["RDREQ"]), share_128b=round(share, 4),
                                  bytes_requested=round(nbytes))
            lines.append(f"| `{k}` | {q['RDREQ']:.0f} | {n32:.0f} | {n64:.0f} | {n128:.0f} | "
                         f"{share:.3f} | {nbytes / 1e6:.3f} MB |")
        lines.append("")
    with open(a.md, "w") as fh:
        fh.write("\n".join(lines))
    if counters and a.json:
        with open(a.json, "w") as fh:
            json.dump(dict(workload=a.workload, source_hash=kernel_source_hash(),
                           hbm_peak_gbs=HBM_PEAK_GBS,
                           fetch_factor=round(f_fac, 4), write_factor=round(w_fac, 4),
                           kernels=kernels, sq=sq_rows or None, read_requests=rd_rows or None),
                      fh, indent=1)
            fh.write("\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
