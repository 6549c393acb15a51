"""Summarise rocprofv3 CSV output into the short text files kept in profiles/.

    python -m paper_1204_0111_amd.profile_summary stats <kernel_stats.csv> <out.txt> "<command>" \
        [<kernel_trace.csv>]
    python -m paper_1204_0111_amd.profile_summary pmc <fetch_counter_collection.csv> \
        <write_counter_collection.csv> <kernel symbol> <workload> <out.txt> "<fetch command>" \
        "<write command>"
    python -m paper_1204_0111_amd.profile_summary sq <counter_collection.csv> <workload> <out.txt> \
        "<command>"

The PMC summary scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by the
factor the same counter reads for the plain 512 MiB device copy the benchmark
runs with --calibrate-copy-mb 512, and records the hash of the kernel's
source so that a changed kernel makes the numbers stale.
"""

import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = {"k_fwd": "solve.hip", "k_bwd": "solve.hip", "k_fwd_mm": "solve.hip", "k_bwd_mm": "solve.hip",
       "k_rhs_scatter": "solve.hip", "k_trailing": "factor.hip",
       "k_update": "factor.hip", "k_inverse": "factor.hip", "k_panel_trsm": "factor.hip", "k_ldlt_diag": "factor.hip",
       "k_assemble": "factor.hip", "k_matvec": "krylov.hip"}
COPY_BYTES = 512 * (1 << 20)


def src_hash(sym):
    p = os.path.join(ROOT, "paper_1204_0111_amd", "csrc", SRC[sym])
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


FAMILIES = ("hsw::k_fwd", "hsw::k_bwd", "hsw::k_fwd_mm", "hsw::k_bwd_mm", "hsw::k_rhs_scatter",
            "hsw::k_update", "hsw::k_inverse", "hsw::k_ldlt_diag", "hsw::k_panel_trsm", "hsw::k_assemble",
            "hsw::k_matvec")


def last_step_families(trace_path):
    """Per kernel (all template instances together) over the last step of a
    kernel trace: the dispatches from the last velocity check on, which is
    the step a benchmark times after its warm-up (and autotuning)."""
    rows = sorted(csv.DictReader(open(trace_path)), key=lambda r: int(r["Start_Timestamp"]))
    last = max(i for i, r in enumerate(rows) if "k_check_velocity" in r["Kernel_Name"])
    fam = {}
    for r in rows[last:]:
        k = r["Kernel_Name"].split("(")[0].replace("void ", "").split("<")[0]
        c, t = fam.get(k, (0, 0.0))
        fam[k] = (c + 1, t + int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return fam


def stats(csv_path, out, cmd, trace_path=None):
    rows = list(csv.DictReader(open(csv_path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    with open(out, "w") as f:
        f.write("# rocprofv3 --kernel-trace --stats summary\n# command: %s\n" % cmd)
        f.write("# total kernel time %.3f ms over %d kernel names\n" % (tot / 1e6, len(rows)))
        f.write("%-34s %7s %11s %10s %6s\n" % ("kernel", "calls", "total_ms", "avg_us", "pct"))
        for r in rows[:20]:
            name = r["Name"].split("(")[0].replace("void ", "")[:34]
            f.write("%-34s %7s %11.3f %10.3f %6.2f\n" % (name, r["Calls"],
                    float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
                    float(r["Percentage"])))
        # one line per kernel over all its template instances (block shapes);
        # these include the autotuner's trial launches of the warm-up step
        f.write("# per kernel, all block shapes together\n")
        fam = {}
        for r in rows:
            k = r["Name"].split("(")[0].replace("void ", "").split("<")[0]
            c, t = fam.get(k, (0, 0.0))
            fam[k] = (c + int(r["Calls"]), t + float(r["TotalDurationNs"]))
        for k in FAMILIES:
            if k in fam:
                c, t = fam[k]
                f.write("%-34s %7d %11.3f %10.3f\n" % (k, c, t / 1e6, t / c / 1e3))
        if trace_path:
            # the step the benchmark times: no warm-up, no autotuner trials
            f.write("# last step only (kernel trace), all block shapes together\n")
            last = last_step_families(trace_path)
            for k in FAMILIES:
                if k in last:
                    c, t = last[k]
                    f.write("%-34s %7d %11.3f %10.3f\n" % (k, c, t / 1e6, t / c / 1e3))


def per_kernel(path):
    """Counter values per kernel name over the last step of the run (the
    dispatches after the last velocity check, which opens a step), and the
    value read for the calibration copy (the first large device copy)."""
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))
    calib = None
    for r in rows:
        if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer") and int(r["Grid_Size"]) >= 65536:
            calib = float(r["Counter_Value"])
            break
    last = max(i for i, r in enumerate(rows) if "k_check_velocity" in r["Kernel_Name"])
    by = {}
    for r in rows[last:]:
        by.setdefault(r["Kernel_Name"].split("(")[0].replace("void ", ""), []).append(
            float(r["Counter_Value"]))
    return by, calib


def of_symbol(by, sym):
    """All dispatches of a kernel, over its template instantiations."""
    vals = []
    for k, v in by.items():
        if k.split("<")[0].endswith(sym):
            vals += v
    return vals


def pmc(fetch_csv, write_csv, sym, workload, out, cmd_f, cmd_w):
    fb, fcal = per_kernel(fetch_csv)
    wb, wcal = per_kernel(write_csv)
    ff = COPY_BYTES / (fcal * 1024.0)
    wf = COPY_BYTES / (wcal * 1024.0)
    fv, wv = of_symbol(fb, sym), of_symbol(wb, sym)
    fk = sum(fv) / len(fv)
    wk = sum(wv) / len(wv)
    res = dict(kernel=sym, workload=workload, dispatches=len(fv),
               fetch_kib_per_dispatch=fk, write_kib_per_dispatch=wk,
               fetch_scale=ff, write_scale=wf,
               hbm_bytes_per_launch=fk * 1024 * ff + wk * 1024 * wf, source_hash=src_hash(sym))
    with open(out, "w") as f:
        f.write("# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, per dispatch of %s (%s), last step\n"
                % (sym, workload))
        f.write("# fetch command: %s\n# write command: %s\n" % (cmd_f, cmd_w))
        f.write("# calibration: 512 MiB device copy read FETCH_SIZE %.1f KiB, WRITE_SIZE %.1f KiB\n"
                % (fcal, wcal))
        f.write("# scale factors: fetch %.4f, write %.4f (bytes per counted KiB / 1024)\n" % (ff, wf))
        for k in sorted(fb, key=lambda k: -sum(fb[k]))[:12]:
            f.write("%-40s fetch %12.1f KiB/dispatch  write %12.1f KiB/dispatch  n=%d\n"
                    % (k[:40], sum(fb[k]) / len(fb[k]), sum(wb.get(k, [0])) / max(len(wb.get(k, [1])), 1),
                       len(fb[k])))
        f.write("result:%s\n" % json.dumps(res))


SQ_COUNTERS = ("SQ_VALU_MFMA_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS",
               "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_VMEM", "GRBM_GUI_ACTIVE")
SIMDS = 1024  # 256 compute units x 4 SIMDs


def sq(csv_path, workload, out, cmd):
    """Matrix-core busy fraction and stall shares per kernel over the last step.

    Each dispatch's value is summed over the counter's instances: the SQ
    counters over all SIMDs, GRBM_GUI_ACTIVE over the eight XCDs (so one
    XCD's active cycles are 1/8 of it).  MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES
    / (GRBM_GUI_ACTIVE / 8 x 1024 SIMDs); the waits and LDS activity are
    fractions of the waves' resident cycles (SQ_WAVE_CYCLES)."""
    rows = sorted(csv.DictReader(open(csv_path)), key=lambda r: int(r["Dispatch_Id"]))
    last = max(i for i, r in enumerate(rows) if "k_check_velocity" in r["Kernel_Name"])
    agg, disp = {}, {}
    for r in rows[last:]:
        k = r["Kernel_Name"].split("(")[0].replace("void ", "").split("<")[0]
        agg.setdefault(k, {c: 0.0 for c in SQ_COUNTERS})
        if r["Counter_Name"] in SQ_COUNTERS:
            agg[k][r["Counter_Name"]] += float(r["Counter_Value"])
        disp.setdefault(k, set()).add(r["Dispatch_Id"])
    with open(out, "w") as f:
        f.write("# rocprofv3 --pmc %s, per kernel over the last step (%s)\n" % (" ".join(SQ_COUNTERS), workload))
        f.write("# command: %s\n" % cmd)
        f.write("# mfma_busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 XCDs x %d SIMDs); "
                "wait_any, wait_lds, lds_active = per SQ_WAVE_CYCLES\n" % SIMDS)
        f.write("%-22s %6s %10s %9s %9s %11s %14s\n" % ("kernel", "calls", "mfma_busy", "wait_any", "wait_lds",
                                                       "lds_active", "lds_bank_confl"))
        for k, c in sorted(agg.items(), key=lambda kv: -kv[1]["GRBM_GUI_ACTIVE"]):
            if not k.startswith("hsw::") or c["GRBM_GUI_ACTIVE"] == 0:
                continue
            wc = max(c["SQ_WAVE_CYCLES"], 1.0)
            mf = c["SQ_VALU_MFMA_BUSY_CYCLES"] / (c["GRBM_GUI_ACTIVE"] / 8.0 * SIMDS)
            f.write("%-22s %6d %9.1f%% %9.3f %9.3f %11.3f %14.3f\n" % (
                k.replace("hsw::", ""), len(disp[k]), 100 * mf, c["SQ_WAIT_INST_ANY"] / wc,
                c["SQ_WAIT_INST_LDS"] / wc, c["SQ_ACTIVE_INST_LDS"] / wc,
                c["SQ_LDS_BANK_CONFLICT"] / max(c["SQ_ACTIVE_INST_LDS"], 1.0)))

if __name__ == "__main__":
    if sys.argv[1] == "sq":
        sq(*sys.argv[2:6])
    elif sys.argv[1] == "stats":
        stats(*sys.argv[2:6])
    else:
        pmc(*sys.argv[2:9])
