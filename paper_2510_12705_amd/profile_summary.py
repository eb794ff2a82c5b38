"""Summarise rocprofv3 CSV output of ``bench.py`` runs into the text files kept
under ``profiles/``.

  python -m paper_2510_12705_amd.profile_summary trace <kernel_stats.csv> <kernel_trace.csv> <out.md> "<command>" \
      [<kernel-name filter for the dispatch table, default bb_stage>]
  python -m paper_2510_12705_amd.profile_summary traffic <fetch_counter_collection.csv> <write_counter_collection.csv> \
      <out.json> <workload> <dtype> "<fetch command>" "<write command>" <copy MiB>
  python -m paper_2510_12705_amd.profile_summary counters <sq_counter_collection.csv> <tcc_counter_collection.csv> \
      <out.md> "<sq command>" "<tcc command>"

``traffic`` calibrates FETCH_SIZE / WRITE_SIZE (KiB per dispatch) against the
device copy of known size that ``bench.py --copy-calib-mib`` runs first (the
``__amd_rocclr_copyBuffer`` dispatch reads and writes that many bytes) and
records the HBM bytes per stage-kernel launch with the hash of the kernel
sources they were measured on; ``bench.py`` reports them only while the hash
matches.
"""
from __future__ import annotations

import csv
import json
import sys


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def trace(stats_csv, trace_csv, out_md, command, kernel="bb_stage"):
    stats = _rows(stats_csv)
    tr = _rows(trace_csv)
    lines = ["# rocprofv3 kernel trace: %s" % out_md.rsplit("/", 1)[-1].replace(".md", ""), "",
             "Command (from the repository root, on one MI355X):", "", "    %s" % command, "",
             "## --stats summary", "", "| kernel | calls | total ms | average ms | min ms | max ms | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in stats:
        lines.append("| `%s` | %s | %.3f | %.3f | %.3f | %.3f | %.2f |" % (
            r["Name"][:90], r["Calls"], float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e6,
            float(r["MinNs"]) / 1e6, float(r["MaxNs"]) / 1e6, float(r["Percentage"])))
    lines += ["", "## dispatches of the kernels named `%s`" % kernel, "",
              "| dispatch | kernel | ms | workgroups | threads/WG | VGPRs | LDS bytes | scratch |",
              "|---:|---|---:|---:|---:|---:|---:|---:|"]
    for r in tr:
        if kernel not in r["Kernel_Name"]:
            continue
        ms = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        wg = int(r["Workgroup_Size_X"])
        lines.append("| %s | `%s` | %.3f | %d | %d | %s | %s | %s |" % (
            r["Dispatch_Id"], r["Kernel_Name"][:60], ms, int(r["Grid_Size_X"]) // max(wg, 1), wg, r["VGPR_Count"],
            r["LDS_Block_Size"], r["Scratch_Size"]))
    lines += ["", "LDS bytes is the static LDS segment as rocprofv3 reports it; LDS requested at launch",
              "(dynamic shared memory) is not included."]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def traffic(fetch_csv, write_csv, out_json, workload, dtype, fetch_cmd, write_cmd, copy_mib):
    sys.path.insert(0, __file__.rsplit("/", 2)[0])
    from bench import kernel_source_hash  # the same hash bench.py checks
    copy_bytes = float(copy_mib) * (1 << 20)
    res = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _rows(path)
        copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
                and r["Counter_Name"] == name]
        stage = [float(r["Counter_Value"]) for r in rows if "bb_stage" in r["Kernel_Name"]
                 and r["Counter_Name"] == name]
        scale = copy_bytes / (max(copy) * 1024.0)
        res[name] = {"copy_kib": max(copy), "scale_bytes_per_kib": scale * 1024.0,
                     "stage_kib": stage, "stage_bytes": [v * 1024.0 * scale for v in stage]}
    nl = min(len(res["FETCH_SIZE"]["stage_bytes"]), len(res["WRITE_SIZE"]["stage_bytes"]))
    per = [res["FETCH_SIZE"]["stage_bytes"][i] + res["WRITE_SIZE"]["stage_bytes"][i] for i in range(nl)]
    out = {"workload": workload, "dtype": dtype, "kernel_source_hash": kernel_source_hash(),
           "copy_calibration_mib": float(copy_mib), "fetch_command": fetch_cmd, "write_command": write_cmd,
           "counters": res, "hbm_bytes_per_launch": sum(per) / max(nl, 1), "hbm_bytes_per_stage": per}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)


def counters(sq_csv, tcc_csv, out_md, sq_cmd, tcc_cmd, simds=1024):
    """Per stage-kernel dispatch: occupancy, L2 hit rate, LDS bank conflicts, memory
    instruction counts.  The stage kernel is persistent (every workgroup lives until
    the stage ends), so the waves resident per SIMD are SQ_WAVES / simds."""
    per = {}
    for path in (sq_csv, tcc_csv):
        for r in _rows(path):
            if "bb_stage" not in r["Kernel_Name"]:
                continue
            d = per.setdefault(int(r["Dispatch_Id"]), {"kernel": r["Kernel_Name"], "wg": r["Workgroup_Size"],
                                                         "grid": r["Grid_Size"], "vgpr": r["VGPR_Count"]})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
            if path == sq_csv:
                d["ms"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    lines = ["# rocprofv3 counters: %s" % out_md.rsplit("/", 1)[-1].replace(".md", ""), "",
             "Commands (from the repository root, on one MI355X; one counter pass each):", "",
             "    %s" % sq_cmd, "", "    %s" % tcc_cmd, "",
             "Per stage-kernel dispatch (one per bandwidth-reduction stage).  The kernel is persistent,",
             "so waves resident per SIMD = SQ_WAVES / %d SIMDs for the whole dispatch;" % simds,
             "L2 hit rate = TCC_HIT / (TCC_HIT + TCC_MISS); LDS conflict cycles per LDS instruction =",
             "SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS.", "",
             "| dispatch | kernel | ms | waves | waves/SIMD resident | L2 hit rate | LDS conflict cycles / LDS instr |"
             " VMEM rd instr | VMEM wr instr | LDS instr |",
             "|---:|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(per):
        d = per[k]
        occ = d.get("SQ_WAVES", 0.0) / simds
        hit = d.get("TCC_HIT_sum", 0.0) / max(d.get("TCC_HIT_sum", 0.0) + d.get("TCC_MISS_sum", 0.0), 1.0)
        lds = d.get("SQ_LDS_BANK_CONFLICT", 0.0) / max(d.get("SQ_INSTS_LDS", 1.0), 1.0)
        lines.append("| %d | `%s` | %.1f | %d | %.2f | %.3f | %.4f | %.3e | %.3e | %.3e |" % (
            k, d["kernel"][:44], d.get("ms", 0.0), int(d.get("SQ_WAVES", 0)), occ, hit, lds,
            d.get("SQ_INSTS_VMEM_RD", 0.0), d.get("SQ_INSTS_VMEM_WR", 0.0), d.get("SQ_INSTS_LDS", 0.0)))
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(*sys.argv[2:7])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:10])
    elif sys.argv[1] == "counters":
        counters(*sys.argv[2:7])
    else:
        raise SystemExit(__doc__)
