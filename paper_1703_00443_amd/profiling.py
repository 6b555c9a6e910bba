"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_1703_00443_amd.profiling stats  <run_kernel_stats.csv>
    python -m paper_1703_00443_amd.profiling traffic <fetch_counter_collection.csv> \
        <write_counter_collection.csv> --kernel qp_forward_kernel --calib-bytes N
    python -m paper_1703_00443_amd.profiling util <counter_collection.csv> --kernel K --active-cus C

`stats` prints the kernel-time table as markdown.  `traffic` computes HBM bytes
per dispatch of a kernel from two --pmc runs (FETCH_SIZE, then WRITE_SIZE, both
in KiB per dispatch), each scaled by what the same counter reads for the
largest device copy in the run (a copy of `--calib-bytes` bytes read and
written), and prints a markdown block with the per-launch figures.
"""
from __future__ import annotations

import argparse
import collections
import csv
import statistics


def kernel_stats_markdown(path: str, top: int = 12) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | average (us) | min (us) | max (us) | share |",
           "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append("| `%s` | %s | %.1f | %.1f | %.1f | %.1f%% |" % (
            r["Name"][:90], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out)


def _per_kernel(path: str):
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        vals[r["Kernel_Name"]].append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    return vals


def traffic(fetch_csv: str, write_csv: str, kernel: str, calib_bytes: int):
    f, w = _per_kernel(fetch_csv), _per_kernel(write_csv)

    def calib(vals):
        # the copy kernel with the largest grid in the run is the calibration copy
        best = None
        for name, lst in vals.items():
            if "copyBuffer" in name or "copy" in name.lower():
                for grid, v in lst:
                    if best is None or grid > best[0]:
                        best = (grid, [x for g, x in lst if g == grid])
        if best is None:
            raise SystemExit("no copy kernel found for calibration")
        return (calib_bytes / 1024.0) / statistics.median(best[1])

    cf, cw = calib(f), calib(w)
    name = next(k for k in f if kernel in k)
    # the first dispatch warms caches and problem data; use the steady state
    fk = [v for _, v in f[name]][1:] or [v for _, v in f[name]]
    wk = [v for _, v in w[name]][1:] or [v for _, v in w[name]]
    fetch = statistics.median(fk) * cf * 1024
    write = statistics.median(wk) * cw * 1024
    return {"kernel": name, "fetch_scale": cf, "write_scale": cw, "fetch_bytes": fetch,
            "write_bytes": write, "hbm_bytes_per_launch": fetch + write}


def utilization(counter_csv: str, kernel: str, active_cus: int, total_cus: int = 256, xcds: int = 8,
                simds_per_cu: int = 4):
    """MFMA and VALU busy fractions of one kernel from a --pmc run that holds
    SQ_VALU_MFMA_BUSY_CYCLES, SQ_ACTIVE_INST_VALU, SQ_BUSY_CU_CYCLES, GRBM_GUI_ACTIVE
    and the MFMA / VALU instruction counters.  Definitions follow rocprofv3's
    derived metrics (MfmaUtil, VALUBusy), with GRBM_GUI_ACTIVE summed over the
    XCDs divided by their number; the '_active' figures divide by the CUs that
    held work (one workgroup per CU)."""
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    name = None
    for r in csv.DictReader(open(counter_csv)):
        if kernel in r["Kernel_Name"]:
            name = r["Kernel_Name"]
            per[int(r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
    if not per:
        raise SystemExit("kernel %s not found" % kernel)
    steady = [per[d] for d in sorted(per)][1:] or [per[d] for d in sorted(per)]
    med = {k: statistics.median(v[k] for v in steady) for k in steady[0]}
    gui = med["GRBM_GUI_ACTIVE"] / xcds
    out = {"kernel": name, "dispatches": len(steady), "gpu_cycles": gui}
    mf = med.get("SQ_VALU_MFMA_BUSY_CYCLES")
    if mf is not None:
        out["mfma_busy_chip"] = mf / (total_cus * simds_per_cu * gui)
        out["mfma_busy_active"] = mf / (active_cus * simds_per_cu * gui)
    va = med.get("SQ_ACTIVE_INST_VALU")
    if va is not None:
        out["valu_busy_chip"] = va / (total_cus * gui)
        out["valu_busy_active"] = va / (active_cus * gui)
    for k in ("SQ_INSTS_MFMA", "SQ_INSTS_VALU", "SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_INSTS_VALU_MFMA_MOPS_F32",
              "SQ_INSTS_VALU_FLOPS_FP64", "SQ_INSTS_VALU_FLOPS_FP32", "SQ_BUSY_CU_CYCLES"):
        if k in med:
            out[k] = med[k]
    for k, f in (("SQ_INSTS_VALU_MFMA_MOPS_F64", 512), ("SQ_INSTS_VALU_MFMA_MOPS_F32", 512)):
        if k in med:
            out["mfma_flops_per_launch"] = med[k] * f
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--kernel", required=True)
    b.add_argument("--calib-bytes", type=int, required=True)
    c = sub.add_parser("util")
    c.add_argument("csv")
    c.add_argument("--kernel", required=True)
    c.add_argument("--active-cus", type=int, required=True)
    args = ap.parse_args()
    if args.cmd == "util":
        for k, v in utilization(args.csv, args.kernel, args.active_cus).items():
            print("%s: %s" % (k, ("%.6g" % v) if isinstance(v, float) else v))
        return
    if args.cmd == "stats":
        print(kernel_stats_markdown(args.csv))
    else:
        t = traffic(args.fetch_csv, args.write_csv, args.kernel, args.calib_bytes)
        print("kernel: %s" % t["kernel"])
        print("fetch_scale: %.4f" % t["fetch_scale"])
        print("write_scale: %.4f" % t["write_scale"])
        print("fetch_bytes_per_launch: %.0f" % t["fetch_bytes"])
        print("write_bytes_per_launch: %.0f" % t["write_bytes"])
        print("hbm_bytes_per_launch: %.0f" % t["hbm_bytes_per_launch"])


if __name__ == "__main__":
    main()
