"""Short text summaries of rocprofv3 CSV output (kernel stats, dispatch trace, PMC).

  python -m paper_2004_03972_amd.profsum stats  <prefix>_kernel_stats.csv [--top 12]
  python -m paper_2004_03972_amd.profsum trace  <prefix>_kernel_trace.csv --kernel SUBSTR
  python -m paper_2004_03972_amd.profsum pmc    <prefix>_counter_collection.csv --kernel SUBSTR
  python -m paper_2004_03972_amd.profsum calib  <prefix>_counter_collection.csv --bytes B

``pmc`` prints the mean counter value (KiB per dispatch) over the dispatches whose
name contains SUBSTR; ``calib`` prints the counter of the largest dispatch (a plain
copy of B bytes) and the factor B / (1024 * value) that turns the counter into bytes.
``srchash`` prints the SHA-256 of the dense step kernel's sources, stored beside PMC
figures so that a later reader can tell whether the kernel changed since.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import statistics
import sys

DENSE_SOURCES = ("csrc/k_md_dense.hip", "csrc/md_epilogue.h", "csrc/hqa_internal.h")
CSR_SOURCES = ("csrc/k_md_csr.hip", "csrc/md_epilogue.h", "csrc/hqa_internal.h")
RESIDENT_SOURCES = ("csrc/k_md_resident.hip", "csrc/md_epilogue.h", "csrc/hqa_internal.h")
PERSIST_SOURCES = ("csrc/k_md_persist.hip", "csrc/md_epilogue.h", "csrc/hqa_internal.h")
CSR_RESIDENT_SOURCES = ("csrc/k_csr_resident.hip", "csrc/md_epilogue.h", "csrc/hqa_internal.h")
BATCH_SOURCES = ("csrc/k_md_batch.hip", "csrc/md_epilogue.h", "csrc/hqa_internal.h")
SOURCES = {"dense": DENSE_SOURCES, "csr": CSR_SOURCES, "resident": RESIDENT_SOURCES,
           "batch": BATCH_SOURCES,
           "persist": PERSIST_SOURCES, "csr_resident": CSR_RESIDENT_SOURCES}


def source_hash(files=DENSE_SOURCES) -> str:
    h = hashlib.sha256()
    base = os.path.dirname(os.path.abspath(__file__))
    for f in files:
        with open(os.path.join(base, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def stats(path, top=12):
    rows = _rows(path)
    print(f"{'kernel':<90} {'calls':>7} {'avg_us':>10} {'total_ms':>10} {'pct':>6}")
    for r in rows[:top]:
        print(f"{r['Name'][:90]:<90} {int(r['Calls']):>7} {float(r['AverageNs']) / 1e3:>10.3f} "
              f"{float(r['TotalDurationNs']) / 1e6:>10.2f} {float(r['Percentage']):>6.2f}")


def trace(path, kernel, last=0):
    rows = [r for r in _rows(path) if kernel in r["Kernel_Name"]]
    if not rows:
        sys.exit(f"no dispatch matches {kernel!r}")
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    if last:                                   # only the last dispatches (the timed runs)
        rows = rows[-last:]
        print(f"last {len(rows)} dispatches of the kernel")
    dur = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows]
    gap = [int(b["Start_Timestamp"]) - int(a["End_Timestamp"]) for a, b in zip(rows, rows[1:])]
    per = [int(b["Start_Timestamp"]) - int(a["Start_Timestamp"]) for a, b in zip(rows, rows[1:])]
    r0 = rows[0]
    print(f"kernel {r0['Kernel_Name']}")
    print(f"grid {r0['Grid_Size_X']}x{r0['Grid_Size_Y']}x{r0['Grid_Size_Z']} workgroup "
          f"{r0['Workgroup_Size_X']} VGPR {r0['VGPR_Count']} AGPR {r0['Accum_VGPR_Count']} "
          f"SGPR {r0['SGPR_Count']} LDS {r0['LDS_Block_Size']} scratch {r0['Scratch_Size']}")
    print(f"dispatches {len(rows)}; duration us: mean {statistics.mean(dur) / 1e3:.3f} "
          f"median {statistics.median(dur) / 1e3:.3f}")
    if gap:
        print(f"start-to-start us: mean {statistics.mean(per) / 1e3:.3f} median "
              f"{statistics.median(per) / 1e3:.3f}; end-to-start gap us: median "
              f"{statistics.median(gap) / 1e3:.3f}")


def pmc(path, kernel, last=0):
    rows = [r for r in _rows(path) if kernel in r["Kernel_Name"]]
    if not rows:
        sys.exit(f"no dispatch matches {kernel!r}")
    if last:                                   # only the last dispatches (the timed runs)
        rows.sort(key=lambda r: int(r.get("Dispatch_Id", 0)))
        rows = rows[-last:]
        print(f"last {len(rows)} dispatches of the kernel")
    by = {}
    for r in rows:
        by.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    print(f"kernel {rows[0]['Kernel_Name']}")
    for c, v in by.items():
        print(f"{c}: dispatches {len(v)} mean {statistics.mean(v):.3f} KiB median "
              f"{statistics.median(v):.3f} KiB")


def calib(path, nbytes):
    rows = _rows(path)
    r = max(rows, key=lambda r: float(r["Counter_Value"]))
    v = float(r["Counter_Value"])
    print(f"largest dispatch {r['Kernel_Name'][:100]}")
    print(f"{r['Counter_Name']}: {v:.3f} KiB for {nbytes} B; factor {nbytes / 1024 / v:.4f}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "trace", "pmc", "calib", "srchash"])
    ap.add_argument("path", nargs="?")
    ap.add_argument("--kernel", default="")
    ap.add_argument("--top", type=int, default=12)
    ap.add_argument("--bytes", type=int, default=0)
    ap.add_argument("--sources", default="dense", choices=sorted(SOURCES))
    ap.add_argument("--last", type=int, default=0, help="only the last N dispatches")
    a = ap.parse_args(argv)
    if a.mode == "stats":
        stats(a.path, a.top)
    elif a.mode == "trace":
        trace(a.path, a.kernel, a.last)
    elif a.mode == "pmc":
        pmc(a.path, a.kernel, a.last)
    elif a.mode == "calib":
        calib(a.path, a.bytes)
    else:
        print(source_hash(SOURCES[a.sources]))


if __name__ == "__main__":
    main()
