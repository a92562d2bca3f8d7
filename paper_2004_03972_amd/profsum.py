"""Short text summaries of rocprofv3 CSV output (kernel stats, dispatch trace, PMC).

  python -m paper_2004_03972_amd.profsum stats  <prefix>_kernel_stats.csv [--top 12]
  python -m paper_2004_03972_amd.profsum trace  <prefix>_kernel_trace.csv --kernel SUBSTR
  python -m paper_2004_03972_amd.profsum pmc    <prefix>_counter_collection.csv --kernel SUBSTR
  python -m paper_2004_03972_amd.profsum calib  <prefix>_counter_collection.csv --bytes B

``pmc`` prints the mean counter value (KiB per dispatch) over the dispatches whose
name contains SUBSTR; ``calib`` prints the counter of the largest dispatch (a plain
copy of B bytes) and the factor B / (1024 * value) that turns the counter into bytes.
``srchash`` prints the SHA-256 of the dense step kernel's sources, stored beside PMC
figures so that a later reader can tell whether the kernel changed since.  ``isahash``
prints the SHA-256 of one kernel's gfx950 machine code as built into libhqa.so (its
instruction text without addresses up to its last s_endpgm, plus its kernel
descriptor): a host-only edit of a shared header, or a change of another kernel, leaves
it unchanged; any change of the kernel's code does not.

  python -m paper_2004_03972_amd.profsum isahash --kernel k_step_batch_lds [--lib PATH]
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
import shutil
import statistics
import subprocess
import sys
import tempfile

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


_LLVM = "/opt/rocm/llvm/bin"
_BUNDLE_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
_TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


def _tool(name):
    p = os.path.join(_LLVM, name)
    return p if os.access(p, os.X_OK) else shutil.which(name)


def isa_hash(kernel: str, lib: str | None = None) -> str | None:
    """SHA-256 of the gfx950 code of the kernel whose demangled name contains
    `kernel` (exactly one such kernel must exist) in the library's offload bundles, or
    None when the ROCm object tools are missing or the kernel is not found.  The
    instruction text is taken without addresses and encodings (branch offsets are
    relative), so the hash does not move when other kernels of the library change."""
    tools = [_tool(t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf",
                                "llvm-objdump")]
    if None in tools:
        return None
    objcopy, bundler, readelf, objdump = tools
    lib = lib or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhqa.so")
    with tempfile.TemporaryDirectory() as tmp:
        fb = os.path.join(tmp, "fatbin")
        r = subprocess.run([objcopy, f"--dump-section=.hip_fatbin={fb}", lib,
                            os.path.join(tmp, "stripped")], capture_output=True)
        if r.returncode or not os.path.exists(fb):
            return None
        data = open(fb, "rb").read()
        offs = [m.start() for m in re.finditer(re.escape(_BUNDLE_MAGIC), data)] + [len(data)]
        found = []
        for i, (a, b) in enumerate(zip(offs, offs[1:])):
            bi, co = os.path.join(tmp, f"b{i}"), os.path.join(tmp, f"c{i}.o")
            with open(bi, "wb") as fh:
                fh.write(data[a:b])
            if subprocess.run([bundler, "--unbundle", "--type=o", f"--input={bi}",
                               f"--targets={_TARGET}", f"--output={co}"],
                              capture_output=True).returncode:
                continue
            # the symbol table twice, mangled and demangled, in the same order
            tabs = [subprocess.run([readelf, "-s", "--wide", *opt, co], capture_output=True,
                                   text=True).stdout.splitlines() for opt in ((), ("-C",))]
            if len(tabs[0]) != len(tabs[1]):
                continue
            for raw, dem in zip(*tabs):
                f = raw.split(None, 7)
                g = dem.split(None, 7)
                if len(f) == 8 and len(g) == 8 and f[3] == "FUNC" and kernel in g[7]:
                    found.append((co, f[7]))
        names = {n for _, n in found}
        if len(names) != 1:
            return None
        co, name = found[0]
        dis = subprocess.run([objdump, "-d", "--no-show-raw-insn", "--no-leading-addr",
                              f"--disassemble-symbols={name}", co],
                             capture_output=True, text=True).stdout
        lines = dis.splitlines()
        start = next((k for k, ln in enumerate(lines) if ln.startswith(f"{name}>:")
                      or ln.endswith(f"<{name}>:")), None)
        if start is None:
            return None
        body = [ln.split("//")[0].rstrip() for ln in lines[start:]]
        body = [ln for ln in body if ln.strip()]
        # the padding after the last s_endpgm depends on what the linker placed next
        ends = [k for k, ln in enumerate(body) if ln.split() and ln.split()[0] == "s_endpgm"]
        if ends:
            body = body[:ends[-1] + 1]
        if len(body) < 2:
            return None
        # the kernel descriptor (register counts, LDS size, launch properties)
        kd = subprocess.run([readelf, "-s", "--wide", co], capture_output=True,
                            text=True).stdout
        h = hashlib.sha256("\n".join(body).encode())
        for line in kd.splitlines():
            f = line.split()
            if len(f) >= 8 and f[7] == name + ".kd":
                kdb = bytearray(_kd_bytes(co, int(f[1], 16), int(f[2])))
                kdb[16:24] = bytes(8)      # the code entry offset depends on the layout
                h.update(bytes(kdb))
                break
        return h.hexdigest()


def _kd_bytes(obj, vaddr, size):
    """Bytes of a symbol at virtual address vaddr in an ELF object's loaded sections."""
    import struct
    d = open(obj, "rb").read()
    shoff, = struct.unpack_from("<Q", d, 0x28)
    shentsize, shnum = struct.unpack_from("<HH", d, 0x3A)
    for k in range(shnum):
        o = shoff + k * shentsize
        _, typ, _, addr, off, sz = struct.unpack_from("<IIQQQQ", d, o)
        if typ != 8 and addr <= vaddr < addr + sz:          # not SHT_NOBITS
            return d[off + vaddr - addr: off + vaddr - addr + size]
    return b""


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def stats(path, top=12):
    rows = _rows(path)
    print(f"{'kernel':<90} {'calls':>7} {'avg_us':>10} {'total_ms':>10} {'pct':>6}")
    for r in rows[:top]:
        print(f"{r['Name'][:90]:<90} {int(r['Calls']):>7} {float(r['AverageNs']) / 1e3:>10.3f} "
              f"{float(r['TotalDurationNs']) / 1e6:>10.2f} {float(r['Percentage']):>6.2f}")


def trace(path, kernel, last=0, span=""):
    rows = [r for r in _rows(path) if kernel in r["Kernel_Name"]]
    if not rows:
        sys.exit(f"no dispatch matches {kernel!r}")
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    if span:                                   # dispatches a..b-1 in launch order
        a, b = (int(x) for x in span.split(":"))
        rows = rows[a:b]
        print(f"dispatches {a}..{b - 1} of the kernel (launch order, from 0)")
    elif last:                                 # only the last dispatches (the timed runs)
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
    ap.add_argument("mode", choices=["stats", "trace", "pmc", "calib", "srchash", "isahash"])
    ap.add_argument("path", nargs="?")
    ap.add_argument("--kernel", default="")
    ap.add_argument("--top", type=int, default=12)
    ap.add_argument("--bytes", type=int, default=0)
    ap.add_argument("--sources", default="dense", choices=sorted(SOURCES))
    ap.add_argument("--last", type=int, default=0, help="only the last N dispatches")
    ap.add_argument("--span", default="", help="trace: only dispatches A..B-1 (A:B)")
    ap.add_argument("--lib", default=None, help="library for isahash (default libhqa.so)")
    a = ap.parse_args(argv)
    if a.mode == "stats":
        stats(a.path, a.top)
    elif a.mode == "trace":
        trace(a.path, a.kernel, a.last, a.span)
    elif a.mode == "pmc":
        pmc(a.path, a.kernel, a.last)
    elif a.mode == "calib":
        calib(a.path, a.bytes)
    elif a.mode == "isahash":
        h = isa_hash(a.kernel, a.lib)
        if h is None:
            sys.exit(f"no unique gfx950 kernel matching {a.kernel!r} (or no ROCm object tools)")
        print(h)
    else:
        print(source_hash(SOURCES[a.sources]))


if __name__ == "__main__":
    main()
