"""Summaries of rocprofv3 output for the profiles kept with the sources.

  python -m paper_1705_04601_amd.profsum stats <out_dir> <prefix>
      per-kernel totals from <prefix>_kernel_stats.csv and, for each Schur
      kernel, the per-launch average from <prefix>_kernel_trace.csv
  python -m paper_1705_04601_amd.profsum traffic <fetch_dir> <fetch_prefix> <write_dir> <write_prefix> <copy_mib> [kernel]
      HBM bytes per launch of one kernel (default the Schur kernel of tile class 1)
      from a FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch), each
      scaled by what the counter reads for the plain copy of <copy_mib> MiB
      that bench.py --copy-probe-mib runs first

  python -m paper_1705_04601_amd.profsum counters <out_dir> <prefix> <kernel substring>
      per kernel matching the substring: every counter summed over its
      dispatches; with SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE the MFMA
      busy fraction (busy SIMD cycles over active cycles of all 1024 SIMDs;
      GRBM_GUI_ACTIVE is summed over the 8 XCDs, so divided by 8)

  python -m paper_1705_04601_amd.profsum busy <out_dir> <prefix> <first_regex> <last_regex> [after_regex]
      device occupancy of one phase from <prefix>_kernel_trace.csv: the window
      from the first start of a kernel matching first_regex (after the last
      kernel matching after_regex, when given) to the last end of a kernel
      matching last_regex, the union of all kernel intervals inside it (busy,
      whatever stream they ran on), and the idle time with its gaps

Reads CSV files only; prints text.
"""

from __future__ import annotations

import csv
import hashlib
import os
import sys

SCHUR = "schur_kernel<float, 1>"  # the Schur kernel of the whole leaf targets
SCHUR_ANY = "schur_kernel<"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, "paper_1705_04601_amd", "csrc", f) for f in ("kernels.hip", "device_common.h", "factor.cpp")]


def _short(name: str) -> str:
    name = name.replace("h2::(anonymous namespace)::", "")
    return name.split("(")[0][:90]


def stats(out_dir: str, prefix: str) -> None:
    rows = list(csv.DictReader(open(os.path.join(out_dir, f"{prefix}_kernel_stats.csv"))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    print(f"{'kernel':92s} {'calls':>7s} {'total ms':>10s} {'avg us':>10s} {'%':>6s}")
    for r in rows[:15]:
        t = float(r["TotalDurationNs"])
        print(f"{_short(r['Name']):92s} {int(r['Calls']):7d} {t / 1e6:10.1f} "
              f"{float(r['AverageNs']) / 1e3:10.1f} {100 * t / total:6.1f}")
    trace = os.path.join(out_dir, f"{prefix}_kernel_trace.csv")
    if os.path.exists(trace):
        per = {}
        for r in csv.DictReader(open(trace)):
            if SCHUR_ANY in r["Kernel_Name"]:
                per.setdefault(_short(r["Kernel_Name"]), []).append(
                    int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        for name, d in sorted(per.items()):
            print(f"\n{name}: {len(d)} launches, {sum(d) / 1e6:.1f} ms, average {sum(d) / len(d) / 1e6:.4f} ms")


def _counter(out_dir: str, prefix: str, counter: str):
    per = {}
    for r in csv.DictReader(open(os.path.join(out_dir, f"{prefix}_counter_collection.csv"))):
        if r["Counter_Name"] != counter:
            continue
        key = int(r["Dispatch_Id"])
        name = r["Kernel_Name"]
        per.setdefault(key, [name, 0.0])[1] += float(r["Counter_Value"])
    return per


def traffic(fdir, fprefix, wdir, wprefix, copy_mib, kernel=SCHUR) -> None:
    copy_bytes = copy_mib * (1 << 20)
    out = {}
    for what, d, p, counter in (("fetch", fdir, fprefix, "FETCH_SIZE"), ("write", wdir, wprefix, "WRITE_SIZE")):
        per = _counter(d, p, counter)
        copies = [v for n, v in per.values() if "copy" in n.lower() and v * 1024 > 0.5 * copy_bytes]
        schur = [v for n, v in per.values() if kernel in n]
        if not copies or not schur:
            raise SystemExit(f"{counter}: no copy probe or no {kernel} dispatch found")
        measured = sorted(copies)[len(copies) // 2] * 1024
        scale = copy_bytes / measured
        per_launch = sum(schur) * 1024 * scale / len(schur)
        out[what] = per_launch
        print(f"{counter}: copy probe reads {measured / 2**20:.1f} MiB for {copy_mib} MiB moved -> scale {scale:.4f}; "
              f"{kernel}: {len(schur)} launches, {per_launch / 1e9:.3f} GB per launch after scaling")
    h = hashlib.sha256()
    for f in SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    print(f"kernel: {kernel}")
    print(f"fetch_bytes_per_launch: {out['fetch']:.6g}")
    print(f"write_bytes_per_launch: {out['write']:.6g}")
    print(f"hbm_bytes_per_launch: {out['fetch'] + out['write']:.6g}")
    print(f"sources_sha256: {h.hexdigest()}")


def counters(out_dir: str, prefix: str, sub: str) -> None:
    tot = {}
    for r in csv.DictReader(open(os.path.join(out_dir, f"{prefix}_counter_collection.csv"))):
        name = _short(r["Kernel_Name"])
        if sub not in name:
            continue
        d = tot.setdefault(name, {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    for name, d in sorted(tot.items()):
        line = ", ".join(f"{c} {v:.4g}" for c, v in sorted(d.items()))
        if "SQ_VALU_MFMA_BUSY_CYCLES" in d and d.get("GRBM_GUI_ACTIVE"):
            busy = d["SQ_VALU_MFMA_BUSY_CYCLES"] / (d["GRBM_GUI_ACTIVE"] / 8 * 1024)
            line += f"; MFMA busy {busy:.3f}"
        print(f"{name}: {line}")


def busy(out_dir: str, prefix: str, first: str, last: str, after: str | None = None) -> None:
    import re
    rows = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"])
            for r in csv.DictReader(open(os.path.join(out_dir, f"{prefix}_kernel_trace.csv")))]
    rf, rl = re.compile(first), re.compile(last)
    ta = max((a for a, _, k in rows if re.search(after, k)), default=0) if after else 0
    t0 = min(a for a, _, k in rows if rf.search(k) and a > ta)
    t1 = max(b for _, b, k in rows if rl.search(k))
    iv = sorted((max(a, t0), min(b, t1)) for a, b, _ in rows if b > t0 and a < t1)
    busy_ns, gaps, cur_a, cur_b = 0, [], iv[0][0], iv[0][1]
    if cur_a > t0:
        gaps.append(cur_a - t0)
    for a, b in iv[1:]:
        if a > cur_b:
            busy_ns += cur_b - cur_a
            gaps.append(a - cur_b)
            cur_a, cur_b = a, b
        else:
            cur_b = max(cur_b, b)
    busy_ns += cur_b - cur_a
    gaps.sort()
    med = gaps[len(gaps) // 2] if gaps else 0
    print(f"window {first!r} .. {last!r}: {len(iv)} kernels over {(t1 - t0) / 1e6:.1f} ms, "
          f"busy {busy_ns / 1e6:.1f} ms ({busy_ns / max(1, t1 - t0):.3f}), idle {sum(gaps) / 1e6:.1f} ms "
          f"in {len(gaps)} gaps (median {med / 1e3:.1f} us, largest {(gaps[-1] if gaps else 0) / 1e6:.2f} ms)")


def main(argv):
    if len(argv) >= 3 and argv[0] == "stats":
        stats(argv[1], argv[2])
    elif len(argv) >= 4 and argv[0] == "counters":
        counters(argv[1], argv[2], argv[3])
    elif len(argv) >= 5 and argv[0] == "busy":
        busy(argv[1], argv[2], argv[3], argv[4], *argv[5:6])
    elif len(argv) >= 6 and argv[0] == "traffic":
        traffic(argv[1], argv[2], argv[3], argv[4], int(argv[5]), *argv[6:7])
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
