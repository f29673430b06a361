"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_1705_02257_amd.profiling stats  TRACE_DIR  OUT.md  --command "..."
    python -m paper_1705_02257_amd.profiling sq     PMC_DIR    OUT.md  --command "..."
    python -m paper_1705_02257_amd.profiling traffic FETCH_DIR WRITE_DIR OUT_DIR \
        --copy-bytes N --command "..."

`stats` reads the kernel_stats.csv of a `rocprofv3 --kernel-trace --stats
--output-format csv` run and writes a markdown table (calls, total and
average duration per kernel) headed by the command that produced it.

`sq` reads the counter_collection.csv of one `rocprofv3 --pmc` run of SQ
counters (SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT
SQ_WAIT_INST_LDS SQ_BUSY_CYCLES) and writes per library kernel the counter
sums and three shares of the kernel's time (its dispatch durations, 256 CUs
at 2.4 GHz): LDS bank conflicts per CU-cycle, SIMD time issuing vector
instructions (a wave64 instruction holds its 16-lane SIMD for 4 cycles),
and wave time waiting to issue LDS instructions (for kernels whose resident
waves per CU are known).

`traffic` reads the counter_collection.csv of two `rocprofv3 --pmc` runs of
the same program, one with FETCH_SIZE and one with WRITE_SIZE (KiB per
dispatch), each summed per kernel kind over its own run.  Records are
stamped with a hash of the kernel and driver code (comments and whitespace
left out).  The program must sort exactly once and contain one plain
device-to-device copy of `copy-bytes` bytes (the largest copyBuffer
dispatch): the ratio between its
known size and what each counter reports for it is the calibration factor
applied to every other dispatch.  For each kernel kind it writes
traffic_<kind>.json with the calibrated HBM bytes of all its dispatches in
the sort (hbm_bytes), stamped with the hash of the kernel sources the
counters were taken on.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f)
                  for f in ("kernels.hpp", "traits.hpp", "driver.hip", "planner.hpp", "wrword.hpp")]

# kernel-name prefix -> the kernel kind the library reports timings under
# (one timing record may span several launches: the overhang copy and the
# cleanup; the counting sort and its merge-sort fallback)
KINDS = [("k_sample", "sample"), ("k_classify", "classify"), ("k_scan", "scan"),
         ("k_fix_empty", "fix_empty"), ("k_permute", "permute"), ("k_overhang", "cleanup"),
         ("k_cleanup", "cleanup"), ("k_basecase", "basecase"), ("k_mark_max", "mark"), ("k_walk", "mark"),
         ("k_search_next", "mark")]
COPY = "__amd_rocclr_copyBuffer"


def _code_only(text: str) -> str:
    """The source without comments and whitespace (string literals kept), so
    that an edit to comments alone leaves the hash as it was."""
    out, i, n = [], 0, len(text)
    while i < n:
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif text[i] == '"':
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            if not text[i].isspace():
                out.append(text[i])
            i += 1
    return "".join(out)


def source_sha(sources=None) -> str:
    """Hash of the kernel and driver code the counters describe."""
    h = hashlib.sha256()
    for p in sources or KERNEL_SOURCES:
        with open(p, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def kind_of(name: str):
    for prefix, kind in KINDS:
        if re.search(r"\b" + prefix, name):
            return kind
    return None


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def stats_summary(trace_dir: str, command: str) -> str:
    rows = list(csv.DictReader(open(_find(trace_dir, "kernel_stats.csv"))))
    out = ["# Kernel time (rocprofv3 --kernel-trace --stats)", "", "Command:", "",
           "```", command, "```", "",
           "| kernel | calls | total ms | average us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows:
        name = r["Name"]
        short = re.sub(r"\(.*", "", name).replace("void ", "")
        out.append(f"| `{short}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def _counter(d: str, counter: str):
    per = []
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        if r["Counter_Name"] == counter:
            per.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return per


# resident waves per CU of the kernels whose occupancy is fixed by their
# LDS and workgroup shape (one 1024-lane workgroup, or two of 512 lanes;
# the permutation runs 8 four-wave workgroups per CU)
RESIDENT_WAVES = [("k_classify<", 16), ("k_basecase_count<", 16), ("k_sample<0, 1024", 16),
                  ("k_sample<1, 1024", 16), ("k_permute<", 32)]
SQ_COUNTERS = ["SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_LDS"]


def sq_table(pmc_dir: str, cus: int = 256, ghz: float = 2.4):
    """{kernel: {dispatches, ms, counter sums, conflict/valu/ldswait shares}}."""
    acc, spans = {}, {}
    for r in csv.DictReader(open(_find(pmc_dir, "counter_collection.csv"))):
        m = re.search(r"ips4o::(k_\w+<[^>]*>)", r["Kernel_Name"])
        if not m:
            continue
        k = m.group(1)
        a = acc.setdefault(k, {c: 0.0 for c in SQ_COUNTERS})
        if r["Counter_Name"] in a:
            a[r["Counter_Name"]] += float(r["Counter_Value"])
        spans.setdefault(k, {})[r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    out = {}
    for k, a in acc.items():
        ms = sum(spans[k].values())
        cyc = ms * 1e-3 * ghz * 1e9
        waves = next((w for pre, w in RESIDENT_WAVES if k.startswith(pre)), None)
        out[k] = dict(a, dispatches=len(spans[k]), ms=ms,
                      conflict=a["SQ_LDS_BANK_CONFLICT"] / (cus * cyc) if cyc else 0.0,
                      valu=4 * a["SQ_INSTS_VALU"] / (cus * 4 * cyc) if cyc else 0.0,
                      ldswait=a["SQ_WAIT_INST_LDS"] / (waves * cus * cyc) if cyc and waves else None)
    return out


def sq_summary(pmc_dir: str, command: str) -> str:
    t = sq_table(pmc_dir)
    out = ["# SQ counters per kernel (rocprofv3 --pmc)", "", "Command:", "", "```", command, "```", "",
           "Counter sums over each kernel's dispatches in the run.  Shares of the kernel's time",
           "(its dispatch durations, 256 CUs at 2.4 GHz): conflict = SQ_LDS_BANK_CONFLICT /",
           "(256 x cycles), the part of each CU's time its LDS spent on bank conflicts; VALU =",
           "4 x SQ_INSTS_VALU / (256 x 4 SIMDs x cycles), SIMD time issuing vector instructions",
           "(a wave64 instruction holds its 16-lane SIMD for 4 cycles); LDS wait =",
           "SQ_WAIT_INST_LDS / (resident waves per CU x 256 x cycles), for kernels whose",
           "resident waves are fixed by their shape (16 per CU; 32 for the permutation).", "",
           "| kernel | dispatches | ms | VALU insts | LDS insts | LDS bank-conflict cycles | "
           "LDS-wait wave-cycles | conflict | VALU | LDS wait |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for k, v in sorted(t.items(), key=lambda kv: -kv[1]["ms"]):
        lw = "–" if v["ldswait"] is None else f"{100 * v['ldswait']:.1f} %"
        out.append(f"| `{k}` | {v['dispatches']} | {v['ms']:.2f} | {v['SQ_INSTS_VALU']:.3g} | "
                   f"{v['SQ_INSTS_LDS']:.3g} | {v['SQ_LDS_BANK_CONFLICT']:.3g} | {v['SQ_WAIT_INST_LDS']:.3g} | "
                   f"{100 * v['conflict']:.1f} % | {100 * v['valu']:.1f} % | {lw} |")
    return "\n".join(out) + "\n"


def traffic(fetch_dir: str, write_dir: str, copy_bytes: int):
    """Calibrated HBM bytes of every library kernel kind over the run.  Each
    counter is summed per kind over its own run; the two runs may differ by
    a small extra recursion level (the sample of a level is random), which
    `same_dispatches` records."""
    fetch = _counter(fetch_dir, "FETCH_SIZE")
    write = _counter(write_dir, "WRITE_SIZE")
    cf = max(v for n, v in fetch if n.startswith(COPY)) * 1024.0
    cw = max(v for n, v in write if n.startswith(COPY)) * 1024.0
    sf, sw = copy_bytes / cf, copy_bytes / cw
    same = [n for n, _ in fetch] == [n for n, _ in write]
    acc = {}
    for runs, field in ((fetch, "fetch_kib"), (write, "write_kib")):
        for name, v in runs:
            kind = kind_of(name)
            if kind is None:
                continue
            a = acc.setdefault(kind, {"launches": 0, "fetch_kib": 0.0, "write_kib": 0.0})
            a[field] += v
            if field == "fetch_kib":
                a["launches"] += 1
    for a in acc.values():
        a["hbm_bytes"] = (a["fetch_kib"] * sf + a["write_kib"] * sw) * 1024.0
        a["same_dispatches"] = same
    return acc, sf, sw


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("trace_dir")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    q = sub.add_parser("sq")
    q.add_argument("pmc_dir")
    q.add_argument("out")
    q.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("out_dir")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--command", required=True)
    a = ap.parse_args(argv)
    if a.what == "stats":
        with open(a.out, "w") as f:
            f.write(stats_summary(a.trace_dir, a.command))
        return 0
    if a.what == "sq":
        with open(a.out, "w") as f:
            f.write(sq_summary(a.pmc_dir, a.command))
        return 0
    acc, sf, sw = traffic(a.fetch_dir, a.write_dir, a.copy_bytes)
    sha = source_sha()
    for kind, rec in acc.items():
        rec.update({"kernel": kind, "source_sha": sha, "scale_fetch": sf, "scale_write": sw,
                    "copy_bytes": a.copy_bytes, "command": a.command})
        with open(os.path.join(a.out_dir, f"traffic_{kind}.json"), "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
    print(json.dumps({k: round(v["hbm_bytes"] / 1e9, 3) for k, v in acc.items()}), file=sys.stderr)
    return 0


if __name__ == "__main__":
    sys.exit(main())
