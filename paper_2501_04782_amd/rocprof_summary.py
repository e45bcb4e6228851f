"""Turn rocprofv3 result databases (rocpd SQLite) into short markdown summaries.

Two summaries are produced:

* ``stats``: per-kernel dispatch count, average and total duration from a
  ``--kernel-trace`` run;
* ``traffic``: HBM bytes per dispatch of one kernel from two ``--pmc`` runs
  (``FETCH_SIZE``, then ``WRITE_SIZE``; KiB per dispatch), each scaled by the
  ratio between the known size and the counter's reading for a plain copy
  kernel profiled the same way.  The summary carries a hash of the kernel's
  sources and the tuning it was taken with, so that a reader can tell when
  the figures no longer describe the code.

* ``kernel-counters``: the SQ counters per dispatch of one kernel from one or
  more ``--pmc`` runs and its average duration from a kernel trace, with the
  same source hash and tuning key, for bench.py to read back.

Usage (from the repository root):
  python3 -m paper_2501_04782_amd.rocprof_summary stats DB --title T --command C
  python3 -m paper_2501_04782_amd.rocprof_summary kernel-counters --kernel K DB [DB ...] --trace T \
      --stage S --workload W --tuning KEY --command C
  python3 -m paper_2501_04782_amd.rocprof_summary traffic --kernel K --fetch-db A --write-db B \
      --copy-fetch-db C --copy-write-db D --copy-bytes N --stage S --workload W --tuning b,c,m --command C
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sqlite3
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))

# sources whose change invalidates a kernel's counter figures
STAGE_SOURCES = {
    "composite_fwd": ("csrc/composite.hip", "csrc/gv_internal.h"),
    "composite_bwd": ("csrc/composite.hip", "csrc/gv_internal.h"),
    "project": ("csrc/project.hip", "csrc/gv_internal.h"),
    "scatter": ("csrc/project.hip", "csrc/gv_internal.h"),
    "sort": ("csrc/sort.hip", "csrc/gv_internal.h"),
    "project_bwd": ("csrc/project_bwd.hip", "csrc/gv_internal.h"),
}


def source_hash(stage: str) -> str:
    h = hashlib.sha256()
    for rel in STAGE_SOURCES[stage]:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_durations(db: str):
    """{kernel name: [duration ns, ...]} of every dispatch in the trace."""
    con = sqlite3.connect(db)
    out = defaultdict(list)
    for name, dur in con.execute("select name, duration from kernels"):
        out[name].append(dur)
    return out


def counter_per_dispatch(db: str, counter: str, kernel_substr: str):
    """Values of `counter` for each dispatch of kernels whose name contains
    `kernel_substr` (rows of one dispatch are summed)."""
    con = sqlite3.connect(db)
    per = defaultdict(float)
    for did, name, val in con.execute(
            "select dispatch_id, kernel_name, value from counters_collection where counter_name = ?", (counter,)):
        if kernel_substr in name:
            per[did] += val
    return [per[k] for k in sorted(per)]


def cmd_stats(a):
    d = kernel_durations(a.db)
    total = sum(sum(v) for v in d.values())
    rows = sorted(d.items(), key=lambda kv: -sum(kv[1]))
    print(f"# {a.title}\n")
    print("Command (from the repository root on the MI355X machine):\n")
    print("```\n" + a.command + "\n```\n")
    print("| kernel | calls | avg (ms) | total (ms) | % of GPU time |")
    print("|---|---|---|---|---|")
    for name, v in rows:
        pct = 100.0 * sum(v) / total
        if pct < 0.05:
            continue
        n = name.replace("|", "/")
        if len(n) > 90:
            n = n[:87] + "..."
        print(f"| `{n}` | {len(v)} | {sum(v) / len(v) / 1e6:.4f} | {sum(v) / 1e6:.2f} | {pct:.2f} |")


def cmd_traffic(a):
    fetch = counter_per_dispatch(a.fetch_db, "FETCH_SIZE", a.kernel)
    write = counter_per_dispatch(a.write_db, "WRITE_SIZE", a.kernel)
    cfetch = counter_per_dispatch(a.copy_fetch_db, "FETCH_SIZE", a.copy_kernel)
    cwrite = counter_per_dispatch(a.copy_write_db, "WRITE_SIZE", a.copy_kernel)
    if not (fetch and write and cfetch and cwrite):
        raise SystemExit(f"missing dispatches: fetch {len(fetch)} write {len(write)} copy {len(cfetch)}/{len(cwrite)}")
    kib = a.copy_bytes / 1024.0
    f_fac = kib / (sum(cfetch) / len(cfetch))
    w_fac = kib / (sum(cwrite) / len(cwrite))
    f_kib = sum(fetch) / len(fetch)
    w_kib = sum(write) / len(write)
    traffic = (f_kib * f_fac + w_kib * w_fac) * 1024.0
    print(f"# HBM traffic of `{a.kernel}` ({a.stage}), workload {a.workload}\n")
    print("Commands (from the repository root on the MI355X machine, after `cd /tmp && export TMPDIR=/tmp`, "
          "R = repository root):\n")
    print("```\n" + a.command + "\n```\n")
    print("| quantity | value |")
    print("|---|---|")
    print(f"| dispatches (fetch / write runs) | {len(fetch)} / {len(write)} |")
    print(f"| FETCH_SIZE per dispatch (KiB) | {f_kib:.1f} |")
    print(f"| WRITE_SIZE per dispatch (KiB) | {w_kib:.1f} |")
    print(f"| copy kernel: bytes moved each way | {a.copy_bytes} |")
    print(f"| copy kernel: FETCH_SIZE / WRITE_SIZE (KiB) | {sum(cfetch) / len(cfetch):.1f} / "
          f"{sum(cwrite) / len(cwrite):.1f} |")
    print(f"| scale factors (fetch, write) | {f_fac:.4f}, {w_fac:.4f} |")
    print(f"| HBM bytes per dispatch (scaled) | {traffic:.4e} |")
    print()
    print("Machine-readable (read by bench.py; ignored when the source hash or tuning differ):\n")
    print("```")
    print(f"stage: {a.stage}")
    print(f"workload: {a.workload}")
    print(f"tuning: {a.tuning}")
    print(f"source_sha256: {source_hash(a.stage)}")
    print(f"traffic_bytes_per_launch: {traffic:.6e}")
    print("```")


def stage_key(stage: str, tuning: dict) -> str:
    """The part of the tuning that changes a stage's kernel (file-name safe)."""
    c = tuning['compact']
    if stage == "composite_fwd":
        return f"b{tuning['batch']}-" + ("compact" if c & 1 else "tile" if c & 32 else "quad" if c & 4
                                         else "block")
    if stage == "composite_bwd":
        return f"b{tuning['bwd_batch']}-" + ("compact" if c & 2 else "tile" if c & 16 else "pair" if c & 8
                                             else "quad")
    if stage == "sort":
        return f"cap{tuning['sort_cap']}"
    return "any"


def read_traffic(path: str, stage: str, workload: str, tuning: str):
    """Scaled HBM bytes per launch from a traffic summary, or None when the
    file is absent or was taken from other sources, tuning or workload."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ": " in line and not line.startswith("|"):
                k, v = line.strip().split(": ", 1)
                kv[k] = v
    try:
        ok = (kv["stage"] == stage and kv["workload"] == workload and kv["tuning"] == tuning
              and kv["source_sha256"] == source_hash(stage))
        return float(kv["traffic_bytes_per_launch"]) if ok else None
    except (KeyError, ValueError):
        return None


def read_counters(path: str, stage: str, workload: str, tuning: str):
    """{counter: value per dispatch, avg_ms} from a kernel-counters summary, or
    None when absent or taken from other sources, tuning or workload."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ": " in line and not line.startswith("|"):
                k, v = line.strip().split(": ", 1)
                kv[k] = v
    try:
        if not (kv["stage"] == stage and kv["workload"] == workload and kv["tuning"] == tuning
                and kv["source_sha256"] == source_hash(stage)):
            return None
        out = {k: float(v) for k, v in kv.items() if k.startswith(("SQ_", "GRBM_"))}
        out["avg_ms"] = float(kv["avg_ms"])
        return out
    except (KeyError, ValueError):
        return None


def cmd_kernel_counters(a):
    merged = {}
    for db in a.dbs:
        for k, d in counters_per_kernel(db).items():
            if a.kernel in k:
                merged.update(d)
    durs = [v for k, vs in kernel_durations(a.trace).items() if a.kernel in k for v in vs]
    if not merged or not durs:
        raise SystemExit(f"no dispatches of {a.kernel}")
    ms = sum(durs) / len(durs) / 1e6
    print(f"# SQ counters of `{a.kernel}` ({a.stage}), workload {a.workload}\n")
    print("Commands (from the repository root on the MI355X machine, after `cd /tmp && export TMPDIR=/tmp`, "
          "R = repository root):\n")
    print("```\n" + a.command + "\n```\n")
    print("| counter | per dispatch |")
    print("|---|---|")
    for c in sorted(merged):
        print(f"| {c} | {merged[c]:.6g} |")
    print(f"| kernel time (ms, trace average over {len(durs)} dispatches) | {ms:.4f} |")
    print()
    print("Machine-readable (read by bench.py; ignored when the source hash or tuning differ):\n")
    print("```")
    print(f"stage: {a.stage}")
    print(f"workload: {a.workload}")
    print(f"tuning: {a.tuning}")
    print(f"source_sha256: {source_hash(a.stage)}")
    print(f"avg_ms: {ms:.6f}")
    for c in sorted(merged):
        print(f"{c}: {merged[c]:.6e}")
    print("```")


def counters_per_kernel(db: str):
    """{kernel: {counter: mean per dispatch}} of a --pmc run."""
    con = sqlite3.connect(db)
    per = defaultdict(lambda: defaultdict(float))
    for did, name, cname, val in con.execute(
            "select dispatch_id, kernel_name, counter_name, value from counters_collection"):
        per[name][(cname, did)] += val
    out = {}
    for name, d in per.items():
        by = defaultdict(list)
        for (cname, _), v in d.items():
            by[cname].append(v)
        out[name] = {c: sum(v) / len(v) for c, v in by.items()}
    return out


def cmd_counters(a):
    """Per-kernel SQ counter means (per dispatch) of one or more --pmc runs,
    with the derived VALU issue share (instructions x 4 cycles over the
    SIMD-cycles of the kernel's duration) when a kernel trace is given."""
    merged = defaultdict(dict)
    for db in a.dbs:
        for k, d in counters_per_kernel(db).items():
            merged[k].update(d)
    dur = {k: sum(v) / len(v) for k, v in kernel_durations(a.trace).items()} if a.trace else {}
    cols = sorted({c for d in merged.values() for c in d})
    print(f"# {a.title}\n")
    print("Commands (from the repository root on the MI355X machine):\n")
    print("```\n" + a.command + "\n```\n")
    print("Means per dispatch.  VALU share = SQ_INSTS_VALU x 4 cycles / (kernel time x 2.4 GHz x 1024 SIMDs).\n")
    print("| kernel | " + " | ".join(cols) + (" | avg ms | VALU share |" if dur else " |"))
    print("|---|" + "---|" * len(cols) + ("---|---|" if dur else ""))
    for k in sorted(merged, key=lambda n: -merged[n].get("SQ_INSTS_VALU", 0.0)):
        d = merged[k]
        if d.get("SQ_WAVES", 1.0) < 100:
            continue
        n = k.split("(")[0].replace("|", "/")
        row = f"| `{n}` | " + " | ".join(f"{d.get(c, 0.0):.3g}" for c in cols)
        if dur:
            t = dur.get(k)
            share = d.get("SQ_INSTS_VALU", 0.0) * 4 / (t * 1e-9 * 2.4e9 * 1024) if t else float("nan")
            row += f" | {t / 1e6:.4f} | {share:.2f} |" if t else " | - | - |"
        else:
            row += " |"
        print(row)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True, help="substring of the kernel name")
    t.add_argument("--copy-kernel", default="copy", help="substring of the copy kernel's name")
    t.add_argument("--fetch-db", required=True)
    t.add_argument("--write-db", required=True)
    t.add_argument("--copy-fetch-db", required=True)
    t.add_argument("--copy-write-db", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--stage", required=True, choices=sorted(STAGE_SOURCES))
    t.add_argument("--workload", required=True)
    t.add_argument("--tuning", required=True, help="the stage key (stage_key) the counters were taken with")
    t.add_argument("--command", required=True)
    c = sub.add_parser("counters")
    c.add_argument("dbs", nargs="+")
    c.add_argument("--trace", help="kernel-trace results db of the same workload (durations)")
    c.add_argument("--title", required=True)
    c.add_argument("--command", required=True)
    k = sub.add_parser("kernel-counters")
    k.add_argument("dbs", nargs="+")
    k.add_argument("--kernel", required=True, help="substring of the kernel name")
    k.add_argument("--trace", required=True, help="kernel-trace results db of the same command")
    k.add_argument("--stage", required=True, choices=sorted(STAGE_SOURCES))
    k.add_argument("--workload", required=True)
    k.add_argument("--tuning", required=True)
    k.add_argument("--command", required=True)
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic, "counters": cmd_counters,
     "kernel-counters": cmd_kernel_counters}[a.cmd](a)


if __name__ == "__main__":
    main()
