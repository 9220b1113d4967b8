"""Text summaries of rocprofv3 results, and the HBM-traffic record the
benchmark reads.

rocprofv3 writes an SQLite results database (``*_results.db``) per run.
Two summaries are made from them:

  kernels  per-kernel call count, total and average duration (the
           ``--kernel-trace --stats`` view), for the top kernels of a run;
  counters per-dispatch averages of any counters for chosen kernels, with the
           matrix-core busy fraction when its counters are present;
  traffic  HBM bytes per dispatch of one kernel from two counter runs
           (FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch), each scaled by
           what the same counter reads for a device copy of known size.

    python -m paper_2505_21404_amd.profiling kernels DIR --cmd "..." --out FILE
    python -m paper_2505_21404_amd.profiling counters DIR --kernels NAME... --cmd "..." --out FILE
    python -m paper_2505_21404_amd.profiling traffic --kernel NAME --source FILE \
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \
        --copy-bytes B --cmd "..." --out FILE

The traffic record carries the SHA-256 of the kernel's source file; a
reader treats it as stale once the source has changed.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import os
import sqlite3
from typing import Dict, List, Optional, Tuple


def _db(path: str) -> str:
    if os.path.isfile(path):
        return path
    hits = sorted(glob.glob(os.path.join(path, "**", "*results.db"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no rocprofv3 results database under {path}")
    return hits[0]


def short_name(name: str) -> str:
    n = name.replace("dngd::(anonymous namespace)::", "").replace("dngd::", "")
    return n.split("(")[0]


def top_kernels(path: str, limit: int = 25) -> List[Tuple[str, int, float, float, float]]:
    """(name, calls, total_us, avg_us, percent) from the stats view (which
    holds microseconds; the per-dispatch tables hold nanoseconds)."""
    con = sqlite3.connect(_db(path))
    rows = con.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels order by total_duration desc limit ?", (limit,)).fetchall()
    con.close()
    return [(short_name(r[0]), int(r[1]), float(r[2]), float(r[3]), float(r[4])) for r in rows]


def counter_avg(path: str, kernel_substr: str, counter: str) -> Tuple[float, int, float]:
    """Average counter value per dispatch of the kernels whose name contains
    ``kernel_substr``: (value, dispatches, average duration in us)."""
    con = sqlite3.connect(_db(path))
    rows = con.execute("select kernel_name, value, duration from counters_collection "
                       "where counter_name = ?", (counter,)).fetchall()
    con.close()
    vals = [(v, d) for k, v, d in rows if kernel_substr in k]
    if not vals:
        raise KeyError(f"no {counter} records for a kernel matching {kernel_substr!r}")
    return (sum(v for v, _ in vals) / len(vals), len(vals),
            sum(d for _, d in vals) / len(vals) / 1e3)


def sha256_file(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def kernels_summary(path: str, cmd: str, title: str, limit: int = 25) -> str:
    lines = [f"# {title}", "", "command:", f"  {cmd}", "",
             f"{'kernel':60s} {'calls':>6s} {'total_us':>11s} {'avg_us':>10s} {'pct':>6s}"]
    for name, calls, tot, avg, pct in top_kernels(path, limit):
        lines.append(f"{name[:60]:60s} {calls:6d} {tot:11.1f} {avg:10.2f} {pct:6.2f}")
    return "\n".join(lines) + "\n"


def traffic_summary(kernel: str, source: str, fetch: str, write: str, copy_fetch: str,
                    copy_write: str, copy_bytes: int, cmd: str, title: str,
                    copy_kernel: str = "", extra: Optional[Dict[str, str]] = None) -> str:
    f_kib, f_n, f_us = counter_avg(fetch, kernel, "FETCH_SIZE")
    w_kib, w_n, w_us = counter_avg(write, kernel, "WRITE_SIZE")
    cf_kib, cf_n, _ = counter_avg(copy_fetch, copy_kernel, "FETCH_SIZE")
    cw_kib, cw_n, _ = counter_avg(copy_write, copy_kernel, "WRITE_SIZE")
    f_scale = copy_bytes / (cf_kib * 1024.0)
    w_scale = copy_bytes / (cw_kib * 1024.0)
    fetch_b = f_kib * 1024.0 * f_scale
    write_b = w_kib * 1024.0 * w_scale
    rec = {
        "kernel": kernel,
        "source": os.path.relpath(source, os.path.dirname(os.path.dirname(os.path.abspath(__file__)))),
        "source_sha256": sha256_file(source),
        "fetch_kib_per_dispatch": f"{f_kib:.1f}",
        "fetch_dispatches": f_n,
        "write_kib_per_dispatch": f"{w_kib:.1f}",
        "write_dispatches": w_n,
        "copy_kernel": copy_kernel,
        "copy_bytes_per_launch": copy_bytes,
        "copy_fetch_kib_per_launch": f"{cf_kib:.1f}",
        "copy_write_kib_per_launch": f"{cw_kib:.1f}",
        "fetch_scale": f"{f_scale:.4f}",
        "write_scale": f"{w_scale:.4f}",
        "fetch_bytes_per_dispatch": f"{fetch_b:.6e}",
        "write_bytes_per_dispatch": f"{write_b:.6e}",
        "traffic_bytes_per_dispatch": f"{fetch_b + write_b:.6e}",
        "avg_dispatch_us_under_counters": f"{(f_us + w_us) / 2:.1f}",
    }
    rec.update(extra or {})
    lines = [f"# {title}", "", "commands:"] + [f"  {c}" for c in cmd.split(" ;; ")] + [""]
    lines += [f"{k}: {v}" for k, v in rec.items()]
    return "\n".join(lines) + "\n"


def counters_summary(path: str, kernels: List[str], cmd: str, title: str, simds: int = 1024,
                     xcds: int = 8) -> str:
    """Per-dispatch averages of every counter in a ``--pmc`` run for the
    kernels whose short names contain one of ``kernels``. With
    SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE present, also the matrix-core
    busy fraction: busy cycles summed over the ``simds`` SIMDs, divided by
    ``simds`` times the active cycles of one XCD (GRBM_GUI_ACTIVE summed over
    the ``xcds`` XCDs, divided by ``xcds``)."""
    con = sqlite3.connect(_db(path))
    rows = con.execute("select kernel_name, counter_name, value, duration from counters_collection"
                       ).fetchall()
    con.close()
    agg: Dict[str, Dict[str, List[float]]] = {}
    for k, c, v, d in rows:
        n = short_name(k).replace("void ", "")
        if not any(q in n for q in kernels):
            continue
        a = agg.setdefault(n, {})
        a.setdefault(c, []).append(float(v))
        a.setdefault("duration_ns", []).append(float(d))
    lines = [f"# {title}", "", "command:", f"  {cmd}", ""]
    for n in sorted(agg, key=lambda x: -sum(agg[x]["duration_ns"])):
        a = agg[n]
        nd = len(a["duration_ns"])
        avg = {c: sum(v) / len(v) for c, v in a.items()}
        lines.append(f"kernel: {n}")
        lines.append(f"  counter samples: {nd}, avg duration under counters: "
                     f"{avg['duration_ns'] / 1e3:.1f} us")
        for c in sorted(avg):
            if c != "duration_ns":
                lines.append(f"  {c}: {avg[c]:.6g}")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in avg and avg.get("GRBM_GUI_ACTIVE", 0) > 0:
            frac = avg["SQ_VALU_MFMA_BUSY_CYCLES"] / (simds * avg["GRBM_GUI_ACTIVE"] / xcds)
            lines.append(f"  mfma_busy_frac: {frac:.3f}")
        lines.append("")
    return "\n".join(lines)


def read_traffic(path: str, repo_root: str) -> Optional[Dict[str, str]]:
    """The traffic record at ``path`` if its kernel source is unchanged,
    else None."""
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ": " in line and not line.startswith(" "):
                k, v = line.rstrip("\n").split(": ", 1)
                rec[k] = v
    src = os.path.join(repo_root, rec.get("source", ""))
    if not os.path.isfile(src) or sha256_file(src) != rec.get("source_sha256"):
        return None
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("dir")
    k.add_argument("--cmd", required=True)
    k.add_argument("--title", default="rocprofv3 --kernel-trace --stats")
    k.add_argument("--limit", type=int, default=25)
    k.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("--kernels", nargs="+", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--title", default="rocprofv3 --pmc counters per dispatch")
    c.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    for a in ("--kernel", "--source", "--fetch", "--write", "--copy-fetch", "--copy-write",
              "--cmd", "--out"):
        t.add_argument(a, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    # the calibration run also launches torch's fill of the source tensor,
    # which fetches nothing: average over the copy kernel's dispatches only
    t.add_argument("--copy-kernel", default="__amd_rocclr_copyBuffer")
    t.add_argument("--title", default="HBM traffic per dispatch (rocprofv3 --pmc)")
    t.add_argument("--extra", nargs="*", default=[], help="key=value pairs to record")
    a = ap.parse_args(argv)
    if a.what == "kernels":
        text = kernels_summary(a.dir, a.cmd, a.title, a.limit)
    elif a.what == "counters":
        text = counters_summary(a.dir, a.kernels, a.cmd, a.title)
    else:
        text = traffic_summary(a.kernel, a.source, a.fetch, a.write, a.copy_fetch, a.copy_write,
                               a.copy_bytes, a.cmd, a.title, a.copy_kernel,
                               dict(kv.split("=", 1) for kv in a.extra))
    with open(a.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
