"""Summaries of rocprofv3 databases (kernel trace and PMC counter runs).

Usage (on the rocprofv3 output of the commands quoted in each summary):

  python -m paper_2310_14712_amd.profiling trace <results.db> <out.md> --cmd "<command>"
  python -m paper_2310_14712_amd.profiling traffic <fetch.db> <write.db> <bench.json> <out.json> \
      --kernel explicit2d_kernel --copy-bytes N --cmd "<commands>"
  python -m paper_2310_14712_amd.profiling counters <out.md> <pmc.db> [<pmc.db> ...] \
      --kernel explicit3d_kron --cmd "<commands>"

`trace` writes the per-kernel statistics (calls, total / mean / min / max
duration).  `traffic` turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of
one kernel into bytes per launch, scaled by what the same counters read for a
plain device-to-device copy of known size (--copy-bytes read and written),
and records the SHA-256 of the kernel source they were taken on, so that a
reader can tell when the figures no longer describe the kernel.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")


def kernel_source_sha256() -> str:
    """SHA-256 over the device sources (every .hip and .h file of csrc, in
    name order): a counter summary describes the kernels only while it
    matches."""
    h = hashlib.sha256()
    for fn in sorted(os.listdir(CSRC)):
        if fn.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, fn), "rb") as f:
                h.update(fn.encode() + b"\0" + f.read())
    return h.hexdigest()


def kernel_stats(db):
    """Per launch shape (kernel, grid size, LDS bytes): calls and durations.
    One kernel launched with several shapes (the candidate tiles of an
    autotuner, or another mesh) gives one row per shape."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select name, grid_x * grid_y * grid_z, lds_size, count(*), sum(end - start), avg(end - start), "
        "min(end - start), max(end - start) from kernels group by name, grid_x * grid_y * grid_z, lds_size "
        "order by count(*) desc, sum(end - start) desc").fetchall()
    con.close()
    return [{"kernel": r[0], "grid": r[1], "lds": r[2], "calls": r[3], "total_us": r[4] / 1e3,
             "mean_us": r[5] / 1e3, "min_us": r[6] / 1e3, "max_us": r[7] / 1e3} for r in rows]


def counter_means(db, counter):
    """Mean value of one counter per dispatch, by launch shape (kernel name,
    grid size, LDS bytes), with the number of dispatches."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select kernel_name, grid_size, lds_block_size, count(distinct dispatch_id), sum(value) "
        "from counters_collection where counter_name = ? group by kernel_name, grid_size, lds_block_size",
        (counter,)).fetchall()
    con.close()
    return {(r[0], r[1], r[2]): (r[4] / max(r[3], 1), r[3]) for r in rows}


def counter_max_dispatch(db, counter, exclude):
    """(kernel, value) of the single dispatch with the largest counter value
    among kernels whose name does not contain `exclude`."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select kernel_name, dispatch_id, sum(value) from counters_collection where counter_name = ? "
        "group by dispatch_id order by sum(value) desc", (counter,)).fetchall()
    con.close()
    for name, _, v in rows:
        if exclude not in name:
            return name, v
    raise KeyError(f"no dispatch outside {exclude!r}")


def _pick(db, counter, key):
    """The launch shape (kernel, grid, LDS bytes) of the last dispatch of a
    kernel matching `key`: the bench times the chosen shape after the
    autotuner has tried every candidate."""
    con = sqlite3.connect(db)
    row = con.execute(
        "select kernel_name, grid_size, lds_block_size from counters_collection "
        "where counter_name = ? and kernel_name like ? order by dispatch_id desc limit 1",
        (counter, f"%{key}%")).fetchone()
    con.close()
    if row is None:
        raise KeyError(f"no kernel matching {key!r}")
    return tuple(row)


def trace_summary(db, out, cmd, exclude=()):
    """Markdown table of kernel_stats; kernels whose name contains one of
    `exclude` (e.g. setup-only kernels) are left out."""
    st = [s for s in kernel_stats(db) if not any(x in s["kernel"] for x in exclude)]
    lines = ["# Kernel trace summary", "", "Command:", "", "```", cmd, "```", "",
             *([f"Left out: kernels whose name contains {', '.join(map(repr, exclude))}.", ""] if exclude else []),
             "One row per launch shape (kernel, grid size in work-items, LDS bytes); the explicit",
             "kernel's autotuner candidates appear as rows of their own with few calls.  Sorted by",
             "calls: the kernels of the timed steps come first.", "",
             "| kernel | grid | LDS | calls | total (us) | mean (us) | min (us) | max (us) |",
             "|---|---|---|---|---|---|---|---|"]
    for s in st:
        lines.append(f"| `{s['kernel']}` | {s['grid']} | {s['lds']} | {s['calls']} | {s['total_us']:.1f} | "
                     f"{s['mean_us']:.3f} | {s['min_us']:.3f} | {s['max_us']:.3f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return st


def traffic_summary(fetch_db, write_db, bench_json, out, kernel, copy_bytes, cmd, key="explicit"):
    fetch = counter_means(fetch_db, "FETCH_SIZE")
    write = counter_means(write_db, "WRITE_SIZE")
    kf, kw = _pick(fetch_db, "FETCH_SIZE", kernel), _pick(write_db, "WRITE_SIZE", kernel)
    if kf != kw:
        raise ValueError(f"the two passes timed different launch shapes: {kf} and {kw}")
    # the calibration copy: the largest single dispatch that is not one of ours
    cf, cfv = counter_max_dispatch(fetch_db, "FETCH_SIZE", "imex")
    cw, cwv = counter_max_dispatch(write_db, "WRITE_SIZE", "imex")
    f_scale = (copy_bytes / 1024.0) / cfv
    w_scale = (copy_bytes / 1024.0) / cwv
    with open(bench_json) as f:
        line = [json.loads(x) for x in f if x.strip().startswith("{")][-1]
    res = {
        "kernel": kf[0], "grid": kf[1], "lds": kf[2], "dispatches": fetch[kf][1],
        "fetch_kib_per_dispatch": fetch[kf][0], "write_kib_per_dispatch": write[kw][0],
        "copy_kernel": cf, "copy_bytes": copy_bytes,
        "copy_fetch_kib": cfv, "copy_write_kib": cwv,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "traffic_bytes_per_launch": 1024.0 * (fetch[kf][0] * f_scale + write[kw][0] * w_scale),
        "kernel_key": key,
        "algorithmic_bytes_per_launch": line["roofline"].get("kernels_bytes", {}).get(
            key, line["roofline"]["bytes_per_launch"]),
        "kernels_sha256": kernel_source_sha256(),
        "workload": line["config"]["workload"],
        "command": cmd,
    }
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    return res


def counters_summary(dbs, out, kernel, cmd):
    """Markdown table of the mean per dispatch of every counter in the PMC
    databases for the launch shapes of kernels whose name contains
    `kernel` (one database per counter pass)."""
    rows = {}
    for db in dbs:
        con = sqlite3.connect(db)
        for name, grid, lds, counter, n, total in con.execute(
                "select kernel_name, grid_size, lds_block_size, counter_name, count(distinct dispatch_id), "
                "sum(value) from counters_collection where kernel_name like ? "
                "group by kernel_name, grid_size, lds_block_size, counter_name", (f"%{kernel}%",)):
            rows.setdefault((name, grid, lds), {})[counter] = (total / max(n, 1), n)
        con.close()
    lines = ["# Hardware counters", "", "Commands (one counter pass each):", "", "```", cmd, "```", "",
             "Mean value per dispatch, summed over the device, per launch shape (kernel, grid size",
             "in work-items, LDS bytes).", ""]
    for (name, grid, lds), cs in sorted(rows.items(), key=lambda kv: -max(v[1] for v in kv[1].values())):
        lines += [f"## `{name}` grid {grid}, LDS {lds}", "", "| counter | mean per dispatch | dispatches |",
                  "|---|---|---|"]
        for c in sorted(cs):
            lines.append(f"| {c} | {cs[c][0]:.6g} | {cs[c][1]} |")
        lines.append("")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return rows


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("out")
    t.add_argument("--cmd", required=True)
    t.add_argument("--exclude", action="append", default=[], help="leave out kernels containing this text")
    r = sub.add_parser("traffic")
    r.add_argument("fetch_db")
    r.add_argument("write_db")
    r.add_argument("bench_json")
    r.add_argument("out")
    r.add_argument("--kernel", required=True)
    r.add_argument("--copy-bytes", type=int, required=True)
    r.add_argument("--cmd", required=True)
    r.add_argument("--key", default="explicit", help="the bench's name of the kernel (explicit, rhs)")
    q = sub.add_parser("counters")
    q.add_argument("out")
    q.add_argument("dbs", nargs="+")
    q.add_argument("--kernel", required=True)
    q.add_argument("--cmd", required=True)
    a = ap.parse_args()
    if a.what == "counters":
        counters_summary(a.dbs, a.out, a.kernel, a.cmd)
        return
    if a.what == "trace":
        for s in trace_summary(a.db, a.out, a.cmd, tuple(a.exclude))[:8]:
            print(s)
    else:
        print(json.dumps(traffic_summary(a.fetch_db, a.write_db, a.bench_json, a.out, a.kernel,
                                         a.copy_bytes, a.cmd, a.key), indent=1))


if __name__ == "__main__":
    main()
