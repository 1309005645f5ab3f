"""Per-kernel statistics of a rocprofv3 kernel trace (its SQLite results
database) as the markdown table of the profile summaries.

Usage:
  python -m paper_1607_04572_amd.trace_summary <run_results.db> [rows]        kernel trace
  python -m paper_1607_04572_amd.trace_summary --sq <run_results.db>          SQ counter pass
  python -m paper_1607_04572_amd.trace_summary --hbm <fetch.db> <write.db> <trace.db> <copy MiB>
                                                                              HBM bytes per kernel
"""
from __future__ import annotations

import sqlite3
import sys


def stats(db: str) -> list:
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), avg(duration), min(duration), max(duration), sum(duration) "
                     "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[5] for r in rows) or 1
    return [dict(name=r[0], calls=r[1], avg_us=r[2] / 1e3, min_us=r[3] / 1e3, max_us=r[4] / 1e3,
                 total_ms=r[5] / 1e6, pct=100.0 * r[5] / total) for r in rows]


def markdown(db: str, limit: int = 30) -> str:
    out = ["| kernel | calls | avg us | min us | max us | total ms | % |", "|---|---:|---:|---:|---:|---:|---:|"]
    for r in stats(db)[:limit]:
        name = r["name"] if len(r["name"]) <= 80 else r["name"][:77] + "..."
        out.append(f"| `{name}` | {r['calls']} | {r['avg_us']:.1f} | {r['min_us']:.1f} | {r['max_us']:.1f} | "
                   f"{r['total_ms']:.2f} | {r['pct']:.1f} |")
    return "\n".join(out)


def _short(name: str) -> str:
    """Kernel name without its argument list."""
    return name.split("(")[0].replace("void ", "")


def _per_dispatch(db: str) -> dict:
    """{kernel: {counter: mean over dispatches of the value summed over a dispatch's instances}}."""
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, dispatch_id, counter_name, sum(value) from counters_collection "
                     "group by kernel_name, dispatch_id, counter_name").fetchall()
    acc: dict = {}
    for k, _, n, v in rows:
        acc.setdefault(_short(k), {}).setdefault(n, []).append(v)
    return {k: {n: sum(v) / len(v) for n, v in d.items()} for k, d in acc.items()}


def sq_markdown(db: str) -> str:
    """Instruction counters per wave (SQ_INSTS_* / SQ_WAVES) and the cycle counters per dispatch."""
    out = ["| kernel | waves | VALU/wave | SALU/wave | LDS/wave | VMEM rd/wave | LDS bank conflict cycles | "
           "LDS wait cycles |", "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for k, d in sorted(_per_dispatch(db).items()):
        w = d.get("SQ_WAVES", 0.0)
        if w <= 0:
            continue
        out.append(f"| `{k}` | {w:.0f} | {d.get('SQ_INSTS_VALU', 0) / w:.0f} | {d.get('SQ_INSTS_SALU', 0) / w:.0f} | "
                   f"{d.get('SQ_INSTS_LDS', 0) / w:.0f} | {d.get('SQ_INSTS_VMEM_RD', 0) / w:.1f} | "
                   f"{d.get('SQ_LDS_BANK_CONFLICT', 0):.3g} | {d.get('SQ_WAIT_INST_LDS', 0):.3g} |")
    return "\n".join(out)


def hbm_markdown(fetch_db: str, write_db: str, trace_db: str, copy_mib: int) -> str:
    """HBM bytes per dispatch of every kernel: FETCH_SIZE and WRITE_SIZE (KiB) scaled by what they read
    for the copy kernel of copy_mib MiB read and written, with the mean durations of a kernel trace."""
    f, w = _per_dispatch(fetch_db), _per_dispatch(write_db)
    copy = [k for k in f if "k_copy16" in k][0]
    fs = copy_mib * 1024.0 / f[copy]["FETCH_SIZE"]
    ws = copy_mib * 1024.0 / w[copy]["WRITE_SIZE"]
    dur = {_short(r["name"]): r["avg_us"] for r in stats(trace_db)}
    rows = []
    for k in f:
        if k not in w or k not in dur or "copy" in k:
            continue
        rd = f[k]["FETCH_SIZE"] * fs * 1024.0
        wr = w[k]["WRITE_SIZE"] * ws * 1024.0
        rows.append((rd + wr, k, rd, wr, dur[k]))
    out = [f"Scale: FETCH_SIZE x {fs:.4f}, WRITE_SIZE x {ws:.4f} (copy kernel, {copy_mib} MiB each way).", "",
           "| kernel | HBM read (MB) | HBM write (MB) | mean duration (us) | GB/s | % of 8 TB/s |",
           "|---|---:|---:|---:|---:|---:|"]
    for tot, k, rd, wr, us in sorted(rows, reverse=True):
        gbs = tot / (us * 1e-6) / 1e9
        out.append(f"| `{k}` | {rd / 1e6:.1f} | {wr / 1e6:.1f} | {us:.1f} | {gbs:.0f} | {100 * gbs / 8000:.1f} |")
    return "\n".join(out)


if __name__ == "__main__":
    if sys.argv[1] == "--sq":
        print(sq_markdown(sys.argv[2]))
    elif sys.argv[1] == "--hbm":
        print(hbm_markdown(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5])))
    else:
        print(markdown(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 30))
