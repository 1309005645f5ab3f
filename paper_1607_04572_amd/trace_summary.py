"""Per-kernel statistics of a rocprofv3 kernel trace (its SQLite results
database) as the markdown table of the profile summaries.

Usage: python -m paper_1607_04572_amd.trace_summary <run_results.db> [rows]
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


if __name__ == "__main__":
    print(markdown(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 30))
