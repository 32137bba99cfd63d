"""Per-kernel summary (calls, total, average, share) of a rocprofv3 rocpd database.

Usage: python -m paper_1601_07384_amd.rocpd_summary <results.db> [top_n]
"""
import sqlite3
import sys


def summarize(path, top=25):
    db = sqlite3.connect(path)
    rows = db.execute("select name, count(*), sum(duration), avg(duration), min(duration), "
                      "max(duration) from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows)
    out = [f"{'kernel':<70} {'calls':>7} {'total_ms':>10} {'avg_us':>10} {'min_us':>9} {'max_us':>9} {'share':>6}"]
    for name, n, tot, avg, mn, mx in rows[:top]:
        out.append(f"{name[:70]:<70} {n:>7} {tot / 1e6:>10.3f} {avg / 1e3:>10.2f} {mn / 1e3:>9.2f} "
                   f"{mx / 1e3:>9.2f} {100 * tot / total:>5.1f}%")
    out.append(f"{'all kernels':<70} {sum(r[1] for r in rows):>7} {total / 1e6:>10.3f}")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarize(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 25))
